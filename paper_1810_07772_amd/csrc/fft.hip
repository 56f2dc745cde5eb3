// Batched 1-D DFT passes for the two transforms of Sec. 4.1 (rows of P to g with exp(-i G.r),
// columns with exp(+i G'.r')), pruned to the G-sphere.
//
// A 3-D transform over a grid index is three passes, one per axis.  In every pass the
// batch axis (the other matrix index, contiguous in memory) runs across the lanes of a
// wave, so each lane owns one whole length-n transform along a strided axis, every load
// and store is coalesced, and no shuffles are needed.  Each pass keeps only the output
// frequencies that the sphere (or its projection onto the remaining axes) still needs,
// through an output-row map built on the host.
//
// The length-n DFT is done in registers as n = R1*R2 (two stages of naive DFTs with an
// inner twiddle).  Twiddle factors are compile-time constants: cos/sin of 2 pi m/n are
// evaluated by a constexpr Taylor series in double and rounded once to float, with the
// quarter-turn values exact, so the unrolled code carries them as literals.
#include "gw_internal.h"

namespace gwi {

// ---- constexpr trigonometry (Taylor series about 0 after reduction to [-pi/4, pi/4]) -----
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) { term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0)); sum += term; }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) { term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k)); sum += term; }
  return sum;
}
// cos and sin of 2 pi m / n using the octant of m/n: exact at multiples of a quarter turn.
constexpr double cos2pi(long m, long n) {
  m %= n; if (m < 0) m += n;
  // 8m/n selects the octant; reduce to an angle in [-pi/4, pi/4] about a multiple of pi/2.
  const long q = (4 * m + n / 2) / n;          // nearest quarter turn (0..4)
  const double r = 2.0 * kPi * ((double)m / (double)n - (double)q / 4.0);
  if (4 * m == q * n) {                        // exactly a quarter-turn multiple
    switch (q & 3) { case 0: return 1.0; case 1: return 0.0; case 2: return -1.0; default: return 0.0; }
  }
  switch (q & 3) {
    case 0: return taylor_cos(r);
    case 1: return -taylor_sin(r);
    case 2: return -taylor_cos(r);
    default: return taylor_sin(r);
  }
}
constexpr double sin2pi(long m, long n) {
  m %= n; if (m < 0) m += n;
  const long q = (4 * m + n / 2) / n;
  const double r = 2.0 * kPi * ((double)m / (double)n - (double)q / 4.0);
  if (4 * m == q * n) {
    switch (q & 3) { case 0: return 0.0; case 1: return 1.0; case 2: return 0.0; default: return -1.0; }
  }
  switch (q & 3) {
    case 0: return taylor_sin(r);
    case 1: return taylor_cos(r);
    case 2: return -taylor_sin(r);
    default: return -taylor_cos(r);
  }
}

template <int N>
struct Twiddle {
  float c[N];
  float s[N];
  constexpr Twiddle() : c(), s() {
    for (int m = 0; m < N; ++m) { c[m] = (float)cos2pi(m, N); s[m] = (float)sin2pi(m, N); }
  }
};

// acc += x * W^m with W^m = (c, sgn * s) a compile-time constant after unrolling.
template <int N, int SIGN>
__device__ __forceinline__ void cmac_tw(float2 &acc, float2 x, int m) {
  constexpr Twiddle<N> tw{};
  m %= N;
  const float c = tw.c[m];
  const float s = SIGN * tw.s[m];
  if (s == 0.0f) {
    if (c == 1.0f) { acc.x += x.x; acc.y += x.y; }
    else if (c == -1.0f) { acc.x -= x.x; acc.y -= x.y; }
    else { acc.x += c * x.x; acc.y += c * x.y; }
  } else if (c == 0.0f) {
    // (x.x + i x.y) * (i s) = -s x.y + i s x.x
    if (s == 1.0f) { acc.x -= x.y; acc.y += x.x; }
    else if (s == -1.0f) { acc.x += x.y; acc.y -= x.x; }
    else { acc.x -= s * x.y; acc.y += s * x.x; }
  } else {
    acc.x += c * x.x - s * x.y;
    acc.y += c * x.y + s * x.x;
  }
}

template <int N, int SIGN>
__device__ __forceinline__ float2 mul_tw(float2 x, int m) {
  float2 acc = make_float2(0.f, 0.f);
  cmac_tw<N, SIGN>(acc, x, m);
  return acc;
}

// ---- in-register mixed-radix FFT ----------------------------------------------------------------
// X[k] = sum_n x[n] W^{n k}, W = exp(SIGN 2 pi i / N), by recursive Cooley-Tukey: N = R M with the radix R
// taken from 4, 3, 2, 5 in that order of preference; n = M n1 + n2, k = k1 + R k2:
//   y[k1][n2] = W_N^{n2 k1} sum_{n1} x[M n1 + n2] W_R^{n1 k1},   X[k1 + R k2] = sum_{n2} y[k1][n2] W_M^{n2 k2}.
// The R-point DFTs are written-out butterflies (radix 4 and 2 need only additions, radix 3 one real
// multiplication pair), the twiddles are compile-time constants (trivial ones skipped by mul_tw), and
// the M-point DFTs recurse.
template <int N> struct Radix { static constexpr int R = (N % 4 == 0) ? 4 : (N % 3 == 0) ? 3 : (N % 2 == 0) ? 2 : N; };

template <int R, int SIGN> struct Butterfly;
template <int SIGN> struct Butterfly<2, SIGN> {
  static __device__ __forceinline__ void run(float2 (&v)[2]) {
    const float2 a = v[0], b = v[1];
    v[0] = make_float2(a.x + b.x, a.y + b.y);
    v[1] = make_float2(a.x - b.x, a.y - b.y);
  }
};
template <int SIGN> struct Butterfly<4, SIGN> {
  // X1 = (a - c) + SIGN i (b - d), X3 = (a - c) - SIGN i (b - d)
  static __device__ __forceinline__ void run(float2 (&v)[4]) {
    const float2 a = v[0], b = v[1], c = v[2], d = v[3];
    const float2 s0 = make_float2(a.x + c.x, a.y + c.y), d0 = make_float2(a.x - c.x, a.y - c.y);
    const float2 s1 = make_float2(b.x + d.x, b.y + d.y), d1 = make_float2(b.x - d.x, b.y - d.y);
    const float2 r = SIGN > 0 ? make_float2(-d1.y, d1.x) : make_float2(d1.y, -d1.x);   // SIGN i (b - d)
    v[0] = make_float2(s0.x + s1.x, s0.y + s1.y);
    v[2] = make_float2(s0.x - s1.x, s0.y - s1.y);
    v[1] = make_float2(d0.x + r.x, d0.y + r.y);
    v[3] = make_float2(d0.x - r.x, d0.y - r.y);
  }
};
template <int SIGN> struct Butterfly<3, SIGN> {
  // X1,2 = a - (b + c)/2 +- SIGN i (sqrt(3)/2) (b - c)
  static __device__ __forceinline__ void run(float2 (&v)[3]) {
    constexpr float h = 0.866025403784438646763723170752936f;   // sqrt(3)/2
    const float2 a = v[0], b = v[1], c = v[2];
    const float2 t = make_float2(b.x + c.x, b.y + c.y), d = make_float2(b.x - c.x, b.y - c.y);
    const float2 m = make_float2(a.x - 0.5f * t.x, a.y - 0.5f * t.y);
    const float2 r = SIGN > 0 ? make_float2(-h * d.y, h * d.x) : make_float2(h * d.y, -h * d.x);
    v[0] = make_float2(a.x + t.x, a.y + t.y);
    v[1] = make_float2(m.x + r.x, m.y + r.y);
    v[2] = make_float2(m.x - r.x, m.y - r.y);
  }
};
template <int R, int SIGN> struct Butterfly {   // any other radix (5): the plain DFT with constant twiddles
  static __device__ __forceinline__ void run(float2 (&v)[R]) {
    float2 o[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int n = 0; n < R; ++n) cmac_tw<R, SIGN>(acc, v[n], n * k % R);
      o[k] = acc;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = o[k];
  }
};

template <int N, int SIGN> struct Fft {
  static __device__ __forceinline__ void run(float2 (&x)[N]) {
    constexpr int R = Radix<N>::R, M = N / R;
    if constexpr (M == 1) {
      Butterfly<N, SIGN>::run(x);
    } else {
      float2 y[R][M];
#pragma unroll
      for (int n2 = 0; n2 < M; ++n2) {
        float2 v[R];
#pragma unroll
        for (int n1 = 0; n1 < R; ++n1) v[n1] = x[M * n1 + n2];
        Butterfly<R, SIGN>::run(v);
#pragma unroll
        for (int k1 = 0; k1 < R; ++k1) y[k1][n2] = (n2 * k1 == 0) ? v[k1] : mul_tw<N, SIGN>(v[k1], n2 * k1);
      }
#pragma unroll
      for (int k1 = 0; k1 < R; ++k1) {
        Fft<M, SIGN>::run(y[k1]);
#pragma unroll
        for (int k2 = 0; k2 < M; ++k2) x[k1 + R * k2] = y[k1][k2];
      }
    }
  }
};

// In-register DFT X = DFT_N(x) (sign SIGN), by the mixed-radix FFT above.
template <int N, int SIGN>
__device__ __forceinline__ void dft_regs(const float2 (&x)[N], float2 (&X)[N]) {
#pragma unroll
  for (int n = 0; n < N; ++n) X[n] = x[n];
  Fft<N, SIGN>::run(X);
}

// The same FFT with its inputs read through ld(n) one first-stage group at a time: the R inputs
// x[M n1 + n2] of one n2 are loaded, combined and twiddled before the next group's loads (a scheduling
// barrier keeps the compiler from issuing every load at once), so at most R inputs and the N partial
// results are live.
template <int N, int SIGN, typename Load>
__device__ __forceinline__ void dft_regs_load(Load ld, float2 (&X)[N]) {
  constexpr int R = Radix<N>::R, M = N / R;
  if constexpr (M == 1) {
#pragma unroll
    for (int n = 0; n < N; ++n) X[n] = ld(n);
    Butterfly<N, SIGN>::run(X);
  } else {
    float2 y[R][M];
#pragma unroll
    for (int n2 = 0; n2 < M; ++n2) {
      float2 v[R];
#pragma unroll
      for (int n1 = 0; n1 < R; ++n1) v[n1] = ld(M * n1 + n2);
      Butterfly<R, SIGN>::run(v);
#pragma unroll
      for (int k1 = 0; k1 < R; ++k1) y[k1][n2] = (n2 * k1 == 0) ? v[k1] : mul_tw<N, SIGN>(v[k1], n2 * k1);
      if (n2 + 1 < M) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) {
      Fft<M, SIGN>::run(y[k1]);
#pragma unroll
      for (int k2 = 0; k2 < M; ++k2) X[k1 + R * k2] = y[k1][k2];
    }
  }
}

constexpr int FFT_THREADS = 256;

// grid.x: batch blocks of 256, grid.y: flattened (o, u).
template <int N, int SIGN>
__global__ __launch_bounds__(FFT_THREADS) void fft_pass_kernel(const float2 *__restrict__ in,
                                                                float2 *__restrict__ out, int U, int B,
                                                                long long ld_in, long long ld_out,
                                                                const int *__restrict__ map) {
  const int b = blockIdx.x * FFT_THREADS + threadIdx.x;
  if (b >= B) return;
  const int ou = blockIdx.y;
  const int o = ou / U, u = ou - o * U;
  const int *mrow = map + (size_t)ou * N;
  float2 x[N], X[N];
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = in[((long long)(o * N + i) * U + u) * ld_in + b];
  dft_regs<N, SIGN>(x, X);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int row = mrow[k];
    if (row >= 0) out[(long long)row * ld_out + b] = X[k];
  }
}

// The adjoint of the pass above: input rows are gathered through a map (-1 reads zero), the N
// outputs go to rows (o*N + k)*U + u.  With the sphere plan's maps this runs a transform from
// the sphere to the full grid (plane-wave coefficients to orbitals), axis by axis in reverse.
template <int N, int SIGN>
__global__ __launch_bounds__(FFT_THREADS) void fft_gather_pass_kernel(const float2 *__restrict__ in,
                                                                       float2 *__restrict__ out, int U, int B,
                                                                       long long ld_in, long long ld_out,
                                                                       const int *__restrict__ map, float scale) {
  const int b = blockIdx.x * FFT_THREADS + threadIdx.x;
  if (b >= B) return;
  const int ou = blockIdx.y;
  const int o = ou / U, u = ou - o * U;
  const int *mrow = map + (size_t)ou * N;
  float2 x[N], X[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int row = mrow[i];
    float2 v = make_float2(0.f, 0.f);
    if (row >= 0) {
      v = in[(long long)row * ld_in + b];
      v.x *= scale;
      v.y *= scale;
    }
    x[i] = v;
  }
  dft_regs<N, SIGN>(x, X);
#pragma unroll
  for (int k = 0; k < N; ++k) out[((long long)(o * N + k) * U + u) * ld_out + b] = X[k];
}

// The gather pass along the last axis (U = 1) with its output transposed on the way: 64 batch columns
// (bands) and 4 consecutive lines per workgroup; each thread transforms one line into an LDS tile, and
// the workgroup then writes each band's 4 N consecutive outputs to its own row, out[b][o N + k].  This
// replaces a [grid][band] intermediate and a separate transpose of it.  Each wave holds one line, so
// its map row is read through the scalar cache; grid.x runs over line groups, so the workgroups in
// flight write a few bands' rows at a time rather than a short run of every band's row.
constexpr int GT_BANDS = 64, GT_LINES = FFT_THREADS / GT_BANDS;
template <int N, int SIGN>
__global__ __launch_bounds__(FFT_THREADS) void fft_gather_pass_t_kernel(const float2 *__restrict__ in,
                                                                         float2 *__restrict__ out, int O, int B,
                                                                         long long ld_in, long long ld_out,
                                                                         const int *__restrict__ map, float scale) {
  __shared__ float2 tile[GT_LINES * N][GT_BANDS + 1];
  static_assert(GT_BANDS == 64, "one line per wave");
  const int tb = threadIdx.x % GT_BANDS, l = __builtin_amdgcn_readfirstlane(threadIdx.x / GT_BANDS);
  const int o0 = blockIdx.x * GT_LINES, o = o0 + l;
  const int b0 = blockIdx.y * GT_BANDS, b = b0 + tb;
  if (o < O) {
    const int *mrow = map + (size_t)o * N;
    float2 x[N], X[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int row = mrow[i];
      float2 v = make_float2(0.f, 0.f);
      if (row >= 0 && b < B) {
        v = in[(long long)row * ld_in + b];
        v.x *= scale;
        v.y *= scale;
      }
      x[i] = v;
    }
    dft_regs<N, SIGN>(x, X);
#pragma unroll
    for (int k = 0; k < N; ++k) tile[l * N + k][tb] = X[k];
  }
  __syncthreads();
  const int nl = min(GT_LINES, O - o0), nb = min(GT_BANDS, B - b0);
  float2 *ob = out + (long long)b0 * ld_out + (long long)o0 * N;
  if (nl == GT_LINES && nb == GT_BANDS) {
    // full block: GT_LINES * N consecutive outputs per band, N stores per thread
    constexpr int RUN = GT_LINES * N;
#pragma unroll 4
    for (int it = 0; it < GT_BANDS * RUN / FFT_THREADS; ++it) {
      const int v = (int)threadIdx.x + it * FFT_THREADS, band = v / RUN, kk = v - band * RUN;
      ob[(long long)band * ld_out + kk] = tile[kk][band];
    }
  } else {
    const int run = nl * N;                     // consecutive outputs per band in this block
    for (int v = threadIdx.x; v < nb * run; v += FFT_THREADS) {
      const int band = v / run, kk = v - band * run;
      ob[(long long)band * ld_out + kk] = tile[kk][band];
    }
  }
}

#define GW_FFT_SIZES(X) X(4) X(5) X(6) X(8) X(9) X(10) X(12) X(15) X(16) X(18) X(20) X(24) X(27) X(30) X(32) X(36) X(40) X(48)

bool fft_size_supported(int n) {
  switch (n) {
#define GW_CASE(n_) case n_:
    GW_FFT_SIZES(GW_CASE)
#undef GW_CASE
    return true;
    default: return false;
  }
}

hipError_t launch_fft_pass(int n, int sign, const float2 *in, float2 *out, int O, int U, int B, long long ld_in,
                           long long ld_out, const int *map, hipStream_t s) {
  if (O * U > 65535 * 1024) return hipErrorInvalidValue;
  dim3 grid((B + FFT_THREADS - 1) / FFT_THREADS, O * U), block(FFT_THREADS);
  if (grid.y > 65535) return hipErrorInvalidValue;
  switch (n) {
#define GW_CASE(n_)                                                                                          \
  case n_:                                                                                                   \
    if (sign < 0)                                                                                            \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(fft_pass_kernel<n_, -1>), grid, block, 0, s, in, out, U, B, ld_in, \
                         ld_out, map);                                                                       \
    else                                                                                                     \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(fft_pass_kernel<n_, 1>), grid, block, 0, s, in, out, U, B, ld_in,  \
                         ld_out, map);                                                                       \
    break;
    GW_FFT_SIZES(GW_CASE)
#undef GW_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fft_gather_pass(int n, int sign, const float2 *in, float2 *out, int O, int U, int B, long long ld_in,
                                  long long ld_out, const int *map, float scale, hipStream_t s) {
  dim3 grid((B + FFT_THREADS - 1) / FFT_THREADS, O * U), block(FFT_THREADS);
  if ((long long)O * U > 65535) return hipErrorInvalidValue;
  switch (n) {
#define GW_CASE(n_)                                                                                            \
  case n_:                                                                                                     \
    if (sign < 0)                                                                                              \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(fft_gather_pass_kernel<n_, -1>), grid, block, 0, s, in, out, U, B,   \
                         ld_in, ld_out, map, scale);                                                           \
    else                                                                                                       \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(fft_gather_pass_kernel<n_, 1>), grid, block, 0, s, in, out, U, B,    \
                         ld_in, ld_out, map, scale);                                                           \
    break;
    GW_FFT_SIZES(GW_CASE)
#undef GW_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fft_gather_pass_t(int n, int sign, const float2 *in, float2 *out, int O, int B, long long ld_in,
                                    long long ld_out, const int *map, float scale, hipStream_t s) {
  dim3 grid((O + GT_LINES - 1) / GT_LINES, (B + GT_BANDS - 1) / GT_BANDS), block(FFT_THREADS);
  if (grid.y > 65535) return hipErrorInvalidValue;
  switch (n) {
#define GW_CASE(n_)                                                                                             \
  case n_:                                                                                                      \
    if (sign < 0)                                                                                               \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(fft_gather_pass_t_kernel<n_, -1>), grid, block, 0, s, in, out, O, B,  \
                         ld_in, ld_out, map, scale);                                                            \
    else                                                                                                        \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(fft_gather_pass_t_kernel<n_, 1>), grid, block, 0, s, in, out, O, B,   \
                         ld_in, ld_out, map, scale);                                                            \
    break;
    GW_FFT_SIZES(GW_CASE)
#undef GW_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---- the row-contiguous form of the two transforms ---------------------------------------------
// With M a matrix whose rows are transformed along their contiguous index,
//   Y[r][g'] = sum_r' M(r, r') exp(+i G_g'.r'),   r' = (i1 n2 + i2) n3 + i3,
// every 3-D transform reads one contiguous row.  The i1 plane of a row (n2 x n3 consecutive values) is
// transformed over i3 and i2 by one wave (plane_ab_kernel), keeping only the (k2, k3) pairs of the
// sphere; plane_c_kernel then transforms over i1 and writes the sphere vectors in their order.  For a
// Hermitian P (P = M + M^H with M its upper triangle and half its real diagonal), only the upper
// triangle is read (HERM): planes wholly left of the diagonal are skipped and read as zero.

// One wave (one workgroup) per row r and pl consecutive i1 planes of it.  Phase 1: item t < pl n3 is
// column i3 = t % n3 of plane t / n3; its lane loads the column (n2 loads, each wave instruction reading
// runs of 8 n3 contiguous bytes), transforms it over i2 in registers and keeps the rows k2 that occur in
// sphere pairs (slot k2s[k2] >= 0) in LDS [plane][slot][i3] (row stride n3 + 1 against bank conflicts).
// Phase 2: item t < pl nk2 (one round: pl nk2 <= 64) is row slot t % nk2 of plane t / nk2; its lane
// loads the row, transforms it over i3 and writes the outputs whose (k2, k3) is a sphere pair to LDS
// [plane][pair], over the rows every lane has read.  The planes of one block are consecutive in y1, so
// the block's output leaves in one contiguous run.  pl is chosen on the host to keep the lanes busy:
// at n = 36 with 19 rows k2, three planes fill 108 of 128 lanes in phase 1 and 57 of 64 in phase 2.
template <int N, bool HERM>
__global__ __launch_bounds__(64) void plane_ab_kernel(const float2 *__restrict__ P, long long ldp, int n1, int pl,
                                                      const int *__restrict__ k2s, int nk2,
                                                      const int *__restrict__ mapab, int npair,
                                                      float2 *__restrict__ y1) {
  constexpr int PLN = N * N, LD = N + 1;
  extern __shared__ float2 lds[];                 // [pl][nk2][LD], then [pl][npair] over it
  const int lane = threadIdx.x;
  const int r = blockIdx.x, i10 = blockIdx.y * pl;
  const int roff = r - i10 * PLN;                 // the diagonal's offset in the first plane of the block
  const int pfirst = (HERM && roff >= 0) ? min(roff / PLN, pl) : 0;   // planes left of it hold no work
  const int pend = min(pl, n1 - i10);
  if (pfirst >= pend) return;
  const int reg = nk2 * LD;
  const bool diag = HERM && roff >= 0 && roff < pl * PLN;   // the diagonal lies in one of the block's planes
  const float2 *src = P + (long long)r * ldp + (long long)i10 * PLN;
  for (int t0 = 0; t0 < pl * N; t0 += 64) {
    const int t = t0 + lane, p = t / N, i3 = t - p * N;
    if (p >= pfirst && p < pend) {
      const float2 *pln = src + (long long)p * PLN;
      const int eo = roff - p * PLN;              // element offset of the diagonal in plane p
      float2 x[N];
      if (HERM && diag) {
        // Lanes left of the diagonal load the diagonal element (finite) and scale it by 0: the value is
        // used on every path, so each load stays unconditional and all of them are in flight at once.
#pragma unroll
        for (int i2 = 0; i2 < N; ++i2) {
          const int e = i2 * N + i3;
          const bool lo = e < eo, dg = e == eo;
          float2 v = pln[lo ? eo : e];
          v.x *= lo ? 0.f : dg ? 0.5f : 1.f;      // M carries half the (real) diagonal
          v.y *= (lo || dg) ? 0.f : 1.f;
          x[i2] = v;
        }
      } else {
#pragma unroll
        for (int i2 = 0; i2 < N; ++i2) x[i2] = pln[i2 * N + i3];
      }
      __builtin_amdgcn_sched_barrier(0);          // every load of the column in flight before the first use
      Fft<N, 1>::run(x);
      float2 *L = lds + p * reg + i3;
#pragma unroll
      for (int k2 = 0; k2 < N; ++k2) {
        const int sl = k2s[k2];
        if (sl >= 0) L[sl * LD] = x[k2];
      }
    }
  }
  __syncthreads();
  const int p = lane / nk2, sl = lane - p * nk2;
  const bool act = p >= pfirst && p < pend;
  float2 x[N];
  if (act) {
    const float2 *row = lds + p * reg + sl * LD;
#pragma unroll
    for (int i3 = 0; i3 < N; ++i3) x[i3] = row[i3];
  }
  __syncthreads();                                // every row is in registers: the region is free
  if (act) {
    Fft<N, 1>::run(x);
    const int *mrow = mapab + sl * N;
    float2 *out = lds + p * npair;
#pragma unroll
    for (int k3 = 0; k3 < N; ++k3) {
      const int pid = mrow[k3];
      if (pid >= 0) out[pid] = x[k3];
    }
  }
  __syncthreads();
  float2 *dst = y1 + ((long long)r * n1 + i10) * npair;
  for (int j = pfirst * npair + lane; j < pend * npair; j += 64) dst[j] = lds[j];
}

// Planes per wave: the fewest wave rounds per plane over both phases, phase 2 in one round.
static int plane_ab_planes(int n, int nk2, int n1) {
  int best = 1;
  double cost = 1e30;
  for (int pl = 1; pl <= 8 && pl <= n1 && pl * nk2 <= 64; ++pl) {
    const double c = double((pl * n + 63) / 64 + 1) / pl;
    if (c < cost - 1e-9) cost = c, best = pl;
  }
  return best;
}

// One workgroup per row r: the i1 transform of every pair (lanes over pairs, loads contiguous across
// lanes), each output k1 sent to its sphere vector through mapct [N1][npair] (-1: not on the sphere).
// The row's ng outputs are staged in LDS and written contiguously when they fit (STAGE), else directly.
constexpr int PLANE_C_STAGE = 8191;   // sphere vectors staged in LDS (with the spare slot, 64 KB)
template <int N1, bool HERM, bool STAGE>
__global__ __launch_bounds__(512) void plane_c_kernel(const float2 *__restrict__ y1, int plane, int npair,
                                                      const int *__restrict__ mapct, int ng,
                                                      float2 *__restrict__ y, long long ldy) {
  extern __shared__ float2 so[];                  // [ng + 1]: the sphere row, then a slot for unmapped outputs
  const int r = blockIdx.x;
  const int i1s = HERM ? r / plane : 0;          // planes left of the diagonal are zero
  const float2 *src = y1 + (long long)r * N1 * npair;
  float2 *yr = y + (long long)r * ldy;
  constexpr int C = 6;                            // map reads per group
#pragma unroll 1
  for (int p = threadIdx.x; p < npair; p += blockDim.x) {
    float2 X[N1];
    const float2 *sp = src + p;
    dft_regs_load<N1, 1>([&](int i1) { return i1 >= i1s ? sp[(long long)i1 * npair] : make_float2(0.f, 0.f); }, X);
    // The sphere index of each output comes from the map in groups of C reads, the next group in flight
    // while the current one is stored: every read is waited for once per group, not once per output,
    // and only 2 C map values are live at a time.
    const int *mp = mapct + p;
    int g[C], gn[C];
#pragma unroll
    for (int j = 0; j < C; ++j) g[j] = j < N1 ? mp[j * npair] : -1;
#pragma unroll
    for (int kc = 0; kc < N1; kc += C) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < C; ++j) gn[j] = kc + C + j < N1 ? mp[(kc + C + j) * npair] : -1;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        if (kc + j < N1) {
          if (STAGE) so[g[j] >= 0 ? g[j] : ng] = X[kc + j];
          else if (g[j] >= 0) yr[g[j]] = X[kc + j];
        }
      }
#pragma unroll
      for (int j = 0; j < C; ++j) g[j] = gn[j];
    }
  }
  if (STAGE) {
    __syncthreads();
    for (int g = threadIdx.x; g < ng; g += blockDim.x) yr[g] = so[g];
  }
}

// out = x + x^H for an [n][n] matrix (32 x 32 tiles, the transposed partner through LDS).
__global__ __launch_bounds__(256) void add_adjoint_kernel(const float2 *__restrict__ x, int n, float2 *__restrict__ out) {
  __shared__ float2 t[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = 0; k < 32; k += 8) {
    const int r = c0 + ty + k, c = r0 + tx;
    if (r < n && c < n) t[ty + k][tx] = x[(size_t)r * n + c];
  }
  __syncthreads();
  for (int k = 0; k < 32; k += 8) {
    const int g = r0 + ty + k, gp = c0 + tx;
    if (g < n && gp < n) {
      const float2 a = x[(size_t)g * n + gp], b = t[tx][ty + k];
      out[(size_t)g * n + gp] = make_float2(a.x + b.x, a.y - b.y);
    }
  }
}

bool plane_path_supported(int n2, int n3) { return n2 == n3 && n3 <= 64 && fft_size_supported(n3); }

hipError_t launch_plane_ab(int n, bool herm, const float2 *p, long long ldp, int nr, int n1, const int *k2s, int nk2,
                           const int *mapab, int npair, float2 *y1, hipStream_t s) {
  if (nk2 < 1 || nk2 > n || nk2 > 64 || npair > nk2 * n) return hipErrorInvalidValue;
  const int pl = plane_ab_planes(n, nk2, n1);
  dim3 grid(nr, (n1 + pl - 1) / pl), block(64);
  const size_t shm = (size_t)pl * nk2 * (n + 1) * sizeof(float2);
  if (grid.y > 65535 || shm > 64 * 1024) return hipErrorInvalidValue;
  switch (n) {
#define GW_CASE(n_)                                                                                                  \
  case n_:                                                                                                           \
    if (herm)                                                                                                        \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(plane_ab_kernel<n_, true>), grid, block, shm, s, p, ldp, n1, pl, k2s, nk2,   \
                         mapab, npair, y1);                                                                          \
    else                                                                                                             \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(plane_ab_kernel<n_, false>), grid, block, shm, s, p, ldp, n1, pl, k2s, nk2,  \
                         mapab, npair, y1);                                                                          \
    break;
    GW_FFT_SIZES(GW_CASE)
#undef GW_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_plane_c(int n1, bool herm, const float2 *y1, int nr, int plane, int npair, const int *mapct, int ng,
                          float2 *y, long long ldy, hipStream_t s) {
  const bool stage = ng <= PLANE_C_STAGE;
  const size_t shm = stage ? (size_t)(ng + 1) * sizeof(float2) : 0;
  // one thread per pair where that fits in 512 threads: a block of whole waves covering npair
  dim3 grid(nr), block(std::min(512, std::max(64, (npair + 63) / 64 * 64)));
  switch (n1) {
#define GW_CASE(n_)                                                                                              \
  case n_:                                                                                                       \
    if (herm && stage)                                                                                           \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(plane_c_kernel<n_, true, true>), grid, block, shm, s, y1, plane, npair,  \
                         mapct, ng, y, ldy);                                                                     \
    else if (herm)                                                                                               \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(plane_c_kernel<n_, true, false>), grid, block, 0, s, y1, plane, npair,   \
                         mapct, ng, y, ldy);                                                                     \
    else if (stage)                                                                                              \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(plane_c_kernel<n_, false, true>), grid, block, shm, s, y1, plane, npair, \
                         mapct, ng, y, ldy);                                                                     \
    else                                                                                                         \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(plane_c_kernel<n_, false, false>), grid, block, 0, s, y1, plane, npair,  \
                         mapct, ng, y, ldy);                                                                     \
    break;
    GW_FFT_SIZES(GW_CASE)
#undef GW_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---- orbitals from plane-wave coefficients, row-contiguous (the sphere transform's plane path run in
// reverse, band-major throughout) ------------------------------------------------------------------------
// psi_b(r) = N_r^-1/2 sum_m c_bm exp(+i G_m.r) in two steps.  orb_c: thread (band b, pair p) gathers the
// pair's k1 column from the band's coefficients (mapct, -1 off the sphere), scaled, and transforms it over
// k1: y[b][i1][p].  orb_plane: one wave per band and pl consecutive i1 planes stages those planes' pair
// values in LDS, transforms each row k2 that carries pairs over k3 (one lane per row), then every column i3
// over k2 (one lane per column, zero where k2 has no pair), and stores the planes of psi_b contiguously.
template <int N1>
__global__ __launch_bounds__(256) void orb_c_kernel(const float2 *__restrict__ coeff, int npw, int nb,
                                                    const int *__restrict__ mapct, int npair, float scale,
                                                    float2 *__restrict__ y) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long long)nb * npair) return;
  const int b = (int)(idx / npair), p = (int)(idx - (long long)b * npair);
  const float2 *cb = coeff + (size_t)b * npw;
  float2 x[N1];
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) {
    // every load unconditional (a valid index, scaled by zero off the sphere), so all are in flight at once
    const int g = mapct[k1 * npair + p];
    const float m = g >= 0 ? scale : 0.f;
    const float2 v = cb[g >= 0 ? g : 0];
    x[k1] = make_float2(v.x * m, v.y * m);
  }
  __builtin_amdgcn_sched_barrier(0);
  Fft<N1, 1>::run(x);
  float2 *yb = y + (size_t)b * N1 * npair + p;
#pragma unroll
  for (int i1 = 0; i1 < N1; ++i1) yb[(size_t)i1 * npair] = x[i1];
}

template <int N>
__global__ __launch_bounds__(128) void orb_plane_kernel(const float2 *__restrict__ y, int n1, int pl,
                                                        const int *__restrict__ k2s, int nk2,
                                                        const int *__restrict__ mapab, int npair,
                                                        float2 *__restrict__ psi, long long ldpsi) {
  // two waves: wave 0 transforms the rows (pl nk2 <= 64), both transform the columns (pl n <= 128 at n = 36)
  constexpr int PLN = N * N, LD = N + 1;
  extern __shared__ float2 lds[];                 // [pl][npair] pair values, then [pl][nk2][LD] rows over them
  const int tid = threadIdx.x;
  const int b = blockIdx.x, i10 = blockIdx.y * pl;
  const int pend = min(pl, n1 - i10);
  const float2 *src = y + ((size_t)b * n1 + i10) * npair;
  for (int j = tid; j < pend * npair; j += 128) lds[j] = src[j];
  __syncthreads();
  {
    const int p = tid / nk2, sl = tid - p * nk2;
    const bool act = tid < 64 && p < pend;         // wave 0 alone: its reads are issued before its writes
    float2 x[N];
    if (act) {
      const int *mrow = mapab + sl * N;
      const float2 *yp = lds + p * npair;
#pragma unroll
      for (int k3 = 0; k3 < N; ++k3) {
        const int pid = mrow[k3];
        x[k3] = pid >= 0 ? yp[pid] : make_float2(0.f, 0.f);
      }
    }
    __syncthreads();                               // every pair value read: the rows may overwrite them
    if (act) {
      Fft<N, 1>::run(x);
      float2 *row = lds + (p * nk2 + sl) * LD;
#pragma unroll
      for (int i3 = 0; i3 < N; ++i3) row[i3] = x[i3];
    }
  }
  __syncthreads();
  for (int t0 = 0; t0 < pl * N; t0 += 128) {
    const int t = t0 + tid, p = t / N, i3 = t - p * N;
    if (p < pend) {
      const float2 *col = lds + p * nk2 * LD + i3;
      float2 x[N];
#pragma unroll
      for (int k2 = 0; k2 < N; ++k2) {
        const int sl = k2s[k2];                        // uniform
        x[k2] = sl >= 0 ? col[sl * LD] : make_float2(0.f, 0.f);
      }
      Fft<N, 1>::run(x);
      float2 *dst = psi + (size_t)b * ldpsi + (size_t)(i10 + p) * PLN + i3;
#pragma unroll
      for (int i2 = 0; i2 < N; ++i2) dst[i2 * N] = x[i2];
    }
  }
}

hipError_t launch_orb_c(int n1, const float2 *coeff, int npw, int nb, const int *mapct, int npair, float scale,
                        float2 *y, hipStream_t s) {
  const long long nt = (long long)nb * npair;
  if (nt <= 0) return hipSuccess;
  if ((nt + 255) / 256 > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((nt + 255) / 256)), block(256);
  switch (n1) {
#define GW_CASE(n_)                                                                                                 \
  case n_:                                                                                                          \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(orb_c_kernel<n_>), grid, block, 0, s, coeff, npw, nb, mapct, npair, scale, y); \
    break;
    GW_FFT_SIZES(GW_CASE)
#undef GW_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_orb_plane(int n, const float2 *y, int nb, int n1, const int *k2s, int nk2, const int *mapab,
                            int npair, float2 *psi, long long ldpsi, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  if (nk2 < 1 || nk2 > n || nk2 > 64 || npair > nk2 * n) return hipErrorInvalidValue;
  const int pl = plane_ab_planes(n, nk2, n1);
  const dim3 grid(nb, (n1 + pl - 1) / pl), block(128);
  const size_t shm = (size_t)pl * std::max(npair, nk2 * (n + 1)) * sizeof(float2);
  if (grid.y > 65535 || shm > 64 * 1024) return hipErrorInvalidValue;
  switch (n) {
#define GW_CASE(n_)                                                                                                  \
  case n_:                                                                                                           \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(orb_plane_kernel<n_>), grid, block, shm, s, y, n1, pl, k2s, nk2, mapab, npair, \
                       psi, ldpsi);                                                                                  \
    break;
    GW_FFT_SIZES(GW_CASE)
#undef GW_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_add_adjoint(const float2 *x, int n, float2 *out, hipStream_t s) {
  dim3 grid((n + 31) / 32, (n + 31) / 32);
  if (grid.y > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(add_adjoint_kernel, grid, dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

// ---- complex64 transpose through LDS: out[c][r] = in[r][c] ----------------------------------
constexpr int TT = 64;
__global__ __launch_bounds__(256) void transpose_c64_kernel(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                            int rows, int cols, long long ld_in, long long ld_out) {
  __shared__ float2 t[TT][TT + 1];
  const int r0 = blockIdx.y * TT, c0 = blockIdx.x * TT;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < TT; k += 4) {
    const int r = r0 + ty + k, c = c0 + tx;
    if (r < rows && c < cols) t[ty + k][tx] = in[(long long)r * ld_in + c];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < TT; k += 4) {
    const int c = c0 + ty + k, r = r0 + tx;
    if (r < rows && c < cols) out[(long long)c * ld_out + r] = t[tx][ty + k];
  }
}

hipError_t launch_transpose_c64(const float2 *in, float2 *out, int rows, int cols, long long ld_in, long long ld_out,
                                hipStream_t s) {
  dim3 grid((cols + TT - 1) / TT, (rows + TT - 1) / TT);
  if (grid.y > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(transpose_c64_kernel, grid, dim3(256), 0, s, in, out, rows, cols, ld_in, ld_out);
  return hipGetLastError();
}

}  // namespace gwi
