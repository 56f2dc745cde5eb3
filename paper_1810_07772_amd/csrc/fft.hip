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

// factor choice R1 * R2 = N with both factors small
template <int N> struct Factor { static constexpr int R1 = N, R2 = 1; };
template <> struct Factor<4> { static constexpr int R1 = 2, R2 = 2; };
template <> struct Factor<6> { static constexpr int R1 = 2, R2 = 3; };
template <> struct Factor<8> { static constexpr int R1 = 2, R2 = 4; };
template <> struct Factor<9> { static constexpr int R1 = 3, R2 = 3; };
template <> struct Factor<10> { static constexpr int R1 = 2, R2 = 5; };
template <> struct Factor<12> { static constexpr int R1 = 3, R2 = 4; };
template <> struct Factor<15> { static constexpr int R1 = 3, R2 = 5; };
template <> struct Factor<16> { static constexpr int R1 = 4, R2 = 4; };
template <> struct Factor<18> { static constexpr int R1 = 3, R2 = 6; };
template <> struct Factor<20> { static constexpr int R1 = 4, R2 = 5; };
template <> struct Factor<24> { static constexpr int R1 = 4, R2 = 6; };
template <> struct Factor<27> { static constexpr int R1 = 3, R2 = 9; };
template <> struct Factor<30> { static constexpr int R1 = 5, R2 = 6; };
template <> struct Factor<32> { static constexpr int R1 = 4, R2 = 8; };
template <> struct Factor<36> { static constexpr int R1 = 6, R2 = 6; };
template <> struct Factor<40> { static constexpr int R1 = 5, R2 = 8; };
template <> struct Factor<48> { static constexpr int R1 = 6, R2 = 8; };

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

// In-register DFT X[k] = sum_n x[n] exp(SIGN * 2 pi i n k / N), n = R2*n1 + n2, k = k1 + R1*k2.
template <int N, int SIGN>
__device__ __forceinline__ void dft_regs(const float2 (&x)[N], float2 (&X)[N]) {
  constexpr int R1 = Factor<N>::R1, R2 = Factor<N>::R2;
  float2 y[R1][R2];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2)
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) cmac_tw<N, SIGN>(acc, x[R2 * n1 + n2], (n1 * k1 % R1) * R2);
      y[k1][n2] = (n2 * k1 == 0) ? acc : mul_tw<N, SIGN>(acc, n2 * k1);
    }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) cmac_tw<N, SIGN>(acc, y[k1][n2], (n2 * k2 % R2) * R1);
      X[k1 + R1 * k2] = acc;
    }
}

// The same DFT with its inputs read through ld(n) one first-stage group at a time: the R1 inputs
// x[R2 n1 + n2] of one n2 are loaded, combined and dropped before the next group's loads, so at most
// R1 inputs and the N partial results are live (the plain form keeps all N inputs as well).
template <int N, int SIGN, typename Load>
__device__ __forceinline__ void dft_regs_load(Load ld, float2 (&X)[N]) {
  constexpr int R1 = Factor<N>::R1, R2 = Factor<N>::R2;
  float2 y[R1][R2];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
    float2 xs[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) xs[n1] = ld(R2 * n1 + n2);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) cmac_tw<N, SIGN>(acc, xs[n1], (n1 * k1 % R1) * R2);
      y[k1][n2] = (n2 * k1 == 0) ? acc : mul_tw<N, SIGN>(acc, n2 * k1);
    }
    if (n2 + 1 < R2) __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) cmac_tw<N, SIGN>(acc, y[k1][n2], (n2 * k2 % R2) * R1);
      X[k1 + R1 * k2] = acc;
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

// One wave per (row r, plane i1); four waves per workgroup.  Lane i3 (< N) loads the plane's column i3
// (N consecutive loads of N consecutive values: each load instruction reads 8 N contiguous bytes),
// transforms it over i2 in registers, and leaves its N outputs k2 in the wave's LDS block [k2][i3].
// Lane s (< nk2) then takes the row k2 = k2list[s], transforms it over i3 in registers, and stores the
// outputs whose (k2, k3) is a sphere pair at that pair's slot; the wave finally writes the npair slots
// to y1[r][i1][.] with contiguous stores.  One wave reads and writes its own LDS block only, in program
// order, so no workgroup barrier is needed.
template <int N, bool HERM>
__global__ __launch_bounds__(256) void plane_ab_kernel(const float2 *__restrict__ P, long long ldp, int nr, int n1,
                                                       const int *__restrict__ k2list, int nk2,
                                                       const int *__restrict__ mapab, int npair,
                                                       float2 *__restrict__ y1) {
  __shared__ float2 lds[4][N * N];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + w, i1 = blockIdx.y;
  constexpr int PL = N * N;
  if (r >= nr) return;
  const long long c0 = (long long)i1 * PL;
  if (HERM && c0 + PL <= r) return;              // left of the diagonal: zero, never read downstream
  float2 *L = lds[w];
  if (lane < N) {
    const float2 *src = P + (long long)r * ldp + c0 + lane;
    float2 x[N], X[N];
#pragma unroll
    for (int i2 = 0; i2 < N; ++i2) {
      float2 v = src[i2 * N];
      if (HERM) {
        const long long c = c0 + i2 * N + lane;
        if (c < r) v = make_float2(0.f, 0.f);
        else if (c == r) v = make_float2(0.5f * v.x, 0.f);     // M carries half the (real) diagonal
      }
      x[i2] = v;
    }
    dft_regs<N, 1>(x, X);
#pragma unroll
    for (int k2 = 0; k2 < N; ++k2) L[k2 * N + lane] = X[k2];
  }
  if (lane < nk2) {
    const int k2 = k2list[lane];
    float2 x[N], X[N];
#pragma unroll
    for (int i3 = 0; i3 < N; ++i3) x[i3] = L[k2 * N + i3];
    dft_regs<N, 1>(x, X);
    const int *mrow = mapab + lane * N;
#pragma unroll
    for (int k3 = 0; k3 < N; ++k3) {
      const int pid = mrow[k3];
      if (pid >= 0) L[pid] = X[k3];                           // after every lane's reads (program order)
    }
  }
  float2 *dst = y1 + ((long long)r * n1 + i1) * npair;
  for (int j = lane; j < npair; j += 64) dst[j] = L[j];
}

// One workgroup per row r: the i1 transform of every pair (lanes over pairs, loads contiguous across
// lanes), each output k1 sent to its sphere vector through mapct [N1][npair] (-1: not on the sphere).
// The row's ng outputs are staged in LDS and written contiguously when they fit (STAGE), else directly.
constexpr int PLANE_C_STAGE = 8192;   // sphere vectors staged in LDS (64 KB)
template <int N1, bool HERM, bool STAGE>
__global__ __launch_bounds__(256, 2) void plane_c_kernel(const float2 *__restrict__ y1, int plane, int npair,
                                                      const int *__restrict__ mapct, int ng,
                                                      float2 *__restrict__ y, long long ldy) {
  extern __shared__ float2 so[];
  const int r = blockIdx.x;
  const int i1s = HERM ? r / plane : 0;          // planes left of the diagonal are zero
  const float2 *src = y1 + (long long)r * N1 * npair;
  float2 *yr = y + (long long)r * ldy;
#pragma unroll 1
  for (int p = threadIdx.x; p < npair; p += 256) {
    float2 X[N1];
    const float2 *sp = src + p;
    dft_regs_load<N1, 1>([&](int i1) { return i1 >= i1s ? sp[(long long)i1 * npair] : make_float2(0.f, 0.f); }, X);
    // outputs in groups of six map reads: a scheduling barrier between groups keeps the compiler from
    // issuing every map read at once (N1 more live registers, and spills at N1 = 36 and 48)
#pragma unroll
    for (int kc = 0; kc < N1; kc += 6) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k1 = kc; k1 < (kc + 6 < N1 ? kc + 6 : N1); ++k1) {
        const int g = mapct[k1 * npair + p];
        if (g >= 0) {
          if (STAGE) so[g] = X[k1];
          else yr[g] = X[k1];
        }
      }
    }
  }
  if (STAGE) {
    __syncthreads();
    for (int g = threadIdx.x; g < ng; g += 256) yr[g] = so[g];
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

hipError_t launch_plane_ab(int n, bool herm, const float2 *p, long long ldp, int nr, int n1, const int *k2list, int nk2,
                           const int *mapab, int npair, float2 *y1, hipStream_t s) {
  if (n1 > 65535 || nk2 > 64 || nk2 > n) return hipErrorInvalidValue;
  dim3 grid((nr + 3) / 4, n1), block(256);
  switch (n) {
#define GW_CASE(n_)                                                                                               \
  case n_:                                                                                                        \
    if (herm)                                                                                                     \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(plane_ab_kernel<n_, true>), grid, block, 0, s, p, ldp, nr, n1, k2list, nk2, \
                         mapab, npair, y1);                                                                      \
    else                                                                                                          \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(plane_ab_kernel<n_, false>), grid, block, 0, s, p, ldp, nr, n1, k2list, nk2, \
                         mapab, npair, y1);                                                                      \
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
  const size_t shm = stage ? (size_t)ng * sizeof(float2) : 0;
  dim3 grid(nr), block(256);
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
