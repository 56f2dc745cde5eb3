// FP64 inverse of a Hermitian positive definite matrix (eps of Sec. 5.1) by Cholesky:
//   eps = L L^H  (blocked: right-looking between panels of 128 columns, left-looking inside one),
//   X = L^-1 (blocked forward substitution on I, panel by panel behind the factorisation),
//   eps^-1 = X^H X.
// The paper inverts eps with a Newton iteration built on matrix products because that
// parallelises across distributed memory; on one GPU the factorisation costs about a
// third of the flops and every large step below is still a matrix product (zgemm).
//
// zgemm: C = alpha * op(A) op(B) + beta * C for complex128, op = identity or conjugate
// transpose, on v_mfma_f64_16x16x4f64.  Complex products use real MFMA with k' = (k, re/im):
//   Re C += [Re A, Im A] . [Re B; -Im B],   Im C += [Re A, Im A] . [Im B; Re B].
#include <algorithm>

#include <utility>

#include "gw_internal.h"

namespace gwi {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;    // output tile
constexpr int GK = 4;     // complex k per stage (8: 2% slower for the inverse at N = 4067, 16: 18% slower)

// The second product of a combined launch (lower_only == 3): same A, K, alpha, beta and leading
// dimensions, its own B, C and column count, over a full grid of tiles numbered after the first
// product's ntile1 lower tiles.
struct Zg2 {
  const double2 *B;
  double2 *C;
  int transB, N, ntile1;
};

__global__ __launch_bounds__(256, 4) void zgemm_kernel(int M, int N, int K, const double2 *__restrict__ A, long long lda,
                                                    int transA, const double2 *__restrict__ B, long long ldb,
                                                    int transB, double2 *__restrict__ C, long long ldc, double alpha,
                                                    double beta, int lower_only, int tri_k, int kchunk,
                                                    long long cz_stride, Zg2 z2) {
  // lower_only == 2: a square product over a one-dimensional grid of its lower tiles only, numbered row
  // by row (t = r (r + 1) / 2 + c), so consecutive workgroups, which the dispatcher deals out to the XCDs
  // in turn, carry equal work and no workgroup is launched for an upper tile
  int row0, col0;
  if (lower_only == 3 && (int)blockIdx.x >= z2.ntile1) {
    const int t = (int)blockIdx.x - z2.ntile1, nct = (z2.N + GT - 1) / GT;
    row0 = (t / nct) * GT;
    col0 = (t % nct) * GT;
    B = z2.B;
    C = z2.C;
    transB = z2.transB;
    N = z2.N;
  } else if (lower_only >= 2) {
    const int t = blockIdx.x;
    int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    row0 = r * GT;
    col0 = (t - r * (r + 1) / 2) * GT;
  } else {
    row0 = blockIdx.y * GT;
    col0 = blockIdx.x * GT;
  }
  // split K: workgroup z takes k in [z kchunk, (z+1) kchunk) and writes its own partial C
  int kend = K;
  if (kchunk > 0) {
    C += blockIdx.z * cz_stride;
    kend = min(K, (int)(blockIdx.z + 1) * kchunk);
  }
  if (lower_only == 1 && col0 >= row0 + GT) return;
  // two LDS stages: the global loads of stage k+1 are in flight in registers while stage k's MFMAs run
  __shared__ double sA[2][GK][2][GT];
  __shared__ double sX[2][GK][2][GT];   // [Re B; -Im B]; the [Im B; Re B] operand is read from it
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  f64x4 accR[2][2], accI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) { accR[a][b][e] = 0.0; accI[a][b][e] = 0.0; }

  int kbeg = kchunk > 0 ? (int)blockIdx.z * kchunk : 0;
  if (tri_k) kbeg = (max(row0, col0) / GK) * GK;
  const int kl = lane >> 4, li = lane & 15;
  constexpr int PER = (GT * GK) / 256;   // elements of each operand per thread and stage
  double2 va[PER], vb[PER];
  // element idx of a stage: A row r / B column c and its k offset kk, in the order that keeps the
  // global reads contiguous for either layout
  auto a_coord = [&](int idx, int &r, int &kk) {
    if (transA) { r = idx % GT; kk = idx / GT; } else { r = idx / GK; kk = idx % GK; }
  };
  auto b_coord = [&](int idx, int &c, int &kk) {
    if (transB) { c = idx / GK; kk = idx % GK; } else { c = idx % GT; kk = idx / GT; }
  };
  // Loads keep the raw values; the conjugation of a transposed operand is applied when they are
  // written to LDS, so no instruction waits on a load before the stage's MFMAs have been issued.
  // Each thread's elements advance by GK along k per stage: running pointers, and no bounds test in
  // the stages of a whole tile that lie inside [kbeg, kend).
  const double2 *pa[PER], *pb[PER];
  int ka[PER], kb[PER];
  bool ra[PER], cb_ok[PER];
#pragma unroll
  for (int it = 0; it < PER; ++it) {
    const int idx = tid + it * 256;
    int r, c, kk;
    a_coord(idx, r, kk);
    ka[it] = kk;
    ra[it] = row0 + r < M;
    const int rr = min(row0 + r, M - 1);   // an address inside A for rows past M (never read)
    pa[it] = transA ? A + (long long)(kbeg + kk) * lda + rr : A + (long long)rr * lda + kbeg + kk;
    b_coord(idx, c, kk);
    kb[it] = kk;
    cb_ok[it] = col0 + c < N;
    const int cc = min(col0 + c, N - 1);
    pb[it] = transB ? B + (long long)cc * ldb + kbeg + kk : B + (long long)(kbeg + kk) * ldb + cc;
  }
  const long long step_a = transA ? (long long)GK * lda : GK, step_b = transB ? GK : (long long)GK * ldb;
  const bool whole = row0 + GT <= M && col0 + GT <= N;
  auto gload = [&](int k0) {
    if (whole && k0 + GK <= kend) {        // uniform
#pragma unroll
      for (int it = 0; it < PER; ++it) {
        va[it] = *pa[it];
        vb[it] = *pb[it];
      }
    } else {
#pragma unroll
      for (int it = 0; it < PER; ++it) {
        va[it] = make_double2(0.0, 0.0);
        if (ra[it] && k0 + ka[it] < kend) va[it] = *pa[it];
        vb[it] = make_double2(0.0, 0.0);
        if (cb_ok[it] && k0 + kb[it] < kend) vb[it] = *pb[it];
      }
    }
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      pa[it] += step_a;
      pb[it] += step_b;
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int idx = tid + it * 256;
      int r, c, kk;
      a_coord(idx, r, kk);
      sA[buf][kk][0][r] = va[it].x;
      sA[buf][kk][1][r] = transA ? -va[it].y : va[it].y;
      b_coord(idx, c, kk);
      const double by = transB ? -vb[it].y : vb[it].y;
      sX[buf][kk][0][c] = vb[it].x;
      sX[buf][kk][1][c] = -by;
    }
  };
  int buf = 0;
  if (kbeg < kend) {
    gload(kbeg);
    lstore(0);
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += GK) {
    const bool more = k0 + GK < kend;
    if (more) gload(k0 + GK);
#pragma unroll
    for (int s = 0; s < GK / 2; ++s) {
      const int kk = 2 * s + (kl >> 1), comp = kl & 1;
      const double a0 = sA[buf][kk][comp][wr * 32 + li], a1 = sA[buf][kk][comp][wr * 32 + 16 + li];
      const double x0 = sX[buf][kk][comp][wc * 32 + li], x1 = sX[buf][kk][comp][wc * 32 + 16 + li];
      // Y = [Im B; Re B] = [-X_1; X_0]: the sign flip of the comp = 0 lanes as one xor of the high word
      const double ys0 = sX[buf][kk][comp ^ 1][wc * 32 + li], ys1 = sX[buf][kk][comp ^ 1][wc * 32 + 16 + li];
      const unsigned long long flip = comp ? 0ull : 0x8000000000000000ull;
      const double y0 = __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, ys0) ^ flip);
      const double y1 = __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, ys1) ^ flip);
      accR[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, x0, accR[0][0], 0, 0, 0);
      accI[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, y0, accI[0][0], 0, 0, 0);
      accR[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, x1, accR[0][1], 0, 0, 0);
      accI[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, y1, accI[0][1], 0, 0, 0);
      accR[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, x0, accR[1][0], 0, 0, 0);
      accI[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, y0, accI[1][0], 0, 0, 0);
      accR[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, x1, accR[1][1], 0, 0, 0);
      accI[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, y1, accI[1][1], 0, 0, 0);
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // lane holds D[i][j] of each 16x16 block in register e with i = 4*e + (lane>>4), j = lane & 15
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = row0 + wr * 32 + rb * 16 + 4 * e + kl;
        const int col = col0 + wc * 32 + cb * 16 + li;
        if (row < M && col < N) {
          double2 *d = C + (long long)row * ldc + col;
          double2 v = make_double2(alpha * accR[rb][cb][e], alpha * accI[rb][cb][e]);
          if (beta != 0.0) { const double2 o = *d; v.x += beta * o.x; v.y += beta * o.y; }
          *d = v;
        }
      }
}

static hipError_t zgemm(int M, int N, int K, const double2 *A, long long lda, int transA, const double2 *B,
                        long long ldb, int transB, double2 *C, long long ldc, double alpha, double beta,
                        int lower_only, int tri_k, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (lower_only && M == N) {
    const long long nt = (N + GT - 1) / GT;
    hipLaunchKernelGGL(zgemm_kernel, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, s, M, N, K, A, lda, transA, B,
                       ldb, transB, C, ldc, alpha, beta, 2, tri_k, 0, 0LL, Zg2{});
    return hipGetLastError();
  }
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  hipLaunchKernelGGL(zgemm_kernel, grid, dim3(256), 0, s, M, N, K, A, lda, transA, B, ldb, transB, C, ldc, alpha,
                     beta, lower_only, tri_k, 0, 0LL, Zg2{});
  return hipGetLastError();
}

// C1 = alpha A B1^H + beta C1 on the lower tiles of the square M x M C1, and C2 = alpha A B2 + beta C2 on
// all tiles of the M x N2 C2, in one launch (both operands B row-major with leading dimension ldb)
static hipError_t zgemm_lower_and_full(int M, int N2, int K, const double2 *A, long long lda, const double2 *B1,
                                       double2 *C1, const double2 *B2, double2 *C2, long long ldb, long long ldc,
                                       double alpha, double beta, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  const long long nt = (M + GT - 1) / GT, nt1 = nt * (nt + 1) / 2, nt2 = N2 > 0 ? nt * ((N2 + GT - 1) / GT) : 0;
  hipLaunchKernelGGL(zgemm_kernel, dim3((unsigned)(nt1 + nt2)), dim3(256), 0, s, M, M, K, A, lda, 0, B1, ldb, 1, C1,
                     ldc, alpha, beta, 3, 0, 0, 0LL, Zg2{B2, C2, 0, N2, (int)nt1});
  return hipGetLastError();
}

// c[i][j] = alpha sum_z w[z][i][j] + beta c[i][j]   (w packed [kz][M][N])
__global__ void splitk_reduce_kernel(const double2 *__restrict__ w, int kz, int M, int N, double2 *__restrict__ c,
                                     long long ldc, double alpha, double beta) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)M * N) return;
  const int i = (int)(idx / N), j = (int)(idx % N);
  double re = 0.0, im = 0.0;
  for (int z = 0; z < kz; ++z) {
    const double2 v = w[(size_t)z * M * N + idx];
    re += v.x;
    im += v.y;
  }
  double2 *d = c + (long long)i * ldc + j;
  double2 out = make_double2(alpha * re, alpha * im);
  if (beta != 0.0) {
    const double2 o = *d;
    out.x += beta * o.x;
    out.y += beta * o.y;
  }
  *d = out;
}

size_t zgemm_splitk_ws_elems(int M, int N, int K) {
  const long long tiles = (long long)((M + GT - 1) / GT) * ((N + GT - 1) / GT);
  if (tiles >= 256 || K < 4 * GK) return 0;
  const int kz = (int)std::min<long long>(std::max<long long>(1, 512 / tiles), (K + 255) / 256);
  return kz > 1 ? (size_t)kz * M * N : 0;
}

hipError_t launch_zgemm_splitk(int M, int N, int K, const double2 *A, long long lda, int transA, const double2 *B,
                               long long ldb, int transB, double2 *C, long long ldc, double alpha, double beta,
                               double2 *ws, size_t ws_elems, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const size_t need = zgemm_splitk_ws_elems(M, N, K);
  if (need == 0 || ws == nullptr || ws_elems < need)
    return zgemm(M, N, K, A, lda, transA, B, ldb, transB, C, ldc, alpha, beta, 0, 0, s);
  const int kz = (int)(need / ((size_t)M * N));
  int kchunk = (K + kz - 1) / kz;
  kchunk = (kchunk + GK - 1) / GK * GK;
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, kz);
  // each z slice writes every (i, j) of its partial (padded k past kend reads zero), so ws needs no clearing
  hipLaunchKernelGGL(zgemm_kernel, grid, dim3(256), 0, s, M, N, K, A, lda, transA, B, ldb, transB, ws, (long long)N,
                     1.0, 0.0, 0, 0, kchunk, (long long)M * N, Zg2{});
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)(((size_t)M * N + 255) / 256)), dim3(256), 0, s, ws, kz, M,
                     N, C, ldc, alpha, beta);
  return hipGetLastError();
}

hipError_t launch_zgemm(int M, int N, int K, const double2 *A, long long lda, int transA, const double2 *B,
                        long long ldb, int transB, double2 *C, long long ldc, double alpha, double beta,
                        hipStream_t s) {
  return zgemm(M, N, K, A, lda, transA, B, ldb, transB, C, ldc, alpha, beta, 0, 0, s);
}

// ---- diagonal block L_kk = chol(A_kk), Linv_kk = L_kk^-1, and the panel column below it -------------
// Every workgroup first applies the panel's earlier columns to the block and to its panel rows, then
// factors and inverts the 32 x 32 block in LDS (cheap, and it saves a dependent launch per step);
// workgroup 0 stores L_kk, Linv_kk and the pivot flag, and workgroup g forms PR rows of the panel
// L[k0+nb+PR g : +PR, k0 : k0+nb] = A Linv_kk^H.  With PR = 16 the panel product of a 4067-row
// matrix spreads over about 250 CUs (64 rows per workgroup left three quarters of the CUs idle).
constexpr int NB = 32;
constexpr int PR = 16;    // panel rows per workgroup of the diagonal-block kernel
constexpr int CHOL_PW = 128;   // panel width of the factorisation and the substitution
constexpr int PD_THREADS = PR * NB;   // diagonal-block kernel: eight waves, one panel entry per thread

// 1 / d for a positive finite d: the hardware estimate refined by two Newton steps r <- r + r (1 - d r),
// each of which squares the relative error (within an ulp or two of the rounded quotient); three
// dependent operations fewer than the correctly rounded division on the factorisation's latency chain
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

// f(integral_constant<int, J>) for J = 0, 1, ...: loop bodies whose index must be a constant
template <typename F, int... J>
__device__ __forceinline__ void static_for(F &&f, std::integer_sequence<int, J...>) {
  (f(std::integral_constant<int, J>{}), ...);
}

__global__ __launch_bounds__(PD_THREADS) void potrf_diag_kernel(const double2 *__restrict__ A, int n, int p0,
                                                                int k0, double2 *__restrict__ L,
                                                                double2 *__restrict__ linv, int *__restrict__ pivot) {
  __shared__ double2 a[NB][NB + 1];
  // L[k0 + i][p0 + k] (the block's rows, the panel's earlier columns) and the same columns of this
  // workgroup's panel rows, planar: [k][re, im][row], the operand layout of the FP64 MFMA
  __shared__ double lbp[CHOL_PW - NB][2][NB + 1];
  __shared__ double lrp[CHOL_PW - NB][2][PR + 1];
  __shared__ double2 x[NB][NB + 1];
  __shared__ double2 pa[PR][NB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int nb = min(NB, n - k0);
  // this workgroup's PR panel rows below the block, loaded now so that their latency overlaps the
  // factorisation: thread (pib, pj) holds A[r0 + pib][k0 + pj]
  const int r0 = k0 + nb + (int)blockIdx.x * PR;
  const int pj = tid % NB, pib = tid / NB;
  static_assert(PR * NB == PD_THREADS, "one panel entry per thread");
  double2 pv = (r0 + pib < n && pj < nb) ? A[(size_t)(r0 + pib) * n + k0 + pj] : make_double2(0.0, 0.0);
  if (tid == 0) bad = 0;
  for (int idx = tid; idx < NB * NB; idx += PD_THREADS) {
    const int i = idx / NB, j = idx % NB;
    double2 v = make_double2(0.0, 0.0);
    if (i < nb && j < nb && j <= i) v = A[(size_t)(k0 + i) * n + k0 + j];
    if (i >= nb && i == j) v = make_double2(1.0, 0.0);      // pad with identity
    a[i][j] = v;
    x[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  pa[pib][pj] = pv;
  // Left-looking inside the panel: the kp = k0 - p0 columns of this panel factored by the earlier steps
  // are applied here, A[k0:, k0:k0+nb] -= L[k0:, p0:k0] L[k0:k0+nb, p0:k0]^H, to this workgroup's copy of
  // the diagonal block and to its panel rows, instead of by a separate product after every step.  Five
  // waves each form one 16 x 16 tile on the FP64 MFMA, with k' = (k, re/im) as in zgemm_kernel:
  // Re C += [Re A, Im A] . [Re B; Im B] and Im C += [Re A, Im A] . [-Im B; Re B] for C = A B^H.  Waves 0
  // and 1 take the panel rows' two column halves, waves 2 to 4 the block's lower tiles (0,0), (1,0), (1,1).
  const int kp = k0 - p0;                                   // a multiple of NB
  static_assert(2 * PR == NB, "rows pib and pib + PR cover the block");
  if (kp > 0) {
#pragma unroll
    for (int q = 0; q < (CHOL_PW - NB) / NB; ++q) {
      if (NB * q < kp) {                                     // column k = pj + NB q; rows pib and pib + PR
        const int k = pj + NB * q;
        const double2 u = pib < nb ? L[(size_t)(k0 + pib) * n + p0 + k] : make_double2(0.0, 0.0);
        const double2 w = pib + PR < nb ? L[(size_t)(k0 + pib + PR) * n + p0 + k] : make_double2(0.0, 0.0);
        const double2 v = r0 + pib < n ? L[(size_t)(r0 + pib) * n + p0 + k] : make_double2(0.0, 0.0);
        lbp[k][0][pib] = u.x;
        lbp[k][1][pib] = u.y;
        lbp[k][0][pib + PR] = w.x;
        lbp[k][1][pib + PR] = w.y;
        lrp[k][0][pib] = v.x;
        lrp[k][1][pib] = v.y;
      }
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63, kl = lane >> 4, li = lane & 15;
    if (wave < 5) {                                          // wave-uniform
      const bool rows = wave < 2;
      const int ra = rows ? 0 : (wave == 2 ? 0 : 16);        // first row of the tile (panel rows or block)
      const int cb = rows ? 16 * wave : (wave == 4 ? 16 : 0);  // first column (block row of B)
      f64x4 accR = {0.0, 0.0, 0.0, 0.0}, accI = {0.0, 0.0, 0.0, 0.0};
      const int comp = kl & 1;
      const unsigned long long flip = comp ? 0ull : 0x8000000000000000ull;   // Y = [-Im B; Re B]
      for (int s2 = 0; s2 < kp; s2 += 2) {
        const int kk = s2 + (kl >> 1);
        const double av = rows ? lrp[kk][comp][li] : lbp[kk][comp][ra + li];
        const double xv = lbp[kk][comp][cb + li];
        const double ys = lbp[kk][comp ^ 1][cb + li];
        const double yv = __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, ys) ^ flip);
        accR = __builtin_amdgcn_mfma_f64_16x16x4f64(av, xv, accR, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f64_16x16x4f64(av, yv, accI, 0, 0, 0);
      }
      // lane holds tile entry (4 e + kl, li) in register e
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 4 * e + kl;
        if (rows) {
          pa[i][cb + li].x -= accR[e];
          pa[i][cb + li].y -= accI[e];
        } else if (ra + i >= cb + li) {                      // lower entries of the block only
          a[ra + i][cb + li].x -= accR[e];
          a[ra + i][cb + li].y -= accI[e];
        }
      }
    }
  }
  // Unblocked right-looking Cholesky on the lower triangle, with unscaled columns: step j subtracts
  // s_j s_j^H / d_j (d_j the pivot, s_j column j) from the trailing lower triangle.  In elimination form
  // A = Lu D Lu^H with Lu = I + sum_j (s_j / d_j) e_j^T below the diagonal, so the same step also applies
  // Lu's j-th elimination to X (started as I): row i > j loses (s_j(i) / d_j) times row j, on the columns
  // m <= j where row j is non-zero.  After the last step X = Lu^-1, and L = Lu D^1/2, L^-1 = D^-1/2 X
  // follow by scaling.
  //
  // The 32 steps form the kernel's latency chain.  The block lives in registers, spread over the first
  // four waves (the other four only take part in the barriers): lane (m, c) = (tid % 32, tid / 32) keeps
  // one column on the rows i = 8t + c, so each lane updates four rows per step.  Column m of A changes
  // only in the steps j < m and column m of X only in the steps j >= m (X is I on it until then), so the
  // lanes of column m hold A's column until step m, where they pass it on and take X's identity column
  // in its place.  Step j's column of the factor and row of X go to LDS rows of their own (colj[j],
  // xrowj[j]), so one barrier per step orders the writes before the reads and no step overwrites what
  // another still reads.  Every lane then subtracts s_j(i) w on its rows i > j, with w = conj(s_j(m)) / d_j
  // while it holds A (m > j) and X[j][m] / d_j once it holds X.  On A's columns this also writes rows
  // j < i < m above the diagonal; those rows are never read, and X's column is zeroed above its diagonal
  // when it is stored.
  __shared__ double2 colj[NB][NB + 1], xrowj[NB][NB + 1];
  {
    constexpr int C = 8, T = NB / C;                        // row classes, rows per lane
    const int m = tid % NB, c = tid / NB;
    const bool fw = c < C;                                  // wave-uniform: one of the factoring waves
    double2 z[T];
    __syncthreads();
    if (fw) {
#pragma unroll
      for (int t = 0; t < T; ++t) z[t] = a[C * t + c][m];
    }
    int badj = 0;
    auto step = [&](auto jc) {                                 // step j, a compile-time index
      constexpr int j = decltype(jc)::value, jt = j / C, jr = j % C;
      if (fw) {
        if (m == j) {
#pragma unroll
          for (int t = jt; t < T; ++t) colj[j][C * t + c] = z[t];     // column j, final from here on
#pragma unroll
          for (int t = jt; t < T; ++t) z[t] = make_double2(C * t + c == m ? 1.0 : 0.0, 0.0);   // X's column
        }
        if (c == jr) xrowj[j][m] = z[jt];                        // row j of X (read only where m <= j)
      }
      __syncthreads();
      if (fw) {
        const double d0 = colj[j][j].x;
        const double2 q = colj[j][m], xq = xrowj[j][m];
        double2 pj[T];
#pragma unroll
        for (int t = jt; t < T; ++t) pj[t] = colj[j][C * t + c];
        const bool okd = d0 > 0.0 && isfinite(d0);
        badj = (!okd && j < nb && badj == 0) ? k0 + j + 1 : badj;
        const double dinv = recip(okd ? d0 : 1.0);
        const bool fac = m > j;
        const double wx = (fac ? q.x : xq.x) * dinv;
        const double wy = (fac ? -q.y : xq.y) * dinv;
#pragma unroll
        for (int t = jt; t < T; ++t) {
          if (t > jt || c > jr) {                                // rows i > j
            z[t].x -= pj[t].x * wx - pj[t].y * wy;
            z[t].y -= pj[t].x * wy + pj[t].y * wx;
          }
        }
      }
    };
    static_for(step, std::make_integer_sequence<int, NB>{});
    if (fw) {
#pragma unroll
      for (int t = 0; t < T; ++t) x[C * t + c][m] = C * t + c >= m ? z[t] : make_double2(0.0, 0.0);
    }
    if (tid == 0) bad = badj;
  }
  __syncthreads();
  // r_j = sqrt(d_j) (bad pivots were replaced by 1 and flagged); L = column j over r_j, L^-1 = row i of X
  // over r_i
  __shared__ double rs[NB];
  if (tid < NB) {
    double d = colj[tid][tid].x;
    if (!(d > 0.0) || !isfinite(d)) d = 1.0;
    rs[tid] = sqrt(d);
  }
  __syncthreads();
  for (int idx = tid; idx < NB * NB; idx += PD_THREADS) {
    const int i = idx / NB, j = idx % NB;
    if (j <= i) {
      const double r = rs[j];
      a[i][j] = (i == j) ? make_double2(r, 0.0) : make_double2(colj[j][i].x / r, colj[j][i].y / r);
    }
    const double ri = rs[i];
    x[i][j] = make_double2(x[i][j].x / ri, x[i][j].y / ri);
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int idx = tid; idx < NB * NB; idx += PD_THREADS) {
      const int i = idx / NB, j = idx % NB;
      if (i < nb && j < nb) L[(size_t)(k0 + i) * n + k0 + j] = (j <= i) ? a[i][j] : make_double2(0.0, 0.0);
      linv[idx] = (i < nb && j < nb) ? x[i][j] : make_double2(0.0, 0.0);
    }
    if (tid == 0 && bad != 0 && *pivot == 0) *pivot = bad;
  }
  // panel below the block, one entry per thread (every workgroup factored the block above for itself):
  // L[r][k0 + j] = sum_{k <= j} A[r][k0 + k] conj(Linv[j][k]).  Linv is lower triangular with its upper
  // part stored as zeros, so the k loop runs to NB for every thread: no divergence.
  if (r0 >= n) return;
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll 8
  for (int k = 0; k < NB; ++k) {
    const double2 v = x[pj][k], av = pa[pib][k];
    acc.x += av.x * v.x + av.y * v.y;
    acc.y += av.y * v.x - av.x * v.y;
  }
  if (r0 + pib < n && pj < nb) L[(size_t)(r0 + pib) * n + k0 + pj] = acc;
}

__global__ void fill_identity_kernel(double2 *__restrict__ a, int n, double diag) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const size_t i = idx / n, j = idx % n;
  a[idx] = make_double2(i == j ? diag : 0.0, 0.0);
}

// out[j][i] = conj(out[i][j]) for i > j (upper triangle from the lower), 32x32 tiles via LDS.
__global__ __launch_bounds__(256) void mirror_lower_kernel(double2 *__restrict__ a, int n) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  __shared__ double2 t[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = 0; k < 32; k += 8) {
    const int i = bi * 32 + ty + k, j = bj * 32 + tx;
    if (i < n && j < n) t[ty + k][tx] = a[(size_t)i * n + j];
  }
  __syncthreads();
  for (int k = 0; k < 32; k += 8) {
    const int i = bj * 32 + ty + k, j = bi * 32 + tx;     // destination (i, j) in the upper tile
    if (i < n && j < n && j > i) {
      const double2 v = t[tx][ty + k];                    // a[j][i]
      a[(size_t)i * n + j] = make_double2(v.x, -v.y);
    }
  }
}

__global__ void fill_int_kernel(int *p, int v) { *p = v; }

hipError_t launch_fill_int(int *p, int value, hipStream_t s) {
  hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(1), 0, s, p, value);
  return hipGetLastError();
}

// ---- block substitution of one panel of rows, X[p0:p1, :] from B[p0:p1, :] ----------------------------
// The columns of B are independent, so a workgroup carries its SUB_CW columns through the panel's
// 32-row steps in LDS: X_k = Linv_kk B_k, then B_i -= L_ik X_k for the panel's later row blocks.
// One launch per panel replaces two small GEMMs per step.
constexpr int SUB_CW = 8;      // columns per workgroup
constexpr int SUB_RS = 256 / SUB_CW;   // row stride of a thread's rows in a 32-row block

__global__ __launch_bounds__(256) void subst_panel_kernel(const double2 *__restrict__ B, const double2 *__restrict__ L,
                                                          const double2 *__restrict__ linv_all,
                                                          double2 *__restrict__ X, int n, int p0, int p1) {
  __shared__ double2 sB[CHOL_PW][SUB_CW + 1];
  __shared__ double2 sM[NB][NB + 1];   // Linv_kk, then one L_ik block at a time
  constexpr int PER = NB * SUB_CW / 256;
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * SUB_CW;
  const int rows = p1 - p0;
  for (int idx = tid; idx < CHOL_PW * SUB_CW; idx += 256) {
    const int i = idx / SUB_CW, c = idx % SUB_CW;
    sB[i][c] = (i < rows && c0 + c < n) ? B[(size_t)(p0 + i) * n + c0 + c] : make_double2(0.0, 0.0);
  }
  // The 32 x 32 blocks pass through sM in the order Linv_(k0), L_(k0+32, k0), ..., Linv_(k0+32), ...; each
  // is loaded into registers (pf) while the block before it is in use, and written to sM when that is free.
  double2 pf[NB * NB / 256];
  auto fetch = [&](int k0, int j0) {   // j0 < 0: Linv of block k0; else L[j0 : j0 + 32, k0 : k0 + 32], zero-padded
    const int nb = min(NB, n - k0), jn = min(NB, p1 - j0);
#pragma unroll
    for (int t = 0; t < NB * NB / 256; ++t) {
      const int idx = tid + 256 * t, i = idx / NB, m = idx % NB;
      if (j0 < 0)
        pf[t] = linv_all[(size_t)(k0 / NB) * NB * NB + idx];
      else
        pf[t] = (i < jn && m < nb) ? L[(size_t)(j0 + i) * n + k0 + m] : make_double2(0.0, 0.0);
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int t = 0; t < NB * NB / 256; ++t) {
      const int idx = tid + 256 * t;
      sM[idx / NB][idx % NB] = pf[t];
    }
  };
  fetch(p0, -1);
  for (int k0 = p0; k0 < p1; k0 += NB) {
    const int nb = min(NB, n - k0), kr = k0 - p0;
    commit();
    __syncthreads();
    if (k0 + NB < p1) fetch(k0, k0 + NB);
    // X_k = Linv_kk B_k.  Linv_kk is stored with zeros above its diagonal, so m runs over the whole
    // block for every thread: thread (i = ib + SUB_RS t, c) keeps PER independent sums.
    const int ib = tid / SUB_CW, c = tid % SUB_CW;
    double2 xv[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) xv[t] = make_double2(0.0, 0.0);
#pragma unroll 4
    for (int m = 0; m < NB; ++m) {
      const double2 v = sB[kr + m][c];
#pragma unroll
      for (int t = 0; t < PER; ++t) {
        const double2 u = sM[ib + SUB_RS * t][m];
        xv[t].x += u.x * v.x - u.y * v.y;
        xv[t].y += u.x * v.y + u.y * v.x;
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int idx = tid + 256 * t, i = idx / SUB_CW, c = idx % SUB_CW;
      if (i < nb) {
        sB[kr + i][c] = xv[t];
        if (c0 + c < n) X[(size_t)(k0 + i) * n + c0 + c] = xv[t];
      }
    }
    // the panel's later row blocks: B_i -= L_ik X_k
    for (int j0 = k0 + NB; j0 < p1; j0 += NB) {
      const int jn = min(NB, p1 - j0), jr = j0 - p0;
      __syncthreads();
      commit();
      __syncthreads();
      if (j0 + NB < p1)
        fetch(k0, j0 + NB);
      else if (k0 + NB < p1)
        fetch(k0 + NB, -1);
      // sM is zero for m >= nb, so m runs over the whole block here too
      double2 acc[PER];
#pragma unroll
      for (int t = 0; t < PER; ++t) acc[t] = make_double2(0.0, 0.0);
#pragma unroll 4
      for (int m = 0; m < NB; ++m) {
        const double2 v = sB[kr + m][c];
#pragma unroll
        for (int t = 0; t < PER; ++t) {
          const double2 u = sM[ib + SUB_RS * t][m];
          acc[t].x += u.x * v.x - u.y * v.y;
          acc[t].y += u.x * v.y + u.y * v.x;
        }
      }
#pragma unroll
      for (int t = 0; t < PER; ++t) {
        const int i = ib + SUB_RS * t;
        if (i < jn) {
          sB[jr + i][c].x -= acc[t].x;
          sB[jr + i][c].y -= acc[t].y;
        }
      }
    }
    __syncthreads();
  }
}

size_t chol_small_bytes(int n) {
  const int nblk = (n + NB - 1) / NB;
  return (size_t)nblk * NB * NB * sizeof(double2);
}

#define GW_TRY(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return e_; } while (0)

hipError_t hpd_inverse(double2 *a, int n, double2 *l, double2 *x, double2 *small, int *pivot_dev, double2 *out,
                       hipStream_t s) {
  const size_t nn = (size_t)n * n;
  const unsigned fill_blocks = (unsigned)((nn + 255) / 256);
  GW_TRY(launch_fill_int(pivot_dev, 0, s));
  hipLaunchKernelGGL(fill_identity_kernel, dim3(fill_blocks), dim3(256), 0, s, l, n, 0.0);
  GW_TRY(hipGetLastError());
  // the substitution's right-hand side B = I lives in out until X^H X overwrites it
  hipLaunchKernelGGL(fill_identity_kernel, dim3(fill_blocks), dim3(256), 0, s, out, n, 1.0);
  GW_TRY(hipGetLastError());
  hipLaunchKernelGGL(fill_identity_kernel, dim3(fill_blocks), dim3(256), 0, s, x, n, 0.0);
  GW_TRY(hipGetLastError());
  // Panels of PW columns, factorisation and substitution interleaved.  Inside a panel each NB-wide step of
  // the factorisation first applies the panel's earlier columns to its own (left-looking, inside the
  // diagonal-block kernel, so a step is one launch).  The panel's rows of X = L^-1 need only L's rows of
  // this panel and B's rows, so they follow at once.  Then one launch of K = PW products updates both
  // what lies right of the panel in A and below it in B, with the same left operand L[p1:, p0:p1]: the
  // large trailing matrices are read and written once per panel, and the two products fill the GPU
  // together where one alone would leave CUs idle (few trailing rows late, few B columns early).
  // (A look-ahead that moved each panel's trailing product to a second stream, so that the next panel's
  // chain could start at once, measured slower at N = 4067: the product's workgroups fill the CUs the
  // chain's small launches wait for.)
  constexpr int PW = CHOL_PW;   // 128, 256 and 512 measured alike; 32 (no panels) 5% slower at N = 4067
  for (int p0 = 0; p0 < n; p0 += PW) {
    const int p1 = min(n, p0 + PW);
    // 1. factor the panel: L[p0:, p0:p1]
    for (int k0 = p0; k0 < p1; k0 += NB) {
      const int kb = k0 / NB, nb = min(NB, n - k0), rest = n - k0 - nb;
      double2 *linv = small + (size_t)kb * NB * NB;
      // the diagonal block and, in the same launch, the panel column L[k0+nb:, k0:k0+nb] = A Linv^H
      hipLaunchKernelGGL(potrf_diag_kernel, dim3(std::max(1, (rest + PR - 1) / PR)), dim3(PD_THREADS), 0, s, a, n, p0,
                         k0, l, linv, pivot_dev);
      GW_TRY(hipGetLastError());
    }
    // 2. the panel's rows of X (columns < p1; X is zero beyond), all 32-row steps in one launch
    hipLaunchKernelGGL(subst_panel_kernel, dim3((p1 + SUB_CW - 1) / SUB_CW), dim3(256), 0, s, out, l, small, x, n, p0,
                       p1);
    GW_TRY(hipGetLastError());
    // 3. A[p1:, p1:] -= Lp Lp^H (lower tiles) and B[p1:, :p1] -= Lp X[p0:p1, :p1], Lp = L[p1:, p0:p1]
    const int rest = n - p1;
    if (rest > 0) {
      const double2 *lp = l + (size_t)p1 * n + p0;
      GW_TRY(zgemm_lower_and_full(rest, p1, p1 - p0, lp, n, lp, a + (size_t)p1 * n + p1, x + (size_t)p0 * n,
                                  out + (size_t)p1 * n, n, n, -1.0, 1.0, s));
    }
  }
  // 3. out = X^H X (lower tiles, k from max(row, col) since X is lower triangular), then mirror
  GW_TRY(zgemm(n, n, n, x, n, 1, x, n, 0, out, n, 1.0, 0.0, 1, 1, s));
  dim3 mg((n + 31) / 32, (n + 31) / 32);
  hipLaunchKernelGGL(mirror_lower_kernel, mg, dim3(256), 0, s, out, n);
  return hipGetLastError();
}

// ---- Newton iteration for the inverse (Sec. 5.1): X_{n+1} = X_n (2I - A X_n), X_0 = alpha A^H -------
// alpha = 1 / max_i sum_j |(A A^H)_ij| (absolute values make alpha <= 1/sigma_max^2, so the iteration
// converges for any nonsingular A).  Every product is the complex FP64 MFMA GEMM above.

// per-row sum of |m_ij| into rs[i]
__global__ void row_abs_sum_kernel(const double2 *__restrict__ m, int n, double *__restrict__ rs) {
  const int i = blockIdx.x;
  __shared__ double red[256];
  double a = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    const double2 v = m[(size_t)i * n + j];
    a += sqrt(v.x * v.x + v.y * v.y);
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) rs[i] = red[0];
}

// out[0] = max of v[0..n) (one workgroup); with inv set, out[0] = 1 / max
__global__ void max_reduce_kernel(const double *__restrict__ v, int n, double *__restrict__ out, int inv) {
  __shared__ double red[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a = fmax(a, v[i]);
  red[threadIdx.x] = a;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = inv ? 1.0 / red[0] : red[0];
}

// x = alpha * a^H with alpha read from device memory
__global__ __launch_bounds__(256) void scaled_conj_transpose_kernel(const double2 *__restrict__ a, int n,
                                                                    const double *__restrict__ alpha,
                                                                    double2 *__restrict__ x) {
  __shared__ double2 t[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double al = alpha[0];
  for (int k = 0; k < 32; k += 8) {
    const int r = r0 + ty + k, c = c0 + tx;
    if (r < n && c < n) t[ty + k][tx] = a[(size_t)r * n + c];
  }
  __syncthreads();
  for (int k = 0; k < 32; k += 8) {
    const int r = c0 + ty + k, c = r0 + tx;        // x[r][c] = alpha conj(a[c][r])
    if (r < n && c < n) {
      const double2 v = t[tx][ty + k];
      x[(size_t)r * n + c] = make_double2(al * v.x, -al * v.y);
    }
  }
}

// per-row max |x_ij - y_ij| into rm[i]
__global__ void row_max_diff_kernel(const double2 *__restrict__ x, const double2 *__restrict__ y, int n,
                                    double *__restrict__ rm) {
  const int i = blockIdx.x;
  __shared__ double red[256];
  double a = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    const double2 u = x[(size_t)i * n + j], v = y[(size_t)i * n + j];
    const double dx = u.x - v.x, dy = u.y - v.y;
    a = fmax(a, sqrt(dx * dx + dy * dy));
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) rm[i] = red[0];
}

size_t newton_ws_bytes(int n) { return 3 * (size_t)n * n * sizeof(double2) + ((size_t)n + 64) * sizeof(double); }

hipError_t newton_start(const double2 *a, int n, double2 *x, double2 *t, double *scratch, hipStream_t s) {
  // t = A A^H, alpha = 1 / max_i sum_j |t_ij|, x = alpha A^H
  GW_TRY(zgemm(n, n, n, a, n, 0, a, n, 1, t, n, 1.0, 0.0, 0, 0, s));
  hipLaunchKernelGGL(row_abs_sum_kernel, dim3(n), dim3(256), 0, s, t, n, scratch + 64);
  GW_TRY(hipGetLastError());
  hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, s, scratch + 64, n, scratch, 1);
  GW_TRY(hipGetLastError());
  dim3 g((n + 31) / 32, (n + 31) / 32);
  hipLaunchKernelGGL(scaled_conj_transpose_kernel, g, dim3(256), 0, s, a, n, scratch, x);
  return hipGetLastError();
}

hipError_t newton_step(const double2 *a, int n, const double2 *x, double2 *t, double2 *xn, double *scratch,
                       hipStream_t s) {
  // t = 2I - A X, xn = X t, scratch[1] = max |xn - x|
  const size_t nn = (size_t)n * n;
  hipLaunchKernelGGL(fill_identity_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, t, n, 2.0);
  GW_TRY(hipGetLastError());
  GW_TRY(zgemm(n, n, n, a, n, 0, x, n, 0, t, n, -1.0, 1.0, 0, 0, s));
  GW_TRY(zgemm(n, n, n, x, n, 0, t, n, 0, xn, n, 1.0, 0.0, 0, 0, s));
  hipLaunchKernelGGL(row_max_diff_kernel, dim3(n), dim3(256), 0, s, xn, x, n, scratch + 64);
  GW_TRY(hipGetLastError());
  hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, s, scratch + 64, n, scratch + 1, 0);
  return hipGetLastError();
}

}  // namespace gwi
