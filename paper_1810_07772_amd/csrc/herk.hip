// Hermitian rank-K update P(r,r') = -sum_k conj(F[k][r]) F[k][r'], K = nv*nc, with the pair
// products F[v*nc + c][r] = conj(psi_v[v][r]) psi_c[c][r] s_vc formed inside the kernel
// (Eq.(fdef) and the outer product below it, N_k = 1).
//
// Complex arithmetic on real MFMA: with f = a + ib,
//   conj(f_i) f_j = (a_i a_j + b_i b_j) + i (a_i b_j - b_i a_j),
// so the real part is a real GEMM over k' = (pair, component) of X = [a; b] with itself
// and the imaginary part is a real GEMM of X (rows) with Y = [b; -a] (columns).
//
// Work decomposition: one workgroup per lower-triangle tile (I, J) of the N_r x N_r output
// (the paper's 2-D PMatrix tiles), with 4 MFMA waves each owning a 64x64 quadrant.  The K loop
// walks occupied bands v and chunks of unoccupied bands; for each chunk the workgroup loads
// psi_c[chunk][I u J] (and psi_v[v][I u J]), forms only the f entries its tile needs (the
// paper's local-f optimisation), and stages them in LDS (double buffered, one barrier per
// stage) so the forming of stage i+1 overlaps the MFMAs of stage i.  The epilogue writes the
// tile and, off the diagonal, its conjugate transpose.
//
// Variants:
//  * FP32:  f in FP32 on v_mfma_f32_32x32x2f32.  Each occupied band's sum (nc pairs) is
//    accumulated in fresh registers and folded into a running FP32 sum (two-level sum).
//  * split BF16 / FP16: f = hi + lo (RNE), products hi*hi + hi*lo + lo*hi on
//    v_mfma_f32_32x32x16_{bf16,f16}, FP32 accumulation.  The FP16 variant multiplies each
//    band's f by 2^e_v (one exponent per occupied band) and undoes it exactly.  The default
//    split kernels are wave-specialised (herk_split_ws_kernel): separate producer waves form
//    and split f while the MFMA waves run, and the partial sums are added into P every
//    32768 pairs.
#include <utility>

#include "gw_internal.h"

namespace gwi {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int HB = 128;       // tile side
constexpr int NTHR = 256;     // 4 waves

// Map a linear block id to a lower-triangle tile so that the tiles sent to one XCD
// (blocks are dealt round-robin over the 8 XCDs) form a contiguous run of the triangle
// and share psi_c rows in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int ntiles) {
  const int q = ntiles >> 3, rem = ntiles & 7;
  const int x = b & 7, s = b >> 3;
  return x * q + min(x, rem) + s;
}

__device__ __forceinline__ void tile_of(int t, int &bi, int &bj) {
  int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  bi = i;
  bj = t - i * (i + 1) / 2;
}

__device__ __forceinline__ float2 cmul_conj(float2 v, float2 c) {   // conj(v) * c
  return make_float2(v.x * c.x + v.y * c.y, v.x * c.y - v.y * c.x);
}

// Epilogue: lane holds element (i, j) of 32x32 block (rb, cb) of its wave's quadrant in
// register e, with i = (e & 3) + 8*(e >> 2) + 4*(lane >> 5), j = lane & 31.
__device__ __forceinline__ void store_tile(float2 *__restrict__ P, int nr, int I0, int J0, bool mirror,
                                           int accumulate, const f32x16 (&re)[2][2], const f32x16 (&im)[2][2],
                                           int wr, int wc, int lane) {
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int i = (e & 3) + 8 * (e >> 2) + 4 * (lane >> 5);
        const int j = lane & 31;
        const int row = I0 + wr * 64 + rb * 32 + i;
        const int col = J0 + wc * 64 + cb * 32 + j;
        if (row < nr && col < nr) {
          const float pr = -re[rb][cb][e], pi = -im[rb][cb][e];
          float2 *d = P + (size_t)row * nr + col;
          if (accumulate) { float2 o = *d; *d = make_float2(o.x + pr, o.y + pi); }
          else *d = make_float2(pr, pi);
          if (mirror) {
            float2 *m = P + (size_t)col * nr + row;
            if (accumulate) { float2 o = *m; *m = make_float2(o.x + pr, o.y - pi); }
            else *m = make_float2(pr, -pi);
          }
        }
      }
}

// Final store after partial sums were folded into the tile: P += -acc on the tile itself, then the
// mirror (off-diagonal tiles) is written as the conjugate of the new value.
__device__ __forceinline__ void store_tile_after_folds(float2 *__restrict__ P, int nr, int I0, int J0, bool mirror,
                                                       const f32x16 (&re)[2][2], const f32x16 (&im)[2][2], int wr,
                                                       int wc, int lane) {
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int i = (e & 3) + 8 * (e >> 2) + 4 * (lane >> 5);
        const int j = lane & 31;
        const int row = I0 + wr * 64 + rb * 32 + i;
        const int col = J0 + wc * 64 + cb * 32 + j;
        if (row < nr && col < nr) {
          float2 *d = P + (size_t)row * nr + col;
          const float2 o = *d;
          const float2 v = make_float2(o.x - re[rb][cb][e], o.y - im[rb][cb][e]);
          *d = v;
          if (mirror) P[(size_t)col * nr + row] = make_float2(v.x, -v.y);
        }
      }
}

// ---------------------------------------------------------------------------------------------
// FP32 variant
// ---------------------------------------------------------------------------------------------
constexpr int KC32 = 16;   // unoccupied bands per stage

template <bool FOLD, bool COUTER>
__global__ __launch_bounds__(NTHR, 1) void herk_fp32_kernel(const float2 *__restrict__ psi_v,
                                                             const float2 *__restrict__ psi_c,
                                                             const float *__restrict__ scale, int ldsc,
                                                             float2 *__restrict__ P, int nr, int nv, int nc,
                                                             int ntiles, int accumulate) {
  // [buf][pair][component][point]; A: f on the tile's rows, B: f on its columns, Y: (im, -re) of B.
  __shared__ float sA[2][KC32][2][HB];
  __shared__ float sB[2][KC32][2][HB];
  __shared__ float sY[2][KC32][2][HB];

  int bi, bj;
  tile_of(xcd_remap(blockIdx.x, ntiles), bi, bj);
  const int I0 = bi * HB, J0 = bj * HB;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int cp = tid & 63;          // producer: grid points 2cp, 2cp+1 of the tile's rows and columns
  const int prow = wave;            // producer: pairs prow + 4*i
  const int ri = I0 + 2 * cp, rj = J0 + 2 * cp;
  const bool oki0 = ri < nr, oki1 = ri + 1 < nr, okj0 = rj < nr, okj1 = rj + 1 < nr;

  const int nchc = (nc + KC32 - 1) / KC32;
  const int nch = nv * nchc;

  float2 vI[2], vJ[2];              // psi_v of the staged chunk
  float2 cI[4][2], cJ[4][2];        // psi_c of the staged chunk
  float sc[4];

  // Stage ch covers occupied band v and unoccupied bands c0 .. c0+KC32-1.  With COUTER the
  // unoccupied chunk is the outer index and v the inner one, so the psi_c chunk stays in
  // registers for nv consecutive stages and only psi_v (one value per point) is loaded per stage.
  auto load_chunk = [&](int ch) {
    const int v = COUTER ? ch % nv : ch / nchc;
    const int c0 = (COUTER ? ch / nv : ch % nchc) * KC32;
    const float2 z = make_float2(0.f, 0.f);
    const float2 *pv = psi_v + (size_t)v * nr;
    vI[0] = oki0 ? pv[ri] : z;  vI[1] = oki1 ? pv[ri + 1] : z;
    vJ[0] = okj0 ? pv[rj] : z;  vJ[1] = okj1 ? pv[rj + 1] : z;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = c0 + prow + 4 * i;
      const bool okc = c < nc;
      sc[i] = okc ? scale[v * ldsc + c] : 0.f;
      if (!COUTER || v == 0) {
        const float2 *pc = psi_c + (size_t)(okc ? c : 0) * nr;
        cI[i][0] = (okc && oki0) ? pc[ri] : z;  cI[i][1] = (okc && oki1) ? pc[ri + 1] : z;
        cJ[i][0] = (okc && okj0) ? pc[rj] : z;  cJ[i][1] = (okc && okj1) ? pc[rj + 1] : z;
      }
    }
  };
  auto produce = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = prow + 4 * i;
      float2 fi0 = cmul_conj(vI[0], cI[i][0]), fi1 = cmul_conj(vI[1], cI[i][1]);
      float2 fj0 = cmul_conj(vJ[0], cJ[i][0]), fj1 = cmul_conj(vJ[1], cJ[i][1]);
      const float s = sc[i];
      fi0.x *= s; fi0.y *= s; fi1.x *= s; fi1.y *= s;
      fj0.x *= s; fj0.y *= s; fj1.x *= s; fj1.y *= s;
      *reinterpret_cast<float2 *>(&sA[buf][p][0][2 * cp]) = make_float2(fi0.x, fi1.x);
      *reinterpret_cast<float2 *>(&sA[buf][p][1][2 * cp]) = make_float2(fi0.y, fi1.y);
      *reinterpret_cast<float2 *>(&sB[buf][p][0][2 * cp]) = make_float2(fj0.x, fj1.x);
      *reinterpret_cast<float2 *>(&sB[buf][p][1][2 * cp]) = make_float2(fj0.y, fj1.y);
      *reinterpret_cast<float2 *>(&sY[buf][p][0][2 * cp]) = make_float2(fj0.y, fj1.y);
      *reinterpret_cast<float2 *>(&sY[buf][p][1][2 * cp]) = make_float2(-fj0.x, -fj1.x);
    }
  };

  f32x16 accR[2][2], accI[2][2];
  f32x16 runR[2][2], runI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) { accR[a][b][e] = 0.f; accI[a][b][e] = 0.f; runR[a][b][e] = 0.f; runI[a][b][e] = 0.f; }

  const int comp = lane >> 5, idx = lane & 31;
  const int ar0 = wr * 64 + idx, bc0 = wc * 64 + idx;

  load_chunk(0);
  produce(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) load_chunk(ch + 1);
#pragma unroll 4
    for (int p = 0; p < KC32; ++p) {
      const float a0 = sA[buf][p][comp][ar0], a1 = sA[buf][p][comp][ar0 + 32];
      const float x0 = sB[buf][p][comp][bc0], x1 = sB[buf][p][comp][bc0 + 32];
      const float y0 = sY[buf][p][comp][bc0], y1 = sY[buf][p][comp][bc0 + 32];
      accR[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, x0, accR[0][0], 0, 0, 0);
      accI[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, y0, accI[0][0], 0, 0, 0);
      accR[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, x1, accR[0][1], 0, 0, 0);
      accI[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, y1, accI[0][1], 0, 0, 0);
      accR[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, x0, accR[1][0], 0, 0, 0);
      accI[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, y0, accI[1][0], 0, 0, 0);
      accR[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, x1, accR[1][1], 0, 0, 0);
      accI[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, y1, accI[1][1], 0, 0, 0);
    }
    // two-level sum: fold after each block of the K loop (one occupied band, or one
    // unoccupied chunk over all occupied bands with COUTER)
    if (FOLD && (COUTER ? (ch % nv) == nv - 1 : (ch % nchc) == nchc - 1)) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          runR[a][b] += accR[a][b];
          runI[a][b] += accI[a][b];
#pragma unroll
          for (int e = 0; e < 16; ++e) { accR[a][b][e] = 0.f; accI[a][b][e] = 0.f; }
        }
    }
    if (ch + 1 < nch) produce(buf ^ 1);
    __syncthreads();
  }
  if (FOLD) {
    store_tile(P, nr, I0, J0, bi != bj, accumulate, runR, runI, wr, wc, lane);
  } else {
    store_tile(P, nr, I0, J0, bi != bj, accumulate, accR, accI, wr, wc, lane);
  }
}

// ---------------------------------------------------------------------------------------------
// Split-precision variants (BF16 or FP16 hi/lo) on v_mfma_f32_32x32x16_{bf16,f16}.
// Inside one MFMA, lane l supplies the 8 consecutive k' = 8*(l>>5) .. +7 of its row (A) or
// column (B): four pairs x (re, im).  A stage holds KS = 16 pairs = two groups of 16 k', and
// each group costs three MFMAs (hi*hi, hi*lo, lo*hi) for Re and three for Im per 32x32 block.
// LDS holds f on the tile's rows and columns as hi and lo planes; the Im operand
// Y = (im, -re) is derived in registers from the column operand (a 16-bit rotate of each
// (re, im) word and a sign flip).
// ---------------------------------------------------------------------------------------------
constexpr int KS = 16;             // pairs per stage
constexpr int SROW = 2 * KS + 8;   // narrow elements per grid-point row (padded against bank conflicts)

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <typename T> struct SplitTraits;
template <> struct SplitTraits<__bf16> {
  typedef bf16x8 vec;
  static __device__ __forceinline__ f32x16 mfma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct SplitTraits<_Float16> {
  typedef f16x8 vec;
  static __device__ __forceinline__ f32x16 mfma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// (re, im) words -> (im, -re) words: one packed 16-bit add whose operand selects swap the halves
// of w and add (0, 0x8000), which flips the sign bit of the new high half (the add wraps mod 2^16).
// The compiler writes this as a shift and an xor; the single instruction halves the VALU work of
// the MFMA waves' rotation.  It is an integer op on 16-bit lanes, not packed FP32 arithmetic.
__device__ __forceinline__ unsigned rot_word(unsigned w) {
  unsigned r;
  asm("v_pk_add_u16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1]" : "=v"(r) : "v"(w), "s"(0x80000000u));
  return r;
}
template <typename V>
__device__ __forceinline__ V rot_neg(V b) {
  u32x4 w = __builtin_bit_cast(u32x4, b);
  u32x4 y;
#pragma unroll
  for (int m = 0; m < 4; ++m) y[m] = rot_word(w[m]);
  return __builtin_bit_cast(V, y);
}

template <typename T, bool SCALED, bool COUTER>
__global__ __launch_bounds__(NTHR, 1) void herk_split_kernel(const float2 *__restrict__ psi_v,
                                                              const float2 *__restrict__ psi_c,
                                                              const float *__restrict__ scale, int ldsc,
                                                              const int *__restrict__ band_exp,
                                                              float2 *__restrict__ P, int nr, int nv, int nc,
                                                              int ntiles, int accumulate) {
  typedef typename SplitTraits<T>::vec vec;
  __shared__ __attribute__((aligned(16))) T sAh[2][HB][SROW];
  __shared__ __attribute__((aligned(16))) T sAl[2][HB][SROW];
  __shared__ __attribute__((aligned(16))) T sBh[2][HB][SROW];
  __shared__ __attribute__((aligned(16))) T sBl[2][HB][SROW];

  int bi, bj;
  tile_of(xcd_remap(blockIdx.x, ntiles), bi, bj);
  const int I0 = bi * HB, J0 = bj * HB;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;

  // Producer: waves 0 and 2 own the tile's rows, waves 1 and 3 its columns; each thread
  // owns one grid point and forms all KS pairs of the stage for it (its KS loads are
  // strided by nr, coalesced across the wave's 64 consecutive points).
  const int pside = wave & 1;
  const int ppt = lane + 64 * (wave >> 1);
  const int gpt = (pside ? J0 : I0) + ppt;
  const bool okp = gpt < nr;
  const int nchc = (nc + KS - 1) / KS;
  const int nch = nv * nchc;

  float2 pvv;
  float2 pc[KS];
  float sc[KS];
  float mul = 1.0f;

  static_assert(!(SCALED && COUTER), "the per-band scale needs the occupied band as the outer K index");
  auto load_chunk = [&](int ch) {
    const int v = COUTER ? ch % nv : ch / nchc;
    const int c0 = (COUTER ? ch / nv : ch % nchc) * KS;
    const float2 z = make_float2(0.f, 0.f);
    pvv = okp ? psi_v[(size_t)v * nr + gpt] : z;
    if (SCALED) mul = ldexpf(1.0f, band_exp[v]);
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int c = c0 + k;
      const bool okc = c < nc;
      sc[k] = okc ? scale[v * ldsc + c] : 0.f;
      if (!COUTER || v == 0) pc[k] = (okc && okp) ? psi_c[(size_t)c * nr + gpt] : z;
    }
  };
  auto produce = [&](int buf) {
    T *dh = pside ? &sBh[buf][ppt][0] : &sAh[buf][ppt][0];
    T *dl = pside ? &sBl[buf][ppt][0] : &sAl[buf][ppt][0];
#pragma unroll
    for (int g = 0; g < KS / 4; ++g) {
      vec hv, lv;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int k = 4 * g + m;
        float2 f = cmul_conj(pvv, pc[k]);
        const float s = sc[k] * mul;
        f.x *= s; f.y *= s;
        const T rh = (T)f.x, ih = (T)f.y;
        hv[2 * m] = rh;  hv[2 * m + 1] = ih;
        lv[2 * m] = (T)(f.x - (float)rh);  lv[2 * m + 1] = (T)(f.y - (float)ih);
      }
      *reinterpret_cast<vec *>(dh + 8 * g) = hv;
      *reinterpret_cast<vec *>(dl + 8 * g) = lv;
    }
  };

  f32x16 accR[2][2], accI[2][2];
  f32x16 runR[2][2], runI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        accR[a][b][e] = 0.f; accI[a][b][e] = 0.f;
        if (SCALED) { runR[a][b][e] = 0.f; runI[a][b][e] = 0.f; }
      }

  const int kq = lane >> 5, idx = lane & 31;
  const int ar0 = wr * 64 + idx, bc0 = wc * 64 + idx;

  load_chunk(0);
  produce(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) load_chunk(ch + 1);
#pragma unroll
    for (int g = 0; g < KS / 8; ++g) {
      const int ko = g * 16 + kq * 8;
      const vec ah0 = *reinterpret_cast<const vec *>(&sAh[buf][ar0][ko]);
      const vec ah1 = *reinterpret_cast<const vec *>(&sAh[buf][ar0 + 32][ko]);
      const vec al0 = *reinterpret_cast<const vec *>(&sAl[buf][ar0][ko]);
      const vec al1 = *reinterpret_cast<const vec *>(&sAl[buf][ar0 + 32][ko]);
      const vec bh0 = *reinterpret_cast<const vec *>(&sBh[buf][bc0][ko]);
      const vec bh1 = *reinterpret_cast<const vec *>(&sBh[buf][bc0 + 32][ko]);
      const vec bl0 = *reinterpret_cast<const vec *>(&sBl[buf][bc0][ko]);
      const vec bl1 = *reinterpret_cast<const vec *>(&sBl[buf][bc0 + 32][ko]);
      const vec yh0 = rot_neg(bh0), yh1 = rot_neg(bh1), yl0 = rot_neg(bl0), yl1 = rot_neg(bl1);
#define GW_SPLIT3(ACC, A_H, A_L, B_H, B_L)   \
  ACC = SplitTraits<T>::mfma(A_H, B_H, ACC); \
  ACC = SplitTraits<T>::mfma(A_H, B_L, ACC); \
  ACC = SplitTraits<T>::mfma(A_L, B_H, ACC);
      GW_SPLIT3(accR[0][0], ah0, al0, bh0, bl0)
      GW_SPLIT3(accI[0][0], ah0, al0, yh0, yl0)
      GW_SPLIT3(accR[0][1], ah0, al0, bh1, bl1)
      GW_SPLIT3(accI[0][1], ah0, al0, yh1, yl1)
      GW_SPLIT3(accR[1][0], ah1, al1, bh0, bl0)
      GW_SPLIT3(accI[1][0], ah1, al1, yh0, yl0)
      GW_SPLIT3(accR[1][1], ah1, al1, bh1, bl1)
      GW_SPLIT3(accI[1][1], ah1, al1, yh1, yl1)
#undef GW_SPLIT3
    }
    if (SCALED && (ch % nchc) == nchc - 1) {
      // end of one occupied band: fold its partial sum back with 2^(-2 e_v)
      const float back = ldexpf(1.0f, -2 * band_exp[ch / nchc]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          runR[a][b] += accR[a][b] * back;
          runI[a][b] += accI[a][b] * back;
#pragma unroll
          for (int e = 0; e < 16; ++e) { accR[a][b][e] = 0.f; accI[a][b][e] = 0.f; }
        }
    }
    if (ch + 1 < nch) produce(buf ^ 1);
    __syncthreads();
  }
  if (SCALED) store_tile(P, nr, I0, J0, bi != bj, accumulate, runR, runI, wr, wc, lane);
  else store_tile(P, nr, I0, J0, bi != bj, accumulate, accR, accI, wr, wc, lane);
}

// ---------------------------------------------------------------------------------------------
// Wave-specialised split kernel: 4 + 4 NPW waves per workgroup.  Waves 0-3 only issue MFMAs (each
// owns a 64x64 quadrant of the 128x128 tile); the other waves only form pair products, split them
// and stage them in LDS for the next stage.  Each SIMD then holds one MFMA wave and NPW producer
// waves, so the producers' VALU work runs while the matrix core executes the other wave's MFMAs.
// One wave issues a VALU instruction only every 8 or so cycles, and beside a busy matrix core one
// producer wave per SIMD does not keep up with the MFMAs; with NPW = 2 each producer takes half of
// the stage's pairs and the consumers fit their operands into the 168 registers that three waves
// per SIMD leave.  K order: unoccupied chunk outer, occupied band inner (the psi_c chunk of a
// producer thread stays in registers for nv stages).  Loads are branch-free: indices are clamped
// and the value masked.
// ---------------------------------------------------------------------------------------------
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// (a, b) -> one word holding (bf16 RNE(a), bf16 RNE(b)); gfx950 does this in one instruction.
__device__ __forceinline__ unsigned pk_bf16(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}

// hi = RNE(a, b) packed in one word, lo = RNE of the remainders, for BF16 or FP16 halves.
template <typename T> struct NarrowSplit;
template <> struct NarrowSplit<__bf16> {
  static __device__ __forceinline__ void split(float a, float b, unsigned &hi, unsigned &lo) {
    hi = pk_bf16(a, b);
    lo = pk_bf16(a - __builtin_bit_cast(float, hi << 16), b - __builtin_bit_cast(float, hi & 0xffff0000u));
  }
};
template <> struct NarrowSplit<_Float16> {
  static __device__ __forceinline__ void split(float a, float b, unsigned &hi, unsigned &lo) {
    const f32x2 v = {a, b};
    const f16x2 h = __builtin_convertvector(v, f16x2);
    const f32x2 r = {a - (float)h[0], b - (float)h[1]};
    hi = __builtin_bit_cast(unsigned, h);
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector(r, f16x2));
  }
};

// Two-level sum: every FOLD_PAIRS pairs of K the consumers add their partial sums into the tile of
// P (read-modify-write of the tile only; with accumulate set, of its mirror too) and restart from
// zero, so FP32 rounding in the accumulators grows with the block length instead of with K.  Without
// accumulate, the final store writes the mirror as the conjugate of the finished tile.
constexpr int FOLD_PAIRS = 32768;

// SCALED (FP16): band v's pair products carry 2^{e_v}, so its products carry 2^{2 e_v}.  The bands
// run in the order `order` (sorted by exponent, from launch_band_exponents), and the accumulators
// are multiplied by the exact power of two 2^{2(e_new - e_old)} whenever the exponent changes
// between stages (a few times per unoccupied chunk), and by 2^{-2 e_last} at the end: the same
// per-band scale as a fold per band, without a second accumulator set.
template <typename T, int KW, bool PRIO, bool SCALED, int NPW>
__global__ __launch_bounds__((1 + NPW) * NTHR, 1) void herk_split_ws_kernel(const float2 *__restrict__ psi_v,
                                                                     const float2 *__restrict__ psi_c,
                                                                     const float *__restrict__ scale, int ldsc,
                                                                     const int *__restrict__ band_exp,
                                                                     float2 *__restrict__ P, int nr, int nv, int nc,
                                                                     int ntiles, int accumulate) {
  typedef typename SplitTraits<T>::vec vec;
  constexpr int SRW = 2 * KW + 8;   // narrow elements per point row (padded against bank conflicts)
  __shared__ __attribute__((aligned(16))) T sAh[2][HB][SRW];
  __shared__ __attribute__((aligned(16))) T sAl[2][HB][SRW];
  __shared__ __attribute__((aligned(16))) T sBh[2][HB][SRW];
  __shared__ __attribute__((aligned(16))) T sBl[2][HB][SRW];
  // band order and sorted exponents (SCALED only): see launch_band_exponents
  const int *order = SCALED ? band_exp + nv : nullptr, *esorted = SCALED ? band_exp + 2 * nv : nullptr;

  int bi, bj;
  tile_of(xcd_remap(blockIdx.x, ntiles), bi, bj);
  const int I0 = bi * HB, J0 = bj * HB;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform role
  const int nchc = (nc + KW - 1) / KW;
  const int nch = nv * nchc;
  const bool producer = wave >= 4;

  // ---- producer state: one grid point of the rows (even pw) or columns (odd pw), and KP of the
  // stage's KW pairs starting at koff (NPW producer waves share a SIMD, each taking KW / NPW pairs)
  constexpr int KP = KW / NPW;
  const int pw = wave - 4;
  const int pside = pw & 1;
  const int ppt = lane + 64 * ((pw >> 1) & 1);
  const int koff = (pw >> 2) * KP;
  // Loads need no masks: the scale table is zero for unoccupied bands past nc (so those pair
  // products vanish), and a point past nr only feeds output entries that are never stored, so
  // out-of-range indices are clamped to valid addresses.
  const int gpt = min((pside ? J0 : I0) + ppt, nr - 1);
  float2 pc[KP], pcn[KP];
  float2 pvv;
  float sc[KP];

  auto load_c = [&](float2 (&dst)[KP], int cc) {   // psi_c of chunk cc at this thread's point
#pragma unroll
    for (int k = 0; k < KP; ++k) dst[k] = psi_c[(size_t)min(cc * KW + koff + k, nc - 1) * nr + gpt];
  };
  auto load_v = [&](int ch) {                       // psi_v and the scales of stage ch
    const int vi = ch % nv, c0 = (ch / nv) * KW;
    const int v = SCALED ? order[vi] : vi;
    pvv = psi_v[(size_t)v * nr + gpt];
    if (SCALED) {
      const float m = ldexpf(1.0f, esorted[vi]);
      pvv.x *= m;
      pvv.y *= m;
    }
    const float *srow = scale + (size_t)v * ldsc + c0 + koff;
#pragma unroll
    for (int k = 0; k < KP; ++k) sc[k] = srow[k];
  };
  auto produce = [&](int buf) {
    u32x4 *dh = reinterpret_cast<u32x4 *>(pside ? &sBh[buf][ppt][2 * koff] : &sAh[buf][ppt][2 * koff]);
    u32x4 *dl = reinterpret_cast<u32x4 *>(pside ? &sBl[buf][ppt][2 * koff] : &sAl[buf][ppt][2 * koff]);
#pragma unroll
    for (int g = 0; g < KP / 4; ++g) {
      u32x4 hv, lv;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int k = 4 * g + m;
        const float fx = (pvv.x * pc[k].x + pvv.y * pc[k].y) * sc[k];
        const float fy = (pvv.x * pc[k].y - pvv.y * pc[k].x) * sc[k];
        unsigned w, wl;
        NarrowSplit<T>::split(fx, fy, w, wl);
        hv[m] = w;
        lv[m] = wl;
      }
      dh[g] = hv;
      dl[g] = lv;
    }
  };

  // The two roles run separate loops (each wave takes one of them as a whole), so the
  // producer's registers and the consumer's accumulators are never live at the same time.
  // Both loops pass the same number of workgroup barriers.
  if (producer) {
    load_c(pc, 0);
    load_v(0);
    produce(0);
    if (nch > 1) load_v(1);
    if (nv == 1 && nch > 1) load_c(pcn, 1);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
      if (ch + 1 < nch) {
        if ((ch + 1) % nv == 0) {                          // stage ch+1 opens the next unoccupied chunk
#pragma unroll
          for (int k = 0; k < KP; ++k) pc[k] = pcn[k];
        }
        produce((ch & 1) ^ 1);
        if (ch + 2 < nch) {
          load_v(ch + 2);                                  // in flight until the next stage
          if ((ch + 2) % nv == 0) load_c(pcn, (ch + 2) / nv);
        }
      }
      __syncthreads();
    }
    return;
  }

  // ---- consumer
  if (PRIO) __builtin_amdgcn_s_setprio(2);   // favour the MFMA waves when both roles can issue
  const int wr = (wave & 3) >> 1, wc = wave & 1;
  const int kq = lane >> 5, idx = lane & 31;
  const int ar0 = wr * 64 + idx, bc0 = wc * 64 + idx;
  f32x16 accR[2][2], accI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) { accR[a][b][e] = 0.f; accI[a][b][e] = 0.f; }
  // accumulators carry 2^{2e}: back to the true scale
  auto unscale = [&](int e) {
    const float f = ldexpf(1.0f, -2 * e);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        accR[a][b] *= f;
        accI[a][b] *= f;
      }
  };
  constexpr int FOLD_STAGES = FOLD_PAIRS / KW;
  int nfold = 0;
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (SCALED && ch > 0 && (ch % FOLD_STAGES) != 0) {
      const int vi = ch % nv;
      const int d = esorted[vi] - esorted[vi == 0 ? nv - 1 : vi - 1];
      if (d != 0) {                                        // uniform: every lane reads the same exponents
        const float f = ldexpf(1.0f, 2 * d);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            accR[a][b] *= f;
            accI[a][b] *= f;
          }
      }
    }
#pragma unroll
    for (int g = 0; g < KW / 8; ++g) {
      const int ko = g * 16 + kq * 8;
      if (NPW == 1) {
        const vec ah0 = *reinterpret_cast<const vec *>(&sAh[buf][ar0][ko]);
        const vec ah1 = *reinterpret_cast<const vec *>(&sAh[buf][ar0 + 32][ko]);
        const vec al0 = *reinterpret_cast<const vec *>(&sAl[buf][ar0][ko]);
        const vec al1 = *reinterpret_cast<const vec *>(&sAl[buf][ar0 + 32][ko]);
        const vec bh0 = *reinterpret_cast<const vec *>(&sBh[buf][bc0][ko]);
        const vec bh1 = *reinterpret_cast<const vec *>(&sBh[buf][bc0 + 32][ko]);
        const vec bl0 = *reinterpret_cast<const vec *>(&sBl[buf][bc0][ko]);
        const vec bl1 = *reinterpret_cast<const vec *>(&sBl[buf][bc0 + 32][ko]);
        const vec yh0 = rot_neg(bh0), yh1 = rot_neg(bh1), yl0 = rot_neg(bl0), yl1 = rot_neg(bl1);
        // eight independent accumulators per product, so consecutive MFMAs never chain
#define GW_PROD8(A0, A1, B0, B1, Y0, Y1)                          \
  accR[0][0] = SplitTraits<T>::mfma(A0, B0, accR[0][0]);           \
  accI[0][0] = SplitTraits<T>::mfma(A0, Y0, accI[0][0]);           \
  accR[0][1] = SplitTraits<T>::mfma(A0, B1, accR[0][1]);           \
  accI[0][1] = SplitTraits<T>::mfma(A0, Y1, accI[0][1]);           \
  accR[1][0] = SplitTraits<T>::mfma(A1, B0, accR[1][0]);           \
  accI[1][0] = SplitTraits<T>::mfma(A1, Y0, accI[1][0]);           \
  accR[1][1] = SplitTraits<T>::mfma(A1, B1, accR[1][1]);           \
  accI[1][1] = SplitTraits<T>::mfma(A1, Y1, accI[1][1]);
        GW_PROD8(ah0, ah1, bh0, bh1, yh0, yh1)     // hi * hi
        GW_PROD8(ah0, ah1, bl0, bl1, yl0, yl1)     // hi * lo
        GW_PROD8(al0, al1, bh0, bh1, yh0, yh1)     // lo * hi
#undef GW_PROD8
      } else {
        // three waves share the SIMD, so at most 168 registers: the products run in an order
        // that keeps three operand pairs live (real parts, then the rotated B in place for the
        // imaginary parts, and B's lo half last)
#define GW_PROD4(ACC, A0, A1, B0, B1)                        \
  ACC[0][0] = SplitTraits<T>::mfma(A0, B0, ACC[0][0]);        \
  ACC[0][1] = SplitTraits<T>::mfma(A0, B1, ACC[0][1]);        \
  ACC[1][0] = SplitTraits<T>::mfma(A1, B0, ACC[1][0]);        \
  ACC[1][1] = SplitTraits<T>::mfma(A1, B1, ACC[1][1]);
        const vec ah0 = *reinterpret_cast<const vec *>(&sAh[buf][ar0][ko]);
        const vec ah1 = *reinterpret_cast<const vec *>(&sAh[buf][ar0 + 32][ko]);
        vec b0 = *reinterpret_cast<const vec *>(&sBh[buf][bc0][ko]);
        vec b1 = *reinterpret_cast<const vec *>(&sBh[buf][bc0 + 32][ko]);
        GW_PROD4(accR, ah0, ah1, b0, b1)           // hi * hi
        {
          const vec al0 = *reinterpret_cast<const vec *>(&sAl[buf][ar0][ko]);
          const vec al1 = *reinterpret_cast<const vec *>(&sAl[buf][ar0 + 32][ko]);
          GW_PROD4(accR, al0, al1, b0, b1)         // lo * hi
          b0 = rot_neg(b0);
          b1 = rot_neg(b1);
          GW_PROD4(accI, ah0, ah1, b0, b1)
          GW_PROD4(accI, al0, al1, b0, b1)
        }
        b0 = *reinterpret_cast<const vec *>(&sBl[buf][bc0][ko]);
        b1 = *reinterpret_cast<const vec *>(&sBl[buf][bc0 + 32][ko]);
        GW_PROD4(accR, ah0, ah1, b0, b1)           // hi * lo
        b0 = rot_neg(b0);
        b1 = rot_neg(b1);
        GW_PROD4(accI, ah0, ah1, b0, b1)
#undef GW_PROD4
      }
    }
    if ((ch + 1) % FOLD_STAGES == 0 && ch + 1 < nch) {
      // two-level sum: this block's partial goes into the tile, the accumulators restart from zero
      if (SCALED) unscale(esorted[ch % nv]);
      // the store addresses do not change between folds; hide that from the compiler, or it keeps
      // all of them live across the loop and spills
      int lane_f = lane;
      asm volatile("" : "+v"(lane_f));
      // the tile only (its mirror is written once at the end), unless accumulating into P
      store_tile(P, nr, I0, J0, accumulate && bi != bj, accumulate || nfold > 0, accR, accI, wr, wc, lane_f);
      ++nfold;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int e = 0; e < 16; ++e) { accR[a][b][e] = 0.f; accI[a][b][e] = 0.f; }
    }
    __syncthreads();
  }
  if (SCALED) unscale(esorted[(nch - 1) % nv]);
  if (nfold == 0 || accumulate) store_tile(P, nr, I0, J0, bi != bj, accumulate || nfold > 0, accR, accI, wr, wc, lane);
  else store_tile_after_folds(P, nr, I0, J0, bi != bj, accR, accI, wr, wc, lane);
}

// ---------------------------------------------------------------------------------------------
// Wide wave-specialised split kernel: a 128 x 256 output block per workgroup (one 128-row block I and
// the two 128-column blocks 2 jp, 2 jp + 1), twelve waves.  Waves 0-7 issue the MFMAs, two per SIMD,
// each on a 64 x 64 quadrant (row half w >> 2, column quarter w & 3); waves 8-11, one per SIMD, form
// and split the pair products of the block's 384 points (128 rows, 256 columns) for the next stage of
// WK = 16 pairs.  Per stage the producers form 384 x 16 pair products for 384 MFMAs, 3 VALU instructions
// per MFMA against 4 for the 128 x 128 block, where the 256 points' 32 pairs feed as many MFMAs.
// Producer work: unit u = lane + 256 j (j < 3) of the 768 (point, half of the stage's pairs) units;
// point u % 384, pairs 8 (u / 384) .. +7, so each lane keeps 3 x 8 psi_c values for the nv stages of an
// unoccupied chunk, and the half (hence the scale row) is uniform across each wave.
// A block whose second column block lies above the diagonal (I even, jp = I / 2) leaves it unused.
// ---------------------------------------------------------------------------------------------
constexpr int WK = 16;                 // pairs per stage
constexpr int WPTS = 3 * HB;           // points of a block: 128 rows + 256 columns

// block t of the row-major enumeration of (I, jp) with 0 <= jp <= I / 2: row I holds I / 2 + 1 blocks,
// so the rows before I = 2m hold m (m + 1) blocks and those before I = 2m + 1 hold (m + 1)^2
__device__ __forceinline__ void wide_block_of(int t, int &bi, int &jp) {
  int m = (int)sqrtf((float)t);                 // candidate: rows before 2m + 1 hold (m + 1)^2 > t
  while ((m + 1) * (m + 1) <= t) ++m;
  while (m > 0 && m * m > t) --m;
  // now m^2 <= t < (m + 1)^2: I is 2m - 1 (if t < m (m + 1)... measured from the row starts below)
  const int start_even = m * (m + 1), start_odd = (m + 1) * (m + 1);   // first blocks of rows 2m, 2m + 1
  if (t >= start_odd) { bi = 2 * m + 1; jp = t - start_odd; }
  else if (t >= start_even) { bi = 2 * m; jp = t - start_even; }
  else { bi = 2 * m - 1; jp = t - m * m; }        // row 2m - 1 starts at m^2
}

int wide_block_count(int nb) {                   // blocks over row blocks 0 .. nb-1
  const int m = nb / 2;
  return (nb & 1) ? (m + 1) * (m + 1) : m * (m + 1);
}

template <typename T, bool SCALED>
__global__ __launch_bounds__(3 * NTHR, 1) void herk_split_wide_kernel(const float2 *__restrict__ psi_v,
                                                                      const float2 *__restrict__ psi_c,
                                                                      const float *__restrict__ scale, int ldsc,
                                                                      const int *__restrict__ band_exp,
                                                                      float2 *__restrict__ P, int nr, int nv, int nc,
                                                                      int nblocks, int accumulate) {
  typedef typename SplitTraits<T>::vec vec;
  constexpr int SRW = 2 * WK + 8;   // narrow elements per point row (padded against bank conflicts)
  __shared__ __attribute__((aligned(16))) T sH[2][WPTS][SRW];
  __shared__ __attribute__((aligned(16))) T sL[2][WPTS][SRW];
  const int *order = SCALED ? band_exp + nv : nullptr, *esorted = SCALED ? band_exp + 2 * nv : nullptr;

  int bi, jp;
  wide_block_of(xcd_remap(blockIdx.x, nblocks), bi, jp);
  const int I0 = bi * HB, J0 = 2 * jp * HB;
  const int ncb = (2 * jp + 1 <= bi) ? 2 : 1;          // column blocks of the pair on or below the diagonal
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nchc = (nc + WK - 1) / WK;
  const int nch = nv * nchc;

  if (wave >= 8) {
    // ---- producers
    const int pw = wave - 8;
    int gpt[3], half[3], row[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int u = lane + 64 * pw + 256 * j;
      const int pt = u % WPTS;
      // 64 pw + 256 j never straddles a multiple of 384 within a wave, so the half is wave-uniform
      half[j] = __builtin_amdgcn_readfirstlane((64 * pw + 256 * j) / WPTS);
      row[j] = pt;
      // points past nr only feed outputs that are never stored: clamp the address
      gpt[j] = min(pt < HB ? I0 + pt : J0 + (pt - HB), nr - 1);
    }
    float2 pc[3][8], pcn[3][8], pvv[3];
    float sc[3][8];                                        // the scale row of each unit's half
    auto load_c = [&](float2 (&dst)[3][8], int cc) {
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < 8; ++k)
          dst[j][k] = psi_c[(size_t)min(cc * WK + 8 * half[j] + k, nc - 1) * nr + gpt[j]];
    };
    auto load_v = [&](int vi, int c0) {                    // psi_v and the scales of stage (vi, c0)
      const int v = SCALED ? order[vi] : vi;
#pragma unroll
      for (int j = 0; j < 3; ++j) pvv[j] = psi_v[(size_t)v * nr + gpt[j]];
      if (SCALED) {
        const float m = ldexpf(1.0f, esorted[vi]);
#pragma unroll
        for (int j = 0; j < 3; ++j) { pvv[j].x *= m; pvv[j].y *= m; }
      }
      const float *srow = scale + (size_t)v * ldsc + c0;     // zero past nc: those pair products vanish
      // per unit, at a wave-uniform offset, so that the multiplies take the scale straight from a scalar
      // register (a select between the two halves' rows cost three VALU instructions per pair)
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < 8; ++k) sc[j][k] = srow[8 * half[j] + k];
    };
    auto produce = [&](int buf) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        u32x4 *dh = reinterpret_cast<u32x4 *>(&sH[buf][row[j]][16 * half[j]]);
        u32x4 *dl = reinterpret_cast<u32x4 *>(&sL[buf][row[j]][16 * half[j]]);
        const float *s8 = sc[j];
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          u32x4 hv, lv;
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int k = 4 * g + m;
            const float fx = (pvv[j].x * pc[j][k].x + pvv[j].y * pc[j][k].y) * s8[k];
            const float fy = (pvv[j].x * pc[j][k].y - pvv[j].y * pc[j][k].x) * s8[k];
            unsigned w, wl;
            NarrowSplit<T>::split(fx, fy, w, wl);
            hv[m] = w;
            lv[m] = wl;
          }
          dh[g] = hv;
          dl[g] = lv;
        }
      }
    };
    // stage ch is (occupied band ch % nv, unoccupied chunk ch / nv); the stage indices ahead of the loop
    // advance by counters, not by a division per stage (a lone producer wave per SIMD issues close to
    // its limit, so its scalar work counts too)
    int v1 = 1 % nv, v2 = 2 % nv, c2 = 2 / nv;             // stages ch + 1 and ch + 2
    load_c(pc, 0);
    load_v(0, 0);
    produce(0);
    if (nch > 1) load_v(v1, (1 / nv) * WK);
    if (nv == 1 && nch > 1) load_c(pcn, 1);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
      if (ch + 1 < nch) {
        if (v1 == 0) {                                     // stage ch+1 opens the next unoccupied chunk
#pragma unroll
          for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 8; ++k) pc[j][k] = pcn[j][k];
        }
        produce((ch & 1) ^ 1);
        if (ch + 2 < nch) {
          load_v(v2, c2 * WK);
          if (v2 == 0) load_c(pcn, c2);
        }
      }
      v1 = v1 + 1 == nv ? 0 : v1 + 1;
      if (++v2 == nv) { v2 = 0; ++c2; }
      __syncthreads();
    }
    return;
  }

  // ---- consumers: quadrant rows I0 + 64 wr, columns J0 + 64 wc
  const int wr = wave >> 2, wc = wave & 3;
  const bool active = (wc >> 1) < ncb;                     // wave-uniform: this quadrant is on or below the diagonal
  const int kq = lane >> 5, idx = lane & 31;
  const int ar0 = wr * 64 + idx, bc0 = HB + wc * 64 + idx;  // LDS rows of the A and B operands
  f32x16 accR[2][2], accI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) { accR[a][b][e] = 0.f; accI[a][b][e] = 0.f; }
  auto unscale = [&](int e) {
    const float f = ldexpf(1.0f, -2 * e);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        accR[a][b] *= f;
        accI[a][b] *= f;
      }
  };
  constexpr int FOLD_STAGES = FOLD_PAIRS / WK;
  const int mrow = bi, mcol = 2 * jp + (wc >> 1);          // 128-blocks of this quadrant
  const bool mirror_q = mcol != mrow;
  int nfold = 0;
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (active) {
      if (SCALED && ch > 0 && (ch % FOLD_STAGES) != 0) {
        const int vi = ch % nv;
        const int d = esorted[vi] - esorted[vi == 0 ? nv - 1 : vi - 1];
        if (d != 0) {
          const float f = ldexpf(1.0f, 2 * d);
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              accR[a][b] *= f;
              accI[a][b] *= f;
            }
        }
      }
#pragma unroll
      for (int g = 0; g < WK / 8; ++g) {
        const int ko = g * 16 + kq * 8;
#define GW_PROD4(ACC, A0, A1, B0, B1)                        \
  ACC[0][0] = SplitTraits<T>::mfma(A0, B0, ACC[0][0]);        \
  ACC[0][1] = SplitTraits<T>::mfma(A0, B1, ACC[0][1]);        \
  ACC[1][0] = SplitTraits<T>::mfma(A1, B0, ACC[1][0]);        \
  ACC[1][1] = SplitTraits<T>::mfma(A1, B1, ACC[1][1]);
        const vec ah0 = *reinterpret_cast<const vec *>(&sH[buf][ar0][ko]);
        const vec ah1 = *reinterpret_cast<const vec *>(&sH[buf][ar0 + 32][ko]);
        vec b0 = *reinterpret_cast<const vec *>(&sH[buf][bc0][ko]);
        vec b1 = *reinterpret_cast<const vec *>(&sH[buf][bc0 + 32][ko]);
        GW_PROD4(accR, ah0, ah1, b0, b1)           // hi * hi
        {
          const vec al0 = *reinterpret_cast<const vec *>(&sL[buf][ar0][ko]);
          const vec al1 = *reinterpret_cast<const vec *>(&sL[buf][ar0 + 32][ko]);
          GW_PROD4(accR, al0, al1, b0, b1)         // lo * hi
          b0 = rot_neg(b0);
          b1 = rot_neg(b1);
          GW_PROD4(accI, ah0, ah1, b0, b1)
          GW_PROD4(accI, al0, al1, b0, b1)
        }
        b0 = *reinterpret_cast<const vec *>(&sL[buf][bc0][ko]);
        b1 = *reinterpret_cast<const vec *>(&sL[buf][bc0 + 32][ko]);
        GW_PROD4(accR, ah0, ah1, b0, b1)           // hi * lo
        b0 = rot_neg(b0);
        b1 = rot_neg(b1);
        GW_PROD4(accI, ah0, ah1, b0, b1)
#undef GW_PROD4
      }
      if ((ch + 1) % FOLD_STAGES == 0 && ch + 1 < nch) {
        if (SCALED) unscale(esorted[ch % nv]);
        int lane_f = lane;
        asm volatile("" : "+v"(lane_f));
        store_tile(P, nr, I0, J0, accumulate && mirror_q, accumulate || nfold > 0, accR, accI, wr, wc, lane_f);
        ++nfold;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 16; ++e) { accR[a][b][e] = 0.f; accI[a][b][e] = 0.f; }
      }
    }
    __syncthreads();
  }
  if (!active) return;
  if (SCALED) unscale(esorted[(nch - 1) % nv]);
  if (nfold == 0 || accumulate) store_tile(P, nr, I0, J0, mirror_q, accumulate || nfold > 0, accR, accI, wr, wc, lane);
  else store_tile_after_folds(P, nr, I0, J0, mirror_q, accR, accI, wr, wc, lane);
}

// ---------------------------------------------------------------------------------------------
// Planar wide kernel: the wide kernel's 128 x 256 block and twelve waves, with each stage's pair
// products stored planar so that the MFMA waves spend no VALU work on their operands.  Within a group
// of four pairs (one MFMA lane's K slice of eight narrow values) a point holds [Re f x 4, Im f x 4].
// The real part of an output entry is then dot(A, B) over the slices, and the imaginary part the
// accumulators carry, ar.bi - ai.br, is dot(A', B) with A' = [-Im f, Re f]: the producers store A'
// beside A for the 128 row points (row words [Re, Im, -Im, Re] per group), and the 256 column points
// need no second copy.  The row side also carries the whole pair weight s^2 = p / (E_c - E_v) and the
// column side none, P(r, r') = sum s^2 g(r) conj(g(r')) with g = conj(psi_v) psi_c, the same sum as
// f(r) conj(f(r')) with two multiplies fewer per column entry; the FP16 instance scales the two sides
// by 2^{e_v -+ shift_v} (launch_band_exponents), which keeps both in range.
// Per thread and stage a producer forms one row point's 8 pairs (its half of the stage) and one
// column point's 16 pairs.
// ---------------------------------------------------------------------------------------------
constexpr int PW_RW = 36;   // 32-bit words per row point and buffer: 4 groups x 8 words, 4 words of padding
constexpr int PW_CW = 20;   // per column point: 4 groups x [Re, Im] (4 words), 4 words of padding
constexpr unsigned PW_SIGNS = 0x80008000u;   // the sign bits of both narrow halves of a word

template <typename T, bool SCALED>
__global__ __launch_bounds__(3 * NTHR, 1) void herk_split_wide_planar_kernel(
    const float2 *__restrict__ psi_v, const float2 *__restrict__ psi_c, const float *__restrict__ scale, int ldsc,
    const int *__restrict__ band_exp, float2 *__restrict__ P, int nr, int nv, int nc, int nblocks, int accumulate) {
  typedef typename SplitTraits<T>::vec vec;
  __shared__ __attribute__((aligned(16))) unsigned sRH[2][HB][PW_RW];
  __shared__ __attribute__((aligned(16))) unsigned sRL[2][HB][PW_RW];
  __shared__ __attribute__((aligned(16))) unsigned sCH[2][2 * HB][PW_CW];
  __shared__ __attribute__((aligned(16))) unsigned sCL[2][2 * HB][PW_CW];
  const int *order = SCALED ? band_exp + nv : nullptr, *esorted = SCALED ? band_exp + 2 * nv : nullptr;
  const int *bshift = SCALED ? band_exp + 4 * nv + nc : nullptr;

  int bi, jp;
  wide_block_of(xcd_remap(blockIdx.x, nblocks), bi, jp);
  const int I0 = bi * HB, J0 = 2 * jp * HB;
  const int ncb = (2 * jp + 1 <= bi) ? 2 : 1;          // column blocks of the pair on or below the diagonal
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nchc = (nc + WK - 1) / WK;
  const int nch = nv * nchc;

  if (wave >= 8) {
    // ---- producers: row point rpt (pairs 8 rh .. 8 rh + 7 of each stage), column point cpt (all 16)
    const int pw = wave - 8;
    const int rpt = lane + 64 * (pw & 1), rh = pw >> 1, cpt = lane + 64 * pw;
    // points past nr only feed outputs that are never stored: clamp the address
    const int grow = min(I0 + rpt, nr - 1), gcol = min(J0 + cpt, nr - 1);
    float2 rc[8], rcn[8], cc[16], ccn[16], pvr, pvc;
    float sr[8];
    auto load_c = [&](float2 (&rd)[8], float2 (&cd)[16], int chunk) {
#pragma unroll
      for (int k = 0; k < 8; ++k) rd[k] = psi_c[(size_t)min(chunk * WK + 8 * rh + k, nc - 1) * nr + grow];
#pragma unroll
      for (int k = 0; k < 16; ++k) cd[k] = psi_c[(size_t)min(chunk * WK + k, nc - 1) * nr + gcol];
    };
    auto load_v = [&](int vi, int c0) {                    // psi_v and the weights of stage (vi, c0)
      const int v = SCALED ? order[vi] : vi;
      pvr = psi_v[(size_t)v * nr + grow];
      pvc = psi_v[(size_t)v * nr + gcol];
      if (SCALED) {                         // rows 2^{e - shift}, columns 2^{e + shift}
        const float mr = ldexpf(1.0f, esorted[vi] - bshift[v]), mc = ldexpf(1.0f, esorted[vi] + bshift[v]);
        pvr.x *= mr; pvr.y *= mr; pvc.x *= mc; pvc.y *= mc;
      }
      // the s^2 table (wave-uniform offsets: scalar loads); zero past nc, so those pairs vanish
      const float *srow = scale + (size_t)nv * ldsc + (size_t)v * ldsc + c0;
#pragma unroll
      for (int k = 0; k < 8; ++k) sr[k] = srow[8 * rh + k];
    };
    auto produce = [&](int buf) {
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        float fx[4], fy[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int k = 4 * g + m;
          fx[m] = (pvr.x * rc[k].x + pvr.y * rc[k].y) * sr[k];
          fy[m] = (pvr.x * rc[k].y - pvr.y * rc[k].x) * sr[k];
        }
        unsigned h[4], l[4];
        NarrowSplit<T>::split(fx[0], fx[1], h[0], l[0]);
        NarrowSplit<T>::split(fx[2], fx[3], h[1], l[1]);
        NarrowSplit<T>::split(fy[0], fy[1], h[2], l[2]);
        NarrowSplit<T>::split(fy[2], fy[3], h[3], l[3]);
        u32x4 *dh = reinterpret_cast<u32x4 *>(&sRH[buf][rpt][8 * (2 * rh + g)]);
        u32x4 *dl = reinterpret_cast<u32x4 *>(&sRL[buf][rpt][8 * (2 * rh + g)]);
        dh[0] = u32x4{h[0], h[1], h[2], h[3]};
        dl[0] = u32x4{l[0], l[1], l[2], l[3]};
        // [-Im, Re] as two 8-byte LDS stores, the second from the registers just stored: one 16-byte store
        // would need [-Im, Re] in four consecutive registers, i.e. eight moves per stage.  The stores are
        // volatile only so that they are not merged back into that 16-byte form.
        typedef __attribute__((address_space(3))) volatile u32x2 lds_u32x2;
        lds_u32x2 *eh = (lds_u32x2 *)(dh + 1), *el = (lds_u32x2 *)(dl + 1);
        eh[0] = u32x2{h[2] ^ PW_SIGNS, h[3] ^ PW_SIGNS};
        eh[1] = u32x2{h[0], h[1]};
        el[0] = u32x2{l[2] ^ PW_SIGNS, l[3] ^ PW_SIGNS};
        el[1] = u32x2{l[0], l[1]};
      }
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        float fx[4], fy[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int k = 4 * g + m;
          fx[m] = pvc.x * cc[k].x + pvc.y * cc[k].y;
          fy[m] = pvc.x * cc[k].y - pvc.y * cc[k].x;
        }
        unsigned h[4], l[4];
        NarrowSplit<T>::split(fx[0], fx[1], h[0], l[0]);
        NarrowSplit<T>::split(fx[2], fx[3], h[1], l[1]);
        NarrowSplit<T>::split(fy[0], fy[1], h[2], l[2]);
        NarrowSplit<T>::split(fy[2], fy[3], h[3], l[3]);
        *reinterpret_cast<u32x4 *>(&sCH[buf][cpt][4 * g]) = u32x4{h[0], h[1], h[2], h[3]};
        *reinterpret_cast<u32x4 *>(&sCL[buf][cpt][4 * g]) = u32x4{l[0], l[1], l[2], l[3]};
      }
    };
    // stage ch is (occupied band ch % nv, unoccupied chunk ch / nv); the indices of stages ch + 1 and
    // ch + 2 advance by counters
    int v1 = 1 % nv, v2 = 2 % nv, c2 = 2 / nv;
    load_c(rc, cc, 0);
    load_v(0, 0);
    produce(0);
    if (nch > 1) load_v(v1, (1 / nv) * WK);
    if (nv == 1 && nch > 1) load_c(rcn, ccn, 1);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
      if (ch + 1 < nch) {
        if (v1 == 0) {                                     // stage ch+1 opens the next unoccupied chunk
#pragma unroll
          for (int k = 0; k < 8; ++k) rc[k] = rcn[k];
#pragma unroll
          for (int k = 0; k < 16; ++k) cc[k] = ccn[k];
        }
        produce((ch & 1) ^ 1);
        if (ch + 2 < nch) {
          load_v(v2, c2 * WK);
          if (v2 == 0) load_c(rcn, ccn, c2);
        }
      }
      v1 = v1 + 1 == nv ? 0 : v1 + 1;
      if (++v2 == nv) { v2 = 0; ++c2; }
      __syncthreads();
    }
    return;
  }

  // ---- consumers: quadrant rows I0 + 64 wr, columns J0 + 64 wc.  They issue at the highest wave priority,
  // so that an MFMA ready beside a producer's VALU instruction goes first: 0.2% shorter launches on one
  // machine, against 2.8% longer with the producers preferred instead.
  __builtin_amdgcn_s_setprio(3);
  const int wr = wave >> 2, wc = wave & 3;
  const bool active = (wc >> 1) < ncb;                     // wave-uniform: this quadrant is on or below the diagonal
  const int kq = lane >> 5, idx = lane & 31;
  const int ar0 = wr * 64 + idx, bc0 = wc * 64 + idx;      // LDS rows of the A and B operands
  f32x16 accR[2][2], accI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) { accR[a][b][e] = 0.f; accI[a][b][e] = 0.f; }
  auto unscale = [&](int e) {
    const float f = ldexpf(1.0f, -2 * e);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        accR[a][b] *= f;
        accI[a][b] *= f;
      }
  };
  constexpr int FOLD_STAGES = FOLD_PAIRS / WK;
  const int mrow = bi, mcol = 2 * jp + (wc >> 1);          // 128-blocks of this quadrant
  const bool mirror_q = mcol != mrow;
  int nfold = 0;
  // one stage per call; the buffer index is a constant of each copy, so the LDS addresses are immediates
  auto stage = [&](int ch, auto bufc) {
    constexpr int buf = decltype(bufc)::value;
    if (active) {
      if (SCALED && ch > 0 && (ch % FOLD_STAGES) != 0) {
        const int vi = ch % nv;
        const int d = esorted[vi] - esorted[vi == 0 ? nv - 1 : vi - 1];
        if (d != 0) {
          const float f = ldexpf(1.0f, 2 * d);
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              accR[a][b] *= f;
              accI[a][b] *= f;
            }
        }
      }
#pragma unroll
      for (int g = 0; g < WK / 8; ++g) {
        const int ao = 8 * (2 * g + kq), bo = 4 * (2 * g + kq);   // this lane half's group of four pairs
#define GW_PROD4(ACC, A0, A1, B0, B1)                        \
  ACC[0][0] = SplitTraits<T>::mfma(A0, B0, ACC[0][0]);        \
  ACC[0][1] = SplitTraits<T>::mfma(A0, B1, ACC[0][1]);        \
  ACC[1][0] = SplitTraits<T>::mfma(A1, B0, ACC[1][0]);        \
  ACC[1][1] = SplitTraits<T>::mfma(A1, B1, ACC[1][1]);
        // at most three operand pairs live: A hi, B hi and one of A lo, A' lo, A' hi; then B lo
        const vec ah0 = *reinterpret_cast<const vec *>(&sRH[buf][ar0][ao]);
        const vec ah1 = *reinterpret_cast<const vec *>(&sRH[buf][ar0 + 32][ao]);
        vec b0 = *reinterpret_cast<const vec *>(&sCH[buf][bc0][bo]);
        vec b1 = *reinterpret_cast<const vec *>(&sCH[buf][bc0 + 32][bo]);
        GW_PROD4(accR, ah0, ah1, b0, b1)           // hi * hi
        {
          const vec al0 = *reinterpret_cast<const vec *>(&sRL[buf][ar0][ao]);
          const vec al1 = *reinterpret_cast<const vec *>(&sRL[buf][ar0 + 32][ao]);
          GW_PROD4(accR, al0, al1, b0, b1)         // lo * hi
        }
        {
          const vec xl0 = *reinterpret_cast<const vec *>(&sRL[buf][ar0][ao + 4]);
          const vec xl1 = *reinterpret_cast<const vec *>(&sRL[buf][ar0 + 32][ao + 4]);
          GW_PROD4(accI, xl0, xl1, b0, b1)         // lo' * hi
        }
        const vec xh0 = *reinterpret_cast<const vec *>(&sRH[buf][ar0][ao + 4]);
        const vec xh1 = *reinterpret_cast<const vec *>(&sRH[buf][ar0 + 32][ao + 4]);
        GW_PROD4(accI, xh0, xh1, b0, b1)           // hi' * hi
        b0 = *reinterpret_cast<const vec *>(&sCL[buf][bc0][bo]);
        b1 = *reinterpret_cast<const vec *>(&sCL[buf][bc0 + 32][bo]);
        GW_PROD4(accR, ah0, ah1, b0, b1)           // hi * lo
        GW_PROD4(accI, xh0, xh1, b0, b1)           // hi' * lo
#undef GW_PROD4
      }
      // FOLD_STAGES is even, so a fold follows only odd stages, which use buffer 1
      if (buf == 1 && (ch + 1) % FOLD_STAGES == 0 && ch + 1 < nch) {
        if (SCALED) unscale(esorted[ch % nv]);
        int lane_f = lane;
        asm volatile("" : "+v"(lane_f));
        store_tile(P, nr, I0, J0, accumulate && mirror_q, accumulate || nfold > 0, accR, accI, wr, wc, lane_f);
        ++nfold;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 16; ++e) { accR[a][b][e] = 0.f; accI[a][b][e] = 0.f; }
      }
    }
    __syncthreads();
  };
  static_assert(FOLD_STAGES % 2 == 0, "folds must follow odd stages");
  __syncthreads();
  int ch = 0;
  for (; ch + 1 < nch; ch += 2) {
    stage(ch, std::integral_constant<int, 0>{});
    stage(ch + 1, std::integral_constant<int, 1>{});
  }
  if (ch < nch) stage(ch, std::integral_constant<int, 0>{});
  if (!active) return;
  if (SCALED) unscale(esorted[(nch - 1) % nv]);
  if (nfold == 0 || accumulate) store_tile(P, nr, I0, J0, mirror_q, accumulate || nfold > 0, accR, accI, wr, wc, lane);
  else store_tile_after_folds(P, nr, I0, J0, mirror_q, accR, accI, wr, wc, lane);
}

// ---------------------------------------------------------------------------------------------
// Per-band exponents of the FP16 path: e_v = floor(log2(2^14 / bound_v)) with
// bound_v = max_r |psi_v(r)| * max_{c,r} |psi_c(r)| * max_c s_vc >= max |f_vc(r)|, so the
// scaled f of band v stays below 2^14 (FP16 max 65504) and its lo part stays normal for
// every entry within 2^-10 of the band's largest.
// ---------------------------------------------------------------------------------------------
__global__ void absmax_rows_kernel(const float2 *__restrict__ psi, int nrows, int nr, float *__restrict__ out) {
  const int row = blockIdx.x;
  float m = 0.f;
  for (int r = threadIdx.x; r < nr; r += blockDim.x) {
    const float2 z = psi[(size_t)row * nr + r];
    m = fmaxf(m, sqrtf(z.x * z.x + z.y * z.y));
  }
  __shared__ float red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[row] = red[0];
}

// shift[v] = floor(log2(max_c s_vc)): the planar kernel carries the whole weight s^2 on its row side and
// none on its column side, and scales them by 2^{e_v - shift_v} and 2^{e_v + shift_v}, so both stay
// within a factor 2 of the bound above (below 2^15) and their product keeps the factor 2^{2 e_v}.
__global__ void band_exponent_kernel(const float *__restrict__ vmax, int nv, const float *__restrict__ cmax, int nc,
                                     const float *__restrict__ scale, int ldsc, int *__restrict__ band_exp,
                                     int *__restrict__ shift) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  float cm = 0.f, sm = 0.f;
  for (int c = 0; c < nc; ++c) { cm = fmaxf(cm, cmax[c]); sm = fmaxf(sm, scale[v * ldsc + c]); }
  const float bound = vmax[v] * cm * sm;
  int e = 0;
  if (bound > 0.f) e = (int)floorf(log2f(16384.0f / bound));
  band_exp[v] = max(-60, min(60, e));
  shift[v] = sm > 0.f ? max(-30, min(30, (int)floorf(log2f(sm)))) : 0;
}

// Bands ordered by exponent (a stable counting sort over the clamped range [-60, 60], one thread):
// order[k] is the k-th band, es[k] its exponent.
__global__ void band_order_kernel(const int *__restrict__ band_exp, int nv, int *__restrict__ order,
                                  int *__restrict__ es) {
  __shared__ int start[122];
  if (threadIdx.x != 0) return;
  for (int i = 0; i < 122; ++i) start[i] = 0;
  for (int v = 0; v < nv; ++v) start[band_exp[v] + 61]++;
  for (int i = 1; i < 122; ++i) start[i] += start[i - 1];     // start[e + 60] = first slot of exponent e
  for (int v = 0; v < nv; ++v) {
    const int e = band_exp[v];
    const int k = start[e + 60]++;
    order[k] = v;
    es[k] = e;
  }
}

size_t band_exp_ints(int nv, int nc) { return (size_t)5 * nv + nc; }

hipError_t launch_band_exponents(const float2 *psi_v, int nv, const float2 *psi_c, int nc, int nr,
                                 const float *scale, int ldsc, int *band_exp, hipStream_t s) {
  // layout (band_exp_ints): exponents [nv], band order [nv], sorted exponents [nv], then the row
  // maxima as floats: occupied [nv], unoccupied [nc], then the per-band shifts [nv]
  float *vmax = reinterpret_cast<float *>(band_exp + 3 * nv);
  float *cmax = vmax + nv;
  hipLaunchKernelGGL(absmax_rows_kernel, dim3(nv), dim3(256), 0, s, psi_v, nv, nr, vmax);
  hipLaunchKernelGGL(absmax_rows_kernel, dim3(nc), dim3(256), 0, s, psi_c, nc, nr, cmax);
  hipLaunchKernelGGL(band_exponent_kernel, dim3((nv + 63) / 64), dim3(64), 0, s, vmax, nv, cmax, nc, scale, ldsc,
                     band_exp, band_exp + 4 * nv + nc);
  hipLaunchKernelGGL(band_order_kernel, dim3(1), dim3(64), 0, s, band_exp, nv, band_exp + nv, band_exp + 2 * nv);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Rate reference for the split update: MFMA-only waves (two per SIMD, no producers) that take their
// BF16 operands from 16 KB of LDS filled with the caller's words, twelve 32x32x16 products per
// iteration over four accumulators.  Under a sustained BF16 MFMA load the chip runs at its power
// limit, below the clock of the peak figure, so this gives the executed-flop rate a kernel fed from
// LDS can reach on the same device: 12 * 32768 flop per wave-iteration.
// ---------------------------------------------------------------------------------------------
constexpr int RATE_SETS = 16;   // operand sets of 64 lanes x 16 bytes

__global__ __launch_bounds__(2 * NTHR, 2) void mfma_rate_kernel(const u32x4 *__restrict__ words, int n_iter,
                                                                float *__restrict__ out) {
  __shared__ u32x4 ops[RATE_SETS * 64];
  for (int i = threadIdx.x; i < RATE_SETS * 64; i += blockDim.x) ops[i] = words[i];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  typedef SplitTraits<__bf16>::vec vec;
  f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int it = 0; it < n_iter; ++it) {
    const int k = (2 * it + wave) & (RATE_SETS - 1);
    const vec a = __builtin_bit_cast(vec, ops[k * 64 + lane]);
    const vec b = __builtin_bit_cast(vec, ops[((k + 5) & (RATE_SETS - 1)) * 64 + lane]);
    const vec c = __builtin_bit_cast(vec, ops[((k + 9) & (RATE_SETS - 1)) * 64 + lane]);
    c0 = SplitTraits<__bf16>::mfma(a, b, c0);
    c1 = SplitTraits<__bf16>::mfma(a, c, c1);
    c2 = SplitTraits<__bf16>::mfma(c, b, c2);
    c3 = SplitTraits<__bf16>::mfma(b, a, c3);
    c0 = SplitTraits<__bf16>::mfma(a, c, c0);
    c1 = SplitTraits<__bf16>::mfma(c, b, c1);
    c2 = SplitTraits<__bf16>::mfma(b, a, c2);
    c3 = SplitTraits<__bf16>::mfma(a, b, c3);
    c0 = SplitTraits<__bf16>::mfma(c, b, c0);
    c1 = SplitTraits<__bf16>::mfma(b, a, c1);
    c2 = SplitTraits<__bf16>::mfma(a, b, c2);
    c3 = SplitTraits<__bf16>::mfma(a, c, c3);
  }
  float r = 0.f;
#pragma unroll
  for (int e = 0; e < 16; ++e) r += c0[e] + c1[e] + c2[e] + c3[e];
  out[(size_t)blockIdx.x * (2 * NTHR) + threadIdx.x] = r;
}

hipError_t launch_mfma_rate(const unsigned *words, int n_iter, int grid, float *out, hipStream_t s) {
  hipLaunchKernelGGL(mfma_rate_kernel, dim3(grid), dim3(2 * NTHR), 0, s, reinterpret_cast<const u32x4 *>(words),
                     n_iter, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Tile table and dispatch
// ---------------------------------------------------------------------------------------------
struct TileCfg { const char *name; int precision; };
static const TileCfg kTiles[] = {
  {"fp32_t128_fold_vouter", GW_FP32},
  {"fp32_t128_vouter", GW_FP32},
  {"bf16split_t128_vouter", GW_SPLIT_BF16},
  {"fp16split_t128_scaled_vouter", GW_SPLIT_FP16_SCALED},
  {"fp32_t128_fold_couter", GW_FP32},
  {"bf16split_t128_couter", GW_SPLIT_BF16},
  {"bf16split_t128_ws", GW_SPLIT_BF16},
  {"bf16split_t128_ws_k32", GW_SPLIT_BF16},
  {"bf16split_t128_ws_prio", GW_SPLIT_BF16},
  {"bf16split_t128_ws_k32_prio", GW_SPLIT_BF16},
  {"fp16split_t128_ws_k32_scaled", GW_SPLIT_FP16_SCALED},
  {"bf16split_t128_ws2_k32", GW_SPLIT_BF16},
  {"fp16split_t128_ws2_k32_scaled", GW_SPLIT_FP16_SCALED},
  {"bf16split_t128x256_wide_k16", GW_SPLIT_BF16},
  {"fp16split_t128x256_wide_k16_scaled", GW_SPLIT_FP16_SCALED},
  {"bf16split_t128x256_planar_k16", GW_SPLIT_BF16},
  {"fp16split_t128x256_planar_k16_scaled", GW_SPLIT_FP16_SCALED},
};

int herk_tile_count() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
const char *herk_tile_name(int t) { return (t >= 0 && t < herk_tile_count()) ? kTiles[t].name : ""; }
bool herk_tile_supports(int t, int precision) {
  return t >= 0 && t < herk_tile_count() && kTiles[t].precision == precision;
}
int herk_default_tile(int precision, int nr) {
  (void)nr;
  switch (precision) {
    case GW_FP32: return 4;
    case GW_SPLIT_BF16: return 15;
    case GW_SPLIT_FP16_SCALED: return 16;
  }
  return -1;
}

hipError_t launch_herk(int precision, int tile, const float2 *psi_v, const float2 *psi_c, const float *scale, int ldsc,
                       const int *band_exp, float2 *p, int nr, int nv, int nc, int accumulate, hipStream_t s) {
  if (tile < 0) tile = herk_default_tile(precision, nr);
  const int nb = (nr + HB - 1) / HB;
  const int ntiles = nb * (nb + 1) / 2;
  dim3 grid(ntiles), block(NTHR);
#define GW_LAUNCH(KERNEL, ...) \
  hipLaunchKernelGGL(HIP_KERNEL_NAME(KERNEL), grid, block, 0, s, __VA_ARGS__)
  switch (tile) {
    case 0: GW_LAUNCH((herk_fp32_kernel<true, false>), psi_v, psi_c, scale, ldsc, p, nr, nv, nc, ntiles, accumulate); break;
    case 1: GW_LAUNCH((herk_fp32_kernel<false, false>), psi_v, psi_c, scale, ldsc, p, nr, nv, nc, ntiles, accumulate); break;
    case 2: GW_LAUNCH((herk_split_kernel<__bf16, false, false>), psi_v, psi_c, scale, ldsc, band_exp, p, nr, nv, nc, ntiles,
                      accumulate); break;
    case 3: GW_LAUNCH((herk_split_kernel<_Float16, true, false>), psi_v, psi_c, scale, ldsc, band_exp, p, nr, nv, nc, ntiles,
                      accumulate); break;
    case 4: GW_LAUNCH((herk_fp32_kernel<true, true>), psi_v, psi_c, scale, ldsc, p, nr, nv, nc, ntiles, accumulate); break;
    case 5: GW_LAUNCH((herk_split_kernel<__bf16, false, true>), psi_v, psi_c, scale, ldsc, band_exp, p, nr, nv, nc, ntiles,
                      accumulate); break;
#define GW_WS(T_, KW_, PRIO_, SC_, NPW_)                                                                  \
  hipLaunchKernelGGL(HIP_KERNEL_NAME(herk_split_ws_kernel<T_, KW_, PRIO_, SC_, NPW_>), grid, dim3((1 + NPW_) * NTHR), \
                     0, s, psi_v, psi_c, scale, ldsc, band_exp, p, nr, nv, nc, ntiles, accumulate)
    case 6: GW_WS(__bf16, 16, false, false, 1); break;
    case 7: GW_WS(__bf16, 32, false, false, 1); break;
    case 8: GW_WS(__bf16, 16, true, false, 1); break;
    case 9: GW_WS(__bf16, 32, true, false, 1); break;
    case 10:
      if (!band_exp) return hipErrorInvalidValue;
      GW_WS(_Float16, 32, false, true, 1);
      break;
    case 11: GW_WS(__bf16, 32, false, false, 2); break;
    case 12:
      if (!band_exp) return hipErrorInvalidValue;
      GW_WS(_Float16, 32, false, true, 2);
      break;
#undef GW_WS
    case 13:
    case 14: {
      const int nw = wide_block_count(nb);
      if (tile == 14 && !band_exp) return hipErrorInvalidValue;
      if (tile == 13)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(herk_split_wide_kernel<__bf16, false>), dim3(nw), dim3(3 * NTHR), 0, s,
                           psi_v, psi_c, scale, ldsc, band_exp, p, nr, nv, nc, nw, accumulate);
      else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(herk_split_wide_kernel<_Float16, true>), dim3(nw), dim3(3 * NTHR), 0, s,
                           psi_v, psi_c, scale, ldsc, band_exp, p, nr, nv, nc, nw, accumulate);
      break;
    }
    case 15:
    case 16: {
      // the BF16 instance reads the s^2 table that follows the s table (scale_table_floats)
      const int nw = wide_block_count(nb);
      if (tile == 16 && !band_exp) return hipErrorInvalidValue;
      if (tile == 15)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(herk_split_wide_planar_kernel<__bf16, false>), dim3(nw), dim3(3 * NTHR), 0,
                           s, psi_v, psi_c, scale, ldsc, band_exp, p, nr, nv, nc, nw, accumulate);
      else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(herk_split_wide_planar_kernel<_Float16, true>), dim3(nw), dim3(3 * NTHR), 0,
                           s, psi_v, psi_c, scale, ldsc, band_exp, p, nr, nv, nc, nw, accumulate);
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
#undef GW_LAUNCH
  return hipGetLastError();
}

}  // namespace gwi
