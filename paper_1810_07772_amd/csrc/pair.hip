// Pair products f_vc(r) = conj(u_v(r)) u_c(r) sqrt(p/(E_c - E_v))  (Eq.(fdef)) and the scale table.
//
// HBM-bound: the kernel writes nv*nc*nr complex64 values.  Layout: one workgroup owns a chunk of 1024
// grid points and PP_CG unoccupied bands; a thread holds the psi_v values of PP_VB occupied bands at its
// four grid points in registers and, for each of its unoccupied bands, issues 2 PP_VB independent 16-byte
// non-temporal stores, so many stores are in flight per thread and each wave writes 2 KB of a row of F
// per band pair.  Chunks run fastest across the grid, so neighbouring workgroups write consecutive
// stretches of the same rows of F.
#include "gw_internal.h"

namespace gwi {

int scale_ld(int nc) { return (nc + 31) / 32 * 32; }
size_t scale_table_floats(int nv, int nc) { return (size_t)2 * nv * scale_ld(nc); }

// s_vc = sqrt(p / (E_c - E_v)) in [nv][ldsc], then s_vc^2 = p / (E_c - E_v) in a second [nv][ldsc] table
// (the planar wide update scales only its row side, by s^2); zero for c >= nc in both
__global__ void scale_table_kernel(const double *__restrict__ e_v, int nv, const double *__restrict__ e_c, int nc,
                                   double prefactor, float *__restrict__ scale, int ldsc) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nv * ldsc) return;
  const int v = idx / ldsc, c = idx - v * ldsc;
  const double q = c < nc ? prefactor / (e_c[c] - e_v[v]) : 0.0;
  scale[idx] = (float)sqrt(q);
  scale[(size_t)nv * ldsc + idx] = (float)q;
}

hipError_t launch_scale_table(const double *e_v, int nv, const double *e_c, int nc, double prefactor, float *scale,
                              int ldsc, hipStream_t s) {
  const int n = nv * ldsc;
  hipLaunchKernelGGL(scale_table_kernel, dim3((n + 255) / 256), dim3(256), 0, s, e_v, nv, e_c, nc, prefactor, scale,
                     ldsc);
  return hipGetLastError();
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int PP_THREADS = 256;
constexpr int PP_NH = 2;   // point pairs per thread, 128 points apart (1: 4.68 TB/s, 2: 4.90, 4: 4.80 at 36^3)
constexpr int PP_SEG = 2 * 64 * PP_NH;                   // consecutive points per wave
constexpr int PP_CHUNK = (PP_THREADS / 64) * PP_SEG;     // grid points per workgroup

__device__ __forceinline__ float2 conj_mul_scale(float2 v, float2 c, float s) {
  // conj(v) * c * s
  return make_float2((v.x * c.x + v.y * c.y) * s, (v.x * c.y - v.y * c.x) * s);
}

constexpr int PP_VB = 8;   // occupied bands whose psi_v values a thread holds in registers
constexpr int PP_CG = 8;   // unoccupied bands per workgroup (4: 4.4 TB/s, 8: 4.7, 16: 4.5 at 36^3)

// Lane l of wave w holds the point pairs (p, p + 1), p = chunk + w PP_SEG + 2 l + 128 h, h < PP_NH: for
// each (v, c) a wave's PP_NH stores cover PP_NH KB of one row of F back to back.
__global__ __launch_bounds__(PP_THREADS) void pair_products_kernel(const float2 *__restrict__ psi_v, int nv,
                                                                   const float2 *__restrict__ psi_c, int nc, int nr,
                                                                   const float *__restrict__ scale, int ldsc,
                                                                   float2 *__restrict__ f) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int base = blockIdx.x * PP_CHUNK + wave * PP_SEG + 2 * lane;
  const int cg0 = blockIdx.y * PP_CG;
  if (base >= nr) return;   // the thread's first point is its smallest
  bool one[PP_NH], two[PP_NH], wide[PP_NH];
#pragma unroll
  for (int h = 0; h < PP_NH; ++h) {
    const int p = base + 128 * h;
    one[h] = p < nr;
    two[h] = p + 1 < nr;
    wide[h] = two[h] && ((nr & 1) == 0);
  }
  if ((nr & 1) == 0 && ((int)blockIdx.x + 1) * PP_CHUNK <= nr) {
    // every point of the workgroup exists and pairs are 16-byte aligned: no per-lane condition anywhere,
    // so the wait for the next band's prefetched psi_c counts past this band's stores instead of draining
    // them (on this architecture one counter covers both)
    for (int vb = 0; vb < nv; vb += PP_VB) {
      const int nvb = min(PP_VB, nv - vb);
      f32x4 vv[PP_NH][PP_VB];
#pragma unroll
      for (int h = 0; h < PP_NH; ++h)
#pragma unroll
        for (int k = 0; k < PP_VB; ++k)
          vv[h][k] = *reinterpret_cast<const f32x4 *>(psi_v + (size_t)(vb + min(k, nvb - 1)) * nr + base + 128 * h);
      f32x4 cv[PP_NH], cn[PP_NH];
#pragma unroll
      for (int h = 0; h < PP_NH; ++h) {
        cv[h] = *reinterpret_cast<const f32x4 *>(psi_c + (size_t)min(cg0, nc - 1) * nr + base + 128 * h);
        cn[h] = cv[h];
      }
      for (int cc = 0; cc < PP_CG; ++cc) {
        const int c = cg0 + cc;
        if (c >= nc) break;
        if (cc + 1 < PP_CG && c + 1 < nc) {
#pragma unroll
          for (int h = 0; h < PP_NH; ++h)
            cn[h] = *reinterpret_cast<const f32x4 *>(psi_c + (size_t)(c + 1) * nr + base + 128 * h);
        }
        float sk[PP_VB];
#pragma unroll
        for (int k = 0; k < PP_VB; ++k) sk[k] = scale[(vb + min(k, nvb - 1)) * ldsc + c];
#pragma unroll
        for (int k = 0; k < PP_VB; ++k) {
          if (k < nvb) {                                     // uniform
#pragma unroll
            for (int h = 0; h < PP_NH; ++h) {
              const float2 a = conj_mul_scale(make_float2(vv[h][k][0], vv[h][k][1]), make_float2(cv[h][0], cv[h][1]), sk[k]);
              const float2 b = conj_mul_scale(make_float2(vv[h][k][2], vv[h][k][3]), make_float2(cv[h][2], cv[h][3]), sk[k]);
              const f32x4 w = {a.x, a.y, b.x, b.y};
              __builtin_nontemporal_store(w, reinterpret_cast<f32x4 *>(f + ((size_t)(vb + k) * nc + c) * nr + base + 128 * h));
            }
          }
        }
#pragma unroll
        for (int h = 0; h < PP_NH; ++h) cv[h] = cn[h];
      }
    }
    return;
  }
  for (int vb = 0; vb < nv; vb += PP_VB) {
    const int nvb = min(PP_VB, nv - vb);
    float2 v0[PP_NH][PP_VB], v1[PP_NH][PP_VB];
#pragma unroll
    for (int h = 0; h < PP_NH; ++h)
#pragma unroll
      for (int k = 0; k < PP_VB; ++k) {
        v0[h][k] = make_float2(0.f, 0.f);
        v1[h][k] = make_float2(0.f, 0.f);
        if (k < nvb && one[h]) {
          const float2 *pv = psi_v + (size_t)(vb + k) * nr + base + 128 * h;
          v0[h][k] = pv[0];
          if (two[h]) v1[h][k] = pv[1];
        }
      }
    // psi_c of the next unoccupied band is loaded while the current band's products are stored, so no
    // band waits for its own loads; the band's PP_VB scales are read together before its stores
    float2 c0[PP_NH], c1[PP_NH], n0[PP_NH] = {}, n1[PP_NH] = {};
    auto load_c = [&](int c, float2 (&a)[PP_NH], float2 (&b)[PP_NH]) {
#pragma unroll
      for (int h = 0; h < PP_NH; ++h) {
        const float2 *pc = psi_c + (size_t)c * nr + base + 128 * h;
        a[h] = one[h] ? pc[0] : make_float2(0.f, 0.f);
        b[h] = two[h] ? pc[1] : make_float2(0.f, 0.f);
      }
    };
    if (cg0 < nc) load_c(cg0, c0, c1);
    for (int cc = 0; cc < PP_CG; ++cc) {
      const int c = cg0 + cc;
      if (c >= nc) break;
      if (cc + 1 < PP_CG && c + 1 < nc) load_c(c + 1, n0, n1);
      float sk[PP_VB];
#pragma unroll
      for (int k = 0; k < PP_VB; ++k) sk[k] = k < nvb ? scale[(vb + k) * ldsc + c] : 0.f;
#pragma unroll
      for (int k = 0; k < PP_VB; ++k) {
        if (k < nvb) {
          const float s = sk[k];
#pragma unroll
          for (int h = 0; h < PP_NH; ++h) {
            if (!one[h]) continue;
            float2 *out = f + ((size_t)(vb + k) * nc + c) * nr + base + 128 * h;
            const float2 a = conj_mul_scale(v0[h][k], c0[h], s);
            if (wide[h]) {
              const float2 b = conj_mul_scale(v1[h][k], c1[h], s);
              const f32x4 w = {a.x, a.y, b.x, b.y};
              __builtin_nontemporal_store(w, reinterpret_cast<f32x4 *>(out));
            } else {
              out[0] = a;
              if (two[h]) out[1] = conj_mul_scale(v1[h][k], c1[h], s);
            }
          }
        }
      }
#pragma unroll
      for (int h = 0; h < PP_NH; ++h) {
        c0[h] = n0[h];
        c1[h] = n1[h];
      }
    }
  }
}

hipError_t launch_pair_products(const float2 *psi_v, int nv, const float2 *psi_c, int nc, int nr, const float *scale,
                                int ldsc, float2 *f, hipStream_t s) {
  dim3 grid((nr + PP_CHUNK - 1) / PP_CHUNK, (nc + PP_CG - 1) / PP_CG);
  hipLaunchKernelGGL(pair_products_kernel, grid, dim3(PP_THREADS), 0, s, psi_v, nv, psi_c, nc, nr, scale, ldsc, f);
  return hipGetLastError();
}

}  // namespace gwi
