// Pair products f_vc(r) = conj(u_v(r)) u_c(r) sqrt(p/(E_c - E_v))  (Eq.(fdef)) and the scale table.
//
// HBM-bound: the kernel writes nv*nc*nr complex64 values and reads each
// psi_c row once per workgroup.  Layout: one workgroup owns a chunk of 512
// grid points of one unoccupied band c and loops over all occupied bands v,
// so the psi_c chunk is read once and held in registers while psi_v chunks
// (nv*512*8 bytes, shared by every c-workgroup of the same chunk) come from
// L2.  Each thread handles two adjacent grid points with 16-byte stores.
#include "gw_internal.h"

namespace gwi {

int scale_ld(int nc) { return (nc + 31) / 32 * 32; }

__global__ void scale_table_kernel(const double *__restrict__ e_v, int nv, const double *__restrict__ e_c, int nc,
                                   double prefactor, float *__restrict__ scale, int ldsc) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nv * ldsc) return;
  const int v = idx / ldsc, c = idx - v * ldsc;
  scale[idx] = c < nc ? (float)sqrt(prefactor / (e_c[c] - e_v[v])) : 0.0f;
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
constexpr int PP_CHUNK = 2 * PP_THREADS;   // grid points per workgroup

__device__ __forceinline__ float2 conj_mul_scale(float2 v, float2 c, float s) {
  // conj(v) * c * s
  return make_float2((v.x * c.x + v.y * c.y) * s, (v.x * c.y - v.y * c.x) * s);
}

__global__ __launch_bounds__(PP_THREADS) void pair_products_kernel(const float2 *__restrict__ psi_v, int nv,
                                                                   const float2 *__restrict__ psi_c, int nc, int nr,
                                                                   const float *__restrict__ scale, int ldsc,
                                                                   float2 *__restrict__ f) {
  const int c = blockIdx.x;                            // unoccupied band (fastest: blocks of one chunk run together)
  const int r0 = blockIdx.y * PP_CHUNK + 2 * threadIdx.x;
  if (r0 >= nr) return;
  const bool two = (r0 + 1 < nr);
  const float2 *pc = psi_c + (size_t)c * nr + r0;
  const float2 c0 = pc[0];
  const float2 c1 = two ? pc[1] : make_float2(0.f, 0.f);
  for (int v = 0; v < nv; ++v) {
    const float s = scale[v * ldsc + c];
    const float2 *pv = psi_v + (size_t)v * nr + r0;
    const float2 v0 = pv[0];
    float2 *out = f + ((size_t)v * nc + c) * nr + r0;
    if (two && ((nr & 1) == 0)) {
      const float2 v1 = pv[1];
      const float2 a = conj_mul_scale(v0, c0, s), b = conj_mul_scale(v1, c1, s);
      const f32x4 w = {a.x, a.y, b.x, b.y};
      __builtin_nontemporal_store(w, reinterpret_cast<f32x4 *>(out));
    } else {
      out[0] = conj_mul_scale(v0, c0, s);
      if (two) out[1] = conj_mul_scale(pv[1], c1, s);
    }
  }
}

hipError_t launch_pair_products(const float2 *psi_v, int nv, const float2 *psi_c, int nc, int nr, const float *scale,
                                int ldsc, float2 *f, hipStream_t s) {
  dim3 grid(nc, (nr + PP_CHUNK - 1) / PP_CHUNK);
  hipLaunchKernelGGL(pair_products_kernel, grid, dim3(PP_THREADS), 0, s, psi_v, nv, psi_c, nc, nr, scale, ldsc, f);
  return hipGetLastError();
}

}  // namespace gwi
