// Static self-energy matrix elements in g-space (the paper's self-energy section):
//   f~_g^{nv} = sum_r exp(-i G.r) conj(u_n(r)) u_v(r)            (pair products + row transform)
//   Sigma_x(n,n')   = -sum_g V(q+g) sum_v f~_g^{nv} conj(f~_g^{n'v})
//   Sigma_sex(n,n') =  sum_v sum_g f~_g^{nv} T_g^{n'v},  T = -S conj(f~)   (T form; S on FP64 MFMA)
//   Sigma_sex(n,n') = -sum_a sigma_a sum_v zeta_a^{nv} conj(zeta_a^{n'v}),  zeta = f~^T A   (eigen form)
// The transforms are FP32 (the library's sphere passes); every contraction accumulates in FP64.
#include "gw_internal.h"

namespace gwi {

__global__ void fill_f32_kernel(float *__restrict__ p, int n, float v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// out[g][j] = conj(in[g][j]) in FP64
__global__ void conj_upcast_kernel(const float2 *__restrict__ in, size_t n, double2 *__restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float2 v = in[i];
  out[i] = make_double2((double)v.x, -(double)v.y);
}

__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }

// out[n][n'] = scale * sum_g w_g sum_v a[g][n*nv+v] * op(b[g][n'*nv+v]), op = conj if CONJ;
// w_g = sv_g^2 when sv is given, else 1.  One workgroup per (n, n').
template <bool CONJ, typename TB>
__global__ __launch_bounds__(256) void contract_kernel(const float2 *__restrict__ a, const TB *__restrict__ b, int ng,
                                                       int nv, long long ld, const double *__restrict__ sv,
                                                       double scale, int nn, double2 *__restrict__ out) {
  const int n = blockIdx.x / nn, np = blockIdx.x % nn;
  __shared__ double rr[256], ri[256];
  double sr = 0.0, si = 0.0;
  const long long total = (long long)ng * nv;
  for (long long idx = threadIdx.x; idx < total; idx += 256) {
    const int g = (int)(idx / nv), v = (int)(idx % nv);
    const double2 x = to_d2(a[(long long)g * ld + (long long)n * nv + v]);
    double2 y = to_d2(b[(long long)g * ld + (long long)np * nv + v]);
    if (CONJ) y.y = -y.y;
    double w = 1.0;
    if (sv) w = sv[g] * sv[g];
    sr += w * (x.x * y.x - x.y * y.y);
    si += w * (x.x * y.y + x.y * y.x);
  }
  rr[threadIdx.x] = sr;
  ri[threadIdx.x] = si;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      rr[threadIdx.x] += rr[threadIdx.x + st];
      ri[threadIdx.x] += ri[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(size_t)n * nn + np] = make_double2(scale * rr[0], scale * ri[0]);
}

// zeta[a][j] = sum_g f[g][j] A[g][a]  (j over the nn*nv pairs, fastest)
__global__ void zeta_kernel(const float2 *__restrict__ f, int ng, int npair, const double2 *__restrict__ modes, int nm,
                            double2 *__restrict__ zeta) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npair * nm) return;
  const int a = idx / npair, j = idx % npair;
  double zr = 0.0, zi = 0.0;
  for (int g = 0; g < ng; ++g) {
    const float2 x = f[(size_t)g * npair + j];
    const double2 m = modes[(size_t)g * nm + a];
    zr += (double)x.x * m.x - (double)x.y * m.y;
    zi += (double)x.x * m.y + (double)x.y * m.x;
  }
  zeta[(size_t)a * npair + j] = make_double2(zr, zi);
}

// out[n][n'] = -sum_a sigma_a sum_v zeta[a][n*nv+v] conj(zeta[a][n'*nv+v]); one workgroup per (n, n')
__global__ __launch_bounds__(256) void contract_modes_kernel(const double2 *__restrict__ zeta, int nm, int nv, int nn,
                                                             const double *__restrict__ sigma,
                                                             double2 *__restrict__ out) {
  const int n = blockIdx.x / nn, np = blockIdx.x % nn;
  const int npair = nn * nv;
  __shared__ double rr[256], ri[256];
  double sr = 0.0, si = 0.0;
  for (int idx = threadIdx.x; idx < nm * nv; idx += 256) {
    const int a = idx / nv, v = idx % nv;
    const double2 x = zeta[(size_t)a * npair + n * nv + v], y = zeta[(size_t)a * npair + np * nv + v];
    const double s = sigma[a];
    sr += s * (x.x * y.x + x.y * y.y);       // x conj(y)
    si += s * (x.y * y.x - x.x * y.y);
  }
  rr[threadIdx.x] = sr;
  ri[threadIdx.x] = si;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      rr[threadIdx.x] += rr[threadIdx.x + st];
      ri[threadIdx.x] += ri[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(size_t)n * nn + np] = make_double2(-rr[0], -ri[0]);
}

hipError_t launch_fill_f32(float *p, int n, float v, hipStream_t s) {
  hipLaunchKernelGGL(fill_f32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_conj_upcast(const float2 *in, size_t n, double2 *out, hipStream_t s) {
  hipLaunchKernelGGL(conj_upcast_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, n, out);
  return hipGetLastError();
}

hipError_t launch_contract_conj(const float2 *a, const float2 *b, int ng, int nv, long long ld, const double *sv,
                                double scale, int nn, double2 *out, hipStream_t s) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(contract_kernel<true, float2>), dim3(nn * nn), dim3(256), 0, s, a, b, ng, nv, ld,
                     sv, scale, nn, out);
  return hipGetLastError();
}

hipError_t launch_contract_t(const float2 *a, const double2 *t, int ng, int nv, long long ld, double scale, int nn,
                             double2 *out, hipStream_t s) {
  hipLaunchKernelGGL(HIP_KERNEL_NAME(contract_kernel<false, double2>), dim3(nn * nn), dim3(256), 0, s, a, t, ng, nv,
                     ld, (const double *)nullptr, scale, nn, out);
  return hipGetLastError();
}

hipError_t launch_zeta(const float2 *f, int ng, int npair, const double2 *modes, int nm, double2 *zeta, hipStream_t s) {
  hipLaunchKernelGGL(zeta_kernel, dim3((npair * nm + 255) / 256), dim3(256), 0, s, f, ng, npair, modes, nm, zeta);
  return hipGetLastError();
}

hipError_t launch_contract_modes(const double2 *zeta, int nm, int nv, int nn, const double *sigma, double2 *out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(contract_modes_kernel, dim3(nn * nn), dim3(256), 0, s, zeta, nm, nv, nn, sigma, out);
  return hipGetLastError();
}

}  // namespace gwi
