// Coulomb scaling and the symmetric dielectric matrix of Sec. 5.1, in FP64:
//   sv(g)      = sqrt(4 pi / (Omega |q+G|^2)),  |q+G| = (2 pi / a) |q + m|  (cubic cell)
//   eps(g,g')  = delta - sv(g) H(g,g') sv(g'),   H = (P~ + P~^H) / 2
// Where |q+G| < 1e-10 * 2pi/a, sv = 0 and eps(g,g) is the caller's head value.
#include "gw_internal.h"

namespace gwi {

__global__ void sqrtv_kernel(const int *__restrict__ miller, int ng, double q0, double q1, double q2, double a_bohr,
                             double *__restrict__ sv) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  const double b = 2.0 * 3.14159265358979323846 / a_bohr;
  const double x = (miller[3 * g] + q0) * b, y = (miller[3 * g + 1] + q1) * b, z = (miller[3 * g + 2] + q2) * b;
  const double k2 = x * x + y * y + z * z;
  const double omega = a_bohr * a_bohr * a_bohr;
  sv[g] = (sqrt(k2) < 1e-10 * b) ? 0.0 : sqrt(4.0 * 3.14159265358979323846 / (omega * k2));
}

hipError_t launch_sqrtv(const int *miller, int ng, double q0, double q1, double q2, double a_bohr, double *sv,
                        hipStream_t s) {
  hipLaunchKernelGGL(sqrtv_kernel, dim3((ng + 255) / 256), dim3(256), 0, s, miller, ng, q0, q1, q2, a_bohr, sv);
  return hipGetLastError();
}

// 32x32 tiles; the transposed tile comes through LDS so both reads are coalesced.
__global__ __launch_bounds__(256) void eps_build_kernel(const float2 *__restrict__ p, int ng,
                                                        const double *__restrict__ sv, double head,
                                                        double2 *__restrict__ eps) {
  __shared__ float2 t[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // load tile P[c0..][r0..] (the transpose partner) into t[col][row]
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int r = c0 + ty + k, c = r0 + tx;
    if (r < ng && c < ng) t[ty + k][tx] = p[(size_t)r * ng + c];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int g = r0 + ty + k, gp = c0 + tx;
    if (g < ng && gp < ng) {
      const float2 a = p[(size_t)g * ng + gp];     // P~(g, g')
      const float2 b = t[tx][ty + k];               // P~(g', g)
      const double hr = 0.5 * ((double)a.x + (double)b.x);
      const double hi = 0.5 * ((double)a.y - (double)b.y);
      const double s = sv[g] * sv[gp];
      double2 e;
      e.x = (g == gp ? 1.0 : 0.0) - s * hr;
      e.y = -s * hi;
      if (g == gp && sv[g] == 0.0) { e.x = head; e.y = 0.0; }
      eps[(size_t)g * ng + gp] = e;
    }
  }
}

hipError_t launch_eps_build(const float2 *p_gg, int ng, const double *sv, double head, double2 *eps, hipStream_t s) {
  dim3 grid((ng + 31) / 32, (ng + 31) / 32);
  hipLaunchKernelGGL(eps_build_kernel, grid, dim3(256), 0, s, p_gg, ng, sv, head, eps);
  return hipGetLastError();
}

}  // namespace gwi
