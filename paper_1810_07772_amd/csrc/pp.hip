// Plasmon-pole model of the dynamic inverse dielectric matrix (the paper's section on it):
//   S = sqrt(V) (eps^-1 - I) sqrt(V)            the polarization part of the static W
//   S = A diag(sigma) A^H                       Eq.(eigdecomp), the few most negative sigma
//   omega_a^2 = (A^H M A)_aa / |sigma_a|,  M(g,g') = V V' [(q+g).(q+g')] rho_{g-g'}   Eq.(ppfreq)
//   S(w) = sum_a A_a sigma_a omega_a^2 / (omega_a^2 - w^2) A_a^H                  Eq.(ppform)
// Kernels for the density and its transform, S and M, the small dense eigenproblems of the
// block iteration (one-workgroup Jacobi), and the pole-form evaluation.  Large products use
// the complex FP64 MFMA GEMM.
#include "gw_internal.h"

namespace gwi {

// rho(r) = occ sum_v |psi_v(r)|^2, written as complex (rho, 0) for the transform that follows
__global__ void density_kernel(const float2 *__restrict__ psi, int nv, int nr, double occ, double2 *__restrict__ rho) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  double a = 0.0;
  for (int v = 0; v < nv; ++v) {
    const float2 p = psi[(size_t)v * nr + r];
    a += (double)p.x * p.x + (double)p.y * p.y;
  }
  rho[r] = make_double2(occ * a, 0.0);
}

// One axis of the FP64 forward DFT on the full grid: out[.. k ..] = sum_i in[.. i ..] exp(-2 pi i k i / n_d).
// Lengths are at most 48, so each output is a direct sum; the phase comes from sincospi in FP64.
__global__ void dft_axis_f64_kernel(const double2 *__restrict__ in, double2 *__restrict__ out, int n1, int n2, int n3,
                                    int axis) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int nr = n1 * n2 * n3;
  if (idx >= nr) return;
  const int i3 = idx % n3, i2 = (idx / n3) % n2, i1 = idx / (n2 * n3);
  int n, k, stride, base;
  if (axis == 0) { n = n1; k = i1; stride = n2 * n3; base = idx - i1 * stride; }
  else if (axis == 1) { n = n2; k = i2; stride = n3; base = idx - i2 * stride; }
  else { n = n3; k = i3; stride = 1; base = idx - i3; }
  double re = 0.0, im = 0.0;
  for (int i = 0; i < n; ++i) {
    double sn, cs;
    sincospi(-2.0 * (double)((k * i) % n) / (double)n, &sn, &cs);
    const double2 x = in[base + i * stride];
    re += x.x * cs - x.y * sn;
    im += x.x * sn + x.y * cs;
  }
  out[idx] = make_double2(re, im);
}

// s = sv_g (eps_inv - delta) sv_g'
__global__ void screening_kernel(const double2 *__restrict__ ei, const double *__restrict__ sv, int ng,
                                 double2 *__restrict__ s) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ng * ng) return;
  const int g = (int)(idx / ng), h = (int)(idx % ng);
  double2 e = ei[idx];
  if (g == h) e.x -= 1.0;
  const double f = sv[g] * sv[h];
  s[idx] = make_double2(f * e.x, f * e.y);
}

// m = V_g V_h (2pi/a)^2 [(q+m_g).(q+m_h)] rho[(m_g - m_h) mod n]
__global__ void sum_rule_kernel(const int *__restrict__ miller, int ng, double q0, double q1, double q2, double b,
                                const double *__restrict__ sv, const double2 *__restrict__ rho_g, int n1, int n2,
                                int n3, double2 *__restrict__ m) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ng * ng) return;
  const int g = (int)(idx / ng), h = (int)(idx % ng);
  const int *mg = miller + 3 * g, *mh = miller + 3 * h;
  const double dot = b * b * ((q0 + mg[0]) * (q0 + mh[0]) + (q1 + mg[1]) * (q1 + mh[1]) + (q2 + mg[2]) * (q2 + mh[2]));
  const double vg = sv[g] * sv[g], vh = sv[h] * sv[h];
  const int d1 = ((mg[0] - mh[0]) % n1 + n1) % n1, d2 = ((mg[1] - mh[1]) % n2 + n2) % n2,
            d3 = ((mg[2] - mh[2]) % n3 + n3) % n3;
  const double2 r = rho_g[((size_t)d1 * n2 + d2) * n3 + d3];
  const double f = vg * vh * dot;
  m[idx] = make_double2(f * r.x, f * r.y);
}

// Start block: entries uniform in [-1, 1) (real and imaginary parts) from SplitMix64 (Steele, Lea and
// Flood, 2014) of a counter, so the iteration is deterministic.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__global__ void start_block_kernel(double2 *__restrict__ x, int ng, int b, unsigned long long seed) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ng * b) return;
  const unsigned long long u = splitmix64(seed * 0x100000000ull + 2 * idx);
  const unsigned long long w = splitmix64(seed * 0x100000000ull + 2 * idx + 1);
  const double s = 1.0 / 9007199254740992.0;     // 2^-53
  x[idx] = make_double2(2.0 * (double)(u >> 11) * s - 1.0, 2.0 * (double)(w >> 11) * s - 1.0);
}

// ---- Hermitian Jacobi eigensolver for b <= 32, one workgroup ------------------------------------
// Cyclic two-sided Jacobi with the round-robin (circle) ordering: each round rotates m/2 disjoint
// index pairs at once.  For a pair (p, q) with a_pq = |a_pq| e^{i phi}, the rotation is
// J = diag(1, e^{-i phi}) R, R the real symmetric Schur rotation of [[a_pp, |a_pq|], [|a_pq|, a_qq]];
// A <- J^H A J, V <- V J.  Eigenvalues are returned in descending order with their vectors as
// columns of z (row-major, leading dimension ldz).
constexpr int JMAX = 32;

// Sum of v over the 64 lanes of a wave.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(256) void herm_jacobi_kernel(const double2 *__restrict__ h, int b, int ldh,
                                                          double *__restrict__ evals, double2 *__restrict__ z,
                                                          int ldz, int max_sweeps) {
  __shared__ double2 A[JMAX][JMAX + 1];
  __shared__ double2 V[JMAX][JMAX + 1];
  __shared__ double rc[JMAX / 2], rs[JMAX / 2];
  __shared__ double2 rph[JMAX / 2];
  __shared__ int rp[JMAX / 2], rq[JMAX / 2];
  __shared__ double red_off[4], red_all[4];
  __shared__ int perm[JMAX];
  __shared__ int stop;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = (b + 1) & ~1;          // even size; a padding index has a zero row and column
  for (int idx = tid; idx < JMAX * JMAX; idx += 256) {
    const int i = idx / JMAX, j = idx % JMAX;
    double2 v = make_double2(0.0, 0.0);
    if (i < b && j < b) {
      const double2 a = h[(size_t)i * ldh + j], c = h[(size_t)j * ldh + i];
      v = make_double2(0.5 * (a.x + c.x), 0.5 * (a.y - c.y));     // Hermitian part
    }
    A[i][j] = v;
    V[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int half = m / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence: off-diagonal mass against the whole
    double off = 0.0, all = 0.0;
    for (int idx = tid; idx < m * m; idx += 256) {
      const int i = idx / m, j = idx % m;
      const double2 v = A[i][j];
      const double s2 = v.x * v.x + v.y * v.y;
      all += s2;
      if (i != j) off += s2;
    }
    // wave sums, then the four waves' partials
    off = wave_sum(off);
    all = wave_sum(all);
    if (lane == 0) { red_off[wave] = off; red_all[wave] = all; }
    __syncthreads();
    if (tid == 0) {
      const double o = red_off[0] + red_off[1] + red_off[2] + red_off[3];
      const double a = red_all[0] + red_all[1] + red_all[2] + red_all[3];
      stop = (o <= 1e-30 * a) || a == 0.0;   // off-diagonal norm below 1e-15 relative
    }
    __syncthreads();
    if (stop) break;
    for (int round = 0; round < m - 1; ++round) {
      if (tid < half) {
        int p, q;
        if (tid == 0) { p = round; q = m - 1; }
        else { p = (round + tid) % (m - 1); q = (round - tid + (m - 1)) % (m - 1); }
        if (p > q) { const int t = p; p = q; q = t; }
        // one reciprocal square root gives the phase and tau; c = 1/sqrt(1 + t^2) is another (three
        // long-latency operations in this serial chain instead of seven)
        const double2 apq = A[p][q];
        const double mag2 = apq.x * apq.x + apq.y * apq.y;
        double c = 1.0, s = 0.0;
        double2 ph = make_double2(1.0, 0.0);
        if (mag2 > 0.0) {
          const double inv_mag = rsqrt(mag2);
          ph = make_double2(apq.x * inv_mag, apq.y * inv_mag);
          const double tau = (A[q][q].x - A[p][p].x) * (0.5 * inv_mag);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = rsqrt(1.0 + t * t);
          s = t * c;
        }
        rp[tid] = p; rq[tid] = q; rc[tid] = c; rs[tid] = s; rph[tid] = ph;
      }
      __syncthreads();
      // columns: A J and V J.  e = e^{-i phi} = conj(ph).
      for (int item = tid; item < 2 * half * m; item += 256) {
        const int which = item / (half * m), rest = item % (half * m);
        const int k = rest / m, i = rest % m;
        const int p = rp[k], q = rq[k];
        const double c = rc[k], s = rs[k];
        const double2 e = make_double2(rph[k].x, -rph[k].y);
        double2 (*M)[JMAX + 1] = which ? V : A;
        const double2 x = M[i][p], y = M[i][q];
        const double2 ey = make_double2(e.x * y.x - e.y * y.y, e.x * y.y + e.y * y.x);
        M[i][p] = make_double2(c * x.x - s * ey.x, c * x.y - s * ey.y);
        M[i][q] = make_double2(s * x.x + c * ey.x, s * x.y + c * ey.y);
      }
      __syncthreads();
      // rows: J^H A.  conj(e) = ph.
      for (int item = tid; item < half * m; item += 256) {
        const int k = item / m, j = item % m;
        const int p = rp[k], q = rq[k];
        const double c = rc[k], s = rs[k];
        const double2 f = rph[k];
        const double2 x = A[p][j], y = A[q][j];
        const double2 fy = make_double2(f.x * y.x - f.y * y.y, f.x * y.y + f.y * y.x);
        A[p][j] = make_double2(c * x.x - s * fy.x, c * x.y - s * fy.y);
        A[q][j] = make_double2(s * x.x + c * fy.x, s * x.y + c * fy.y);
      }
      __syncthreads();
    }
  }
  // descending order of the b real eigenvalues (padding excluded)
  if (tid == 0) {
    for (int i = 0; i < b; ++i) perm[i] = i;
    for (int i = 0; i < b; ++i) {
      int best = i;
      for (int j = i + 1; j < b; ++j)
        if (A[perm[j]][perm[j]].x > A[perm[best]][perm[best]].x) best = j;
      const int t = perm[i]; perm[i] = perm[best]; perm[best] = t;
    }
  }
  __syncthreads();
  for (int idx = tid; idx < b * b; idx += 256) {
    const int i = idx / b, j = idx % b;
    z[(size_t)i * ldz + j] = V[i][perm[j]];
  }
  if (tid < b) evals[tid] = A[perm[tid]][perm[tid]].x;
}

// Column j of w (leading dimension ld) scaled to unit norm; zero columns stay zero.  One block per column.
__global__ void col_normalize_kernel(double2 *__restrict__ w, int rows, int ld) {
  const int j = blockIdx.x;
  __shared__ double red[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < rows; i += 256) {
    const double2 v = w[(size_t)i * ld + j];
    a += v.x * v.x + v.y * v.y;
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double nrm = sqrt(red[0]);
  if (nrm == 0.0) return;
  const double inv = 1.0 / nrm;
  for (int i = threadIdx.x; i < rows; i += 256) {
    double2 v = w[(size_t)i * ld + j];
    w[(size_t)i * ld + j] = make_double2(v.x * inv, v.y * inv);
  }
}

// u[:, j] *= lambda_j^-1/2 for lambda_j above rel * lambda_0 (descending), else 0 (drops a dependent direction)
__global__ void svqb_scale_kernel(double2 *__restrict__ u, const double *__restrict__ lam, int b, double rel) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= b * b) return;
  const int j = idx % b;
  const double l = lam[j];
  const double f = (l > rel * lam[0] && l > 0.0) ? 1.0 / sqrt(l) : 0.0;
  u[idx] = make_double2(u[idx].x * f, u[idx].y * f);
}

// out[0] = max_{j < nm} ||y_j - theta_j x_j|| / theta_0 (one workgroup; each wave takes modes in turn)
__global__ __launch_bounds__(256) void ritz_residual_kernel(const double2 *__restrict__ x, const double2 *__restrict__ y,
                                                            int ng, int ld, const double *__restrict__ theta, int nm,
                                                            double *__restrict__ out) {
  __shared__ double res[JMAX];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int j = wave; j < nm; j += 4) {
    const double t = theta[j];
    double a = 0.0;
    for (int g = lane; g < ng; g += 64) {
      const double2 xv = x[(size_t)g * ld + j], yv = y[(size_t)g * ld + j];
      const double dx = yv.x - t * xv.x, dy = yv.y - t * xv.y;
      a += dx * dx + dy * dy;
    }
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if (lane == 0) res[j] = sqrt(a);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int j = 0; j < nm; ++j) mx = fmax(mx, res[j]);
    out[0] = theta[0] > 0.0 ? mx / theta[0] : (mx == 0.0 ? 0.0 : INFINITY);
  }
}

// sigma_a = -theta_a, omega_a = sqrt(Re(a^H t_a) / theta_a) with t = M A (one workgroup per mode)
__global__ void pp_frequency_kernel(const double2 *__restrict__ a, int lda, const double2 *__restrict__ t, int ldt,
                                    int ng, const double *__restrict__ theta, double *__restrict__ sigma,
                                    double *__restrict__ omega) {
  const int j = blockIdx.x;
  __shared__ double red[256];
  double s = 0.0;
  for (int g = threadIdx.x; g < ng; g += 256) {
    const double2 av = a[(size_t)g * lda + j], tv = t[(size_t)g * ldt + j];
    s += av.x * tv.x + av.y * tv.y;         // Re(conj(a) t)
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double th = theta[j];
    sigma[j] = -th;
    omega[j] = sqrt(fmax(red[0], 0.0) / th);
  }
}

// b[g][a] = A[g][a] * sigma_a omega_a^2 / (omega_a^2 - w^2)
__global__ void pp_weight_kernel(const double2 *__restrict__ modes, int ng, int nm, const double *__restrict__ sigma,
                                 const double *__restrict__ omega, double w, double2 *__restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ng * nm) return;
  const int j = idx % nm;
  const double o2 = omega[j] * omega[j];
  const double c = sigma[j] * o2 / (o2 - w * w);
  const double2 v = modes[idx];
  out[idx] = make_double2(c * v.x, c * v.y);
}

// e = I + S(w) / (sv_g sv_h) where both sv > 0, else the static eps^-1 entry
__global__ void pp_finish_kernel(double2 *__restrict__ e, const double2 *__restrict__ ei_static,
                                 const double *__restrict__ sv, int ng) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ng * ng) return;
  const int g = (int)(idx / ng), h = (int)(idx % ng);
  if (sv[g] > 0.0 && sv[h] > 0.0) {
    const double f = 1.0 / (sv[g] * sv[h]);
    double2 v = e[idx];
    v.x *= f;
    v.y *= f;
    if (g == h) v.x += 1.0;
    e[idx] = v;
  } else {
    e[idx] = ei_static[idx];
  }
}

static inline unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_density(const float2 *psi, int nv, int nr, double occ, double2 *rho, hipStream_t s) {
  hipLaunchKernelGGL(density_kernel, dim3(blocks_for(nr)), dim3(256), 0, s, psi, nv, nr, occ, rho);
  return hipGetLastError();
}

hipError_t launch_density_transform(double2 *rho, double2 *tmp, int n1, int n2, int n3, hipStream_t s) {
  // rho -> tmp (axis 0) -> rho (axis 1) -> tmp (axis 2); the result is left in tmp
  const int nr = n1 * n2 * n3;
  hipLaunchKernelGGL(dft_axis_f64_kernel, dim3(blocks_for(nr)), dim3(256), 0, s, rho, tmp, n1, n2, n3, 0);
  hipLaunchKernelGGL(dft_axis_f64_kernel, dim3(blocks_for(nr)), dim3(256), 0, s, tmp, rho, n1, n2, n3, 1);
  hipLaunchKernelGGL(dft_axis_f64_kernel, dim3(blocks_for(nr)), dim3(256), 0, s, rho, tmp, n1, n2, n3, 2);
  return hipGetLastError();
}

hipError_t launch_screening(const double2 *ei, const double *sv, int ng, double2 *out, hipStream_t s) {
  hipLaunchKernelGGL(screening_kernel, dim3(blocks_for((size_t)ng * ng)), dim3(256), 0, s, ei, sv, ng, out);
  return hipGetLastError();
}

hipError_t launch_sum_rule(const int *miller, int ng, const double *q, double a_bohr, const double *sv,
                           const double2 *rho_g, int n1, int n2, int n3, double2 *m, hipStream_t s) {
  const double b = 2.0 * 3.14159265358979323846 / a_bohr;
  hipLaunchKernelGGL(sum_rule_kernel, dim3(blocks_for((size_t)ng * ng)), dim3(256), 0, s, miller, ng, q[0], q[1],
                     q[2], b, sv, rho_g, n1, n2, n3, m);
  return hipGetLastError();
}

hipError_t launch_start_block(double2 *x, int ng, int b, unsigned long long seed, hipStream_t s) {
  hipLaunchKernelGGL(start_block_kernel, dim3(blocks_for((size_t)ng * b)), dim3(256), 0, s, x, ng, b, seed);
  return hipGetLastError();
}

hipError_t launch_herm_jacobi(const double2 *h, int b, int ldh, double *evals, double2 *z, int ldz, hipStream_t s) {
  if (b < 1 || b > JMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(herm_jacobi_kernel, dim3(1), dim3(256), 0, s, h, b, ldh, evals, z, ldz, 40);
  return hipGetLastError();
}

hipError_t launch_col_normalize(double2 *w, int rows, int ld, int cols, hipStream_t s) {
  hipLaunchKernelGGL(col_normalize_kernel, dim3(cols), dim3(256), 0, s, w, rows, ld);
  return hipGetLastError();
}

hipError_t launch_svqb_scale(double2 *u, const double *lam, int b, double rel, hipStream_t s) {
  hipLaunchKernelGGL(svqb_scale_kernel, dim3(blocks_for((size_t)b * b)), dim3(256), 0, s, u, lam, b, rel);
  return hipGetLastError();
}

hipError_t launch_ritz_residual(const double2 *x, const double2 *y, int ng, int ld, const double *theta, int nm,
                                double *out, hipStream_t s) {
  if (nm < 1 || nm > JMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ritz_residual_kernel, dim3(1), dim3(256), 0, s, x, y, ng, ld, theta, nm, out);
  return hipGetLastError();
}

hipError_t launch_pp_frequency(const double2 *a, int lda, const double2 *t, int ldt, int ng, const double *theta,
                               int nm, double *sigma, double *omega, hipStream_t s) {
  hipLaunchKernelGGL(pp_frequency_kernel, dim3(nm), dim3(256), 0, s, a, lda, t, ldt, ng, theta, sigma, omega);
  return hipGetLastError();
}

hipError_t launch_pp_weight(const double2 *modes, int ng, int nm, const double *sigma, const double *omega, double w,
                            double2 *out, hipStream_t s) {
  hipLaunchKernelGGL(pp_weight_kernel, dim3(blocks_for((size_t)ng * nm)), dim3(256), 0, s, modes, ng, nm, sigma, omega,
                     w, out);
  return hipGetLastError();
}

hipError_t launch_pp_finish(double2 *e, const double2 *ei_static, const double *sv, int ng, hipStream_t s) {
  hipLaunchKernelGGL(pp_finish_kernel, dim3(blocks_for((size_t)ng * ng)), dim3(256), 0, s, e, ei_static, sv, ng);
  return hipGetLastError();
}

}  // namespace gwi
