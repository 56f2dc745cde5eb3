// Learned band-tail correction of the truncated unoccupied-band sum.
//
// The paper lists the truncation of the unoccupied-band sum of Eq.(Pstatic) as its first
// technical issue.  This correction predicts, per G, the missing part of P~ from a truncated
// build:  dP~ = -(diag(d) + U U^H) with d_G = softplus(o_G0) s_G and
// u_Gk = (o_G,1+k + i o_G,17+k) sqrt(s_G) for k < r (zero beyond; the rank r <= 16 is a model setting),
// s_G = |Re P~_Nc(G,G)|, where o_G is a 4-128-128-33
// MLP (SiLU, BF16 weights, FP32 arithmetic) of the raw features
// x_G = (|q+G|, log|Re P~_Nc(G,G)|, Nc/N_g, E_max) normalised by stored mean and std.
// Training minimises ||dP~ - T||_F^2 / ||T||_F^2 with T = H(P~_4Nc) - H(P~_Nc), H(X) = (X+X^H)/2.
//
// These are small dense products (widths <= 128, N_g <= a few thousand), launch-bound rather than
// compute-bound, so each kernel maps one thread to one output element (or one workgroup to one row
// with a workgroup reduction) with FP32 accumulation.
#include "gw_internal.h"

namespace gwi {

constexpr int TW = 128;     // hidden width
constexpr int TO = 33;      // outputs: 1 + 2 * TR
constexpr int TR = 16;      // rank of the off-diagonal part

__device__ __forceinline__ float bf2f(const __bf16 x) { return (float)x; }
__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}
__device__ __forceinline__ float softplus(float z) { return z > 20.f ? z : log1pf(expf(z)); }

// ---- features and target -------------------------------------------------------------------------
__global__ void tail_features_kernel(const float2 *__restrict__ p, int ng, const int *__restrict__ miller, double q0,
                                     double q1, double q2, double a_bohr, int nc, double e_max,
                                     float *__restrict__ feat) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  const double b = 2.0 * 3.14159265358979323846 / a_bohr;
  const double x = (miller[3 * g] + q0) * b, y = (miller[3 * g + 1] + q1) * b, z = (miller[3 * g + 2] + q2) * b;
  const float diag = fabsf(p[(size_t)g * ng + g].x);
  feat[4 * g + 0] = (float)sqrt(x * x + y * y + z * z);
  feat[4 * g + 1] = logf(fmaxf(diag, 1e-30f));
  feat[4 * g + 2] = (float)nc / (float)ng;
  feat[4 * g + 3] = (float)e_max;
}

// T = H(full) - H(trunc), 32x32 tiles with the transposed partners through LDS.
__global__ __launch_bounds__(256) void tail_target_kernel(const float2 *__restrict__ full,
                                                          const float2 *__restrict__ trunc, int ng,
                                                          float2 *__restrict__ t) {
  __shared__ float2 tf[32][33], tt[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = 0; k < 32; k += 8) {
    const int r = c0 + ty + k, c = r0 + tx;
    if (r < ng && c < ng) {
      tf[ty + k][tx] = full[(size_t)r * ng + c];
      tt[ty + k][tx] = trunc[(size_t)r * ng + c];
    }
  }
  __syncthreads();
  for (int k = 0; k < 32; k += 8) {
    const int g = r0 + ty + k, gp = c0 + tx;
    if (g < ng && gp < ng) {
      const float2 a = full[(size_t)g * ng + gp], at = tf[tx][ty + k];
      const float2 b = trunc[(size_t)g * ng + gp], bt = tt[tx][ty + k];
      t[(size_t)g * ng + gp] = make_float2(0.5f * (a.x + at.x) - 0.5f * (b.x + bt.x),
                                           0.5f * (a.y - at.y) - 0.5f * (b.y - bt.y));
    }
  }
}

// ---- MLP forward ----------------------------------------------------------------------------------
// layer 1: xn = (x - mean)/std, z1 = xn W1 + b1, h1 = silu(z1)
__global__ void tail_l1_kernel(const float *__restrict__ feat, int n, const __bf16 *__restrict__ w1,
                               const float *__restrict__ b1, const float *__restrict__ norm, float *__restrict__ xn,
                               float *__restrict__ z1, float *__restrict__ h1) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * TW) return;
  const int g = idx / TW, j = idx % TW;
  float acc = b1[j];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float x = (feat[4 * g + i] - norm[i]) / norm[4 + i];
    acc += x * bf2f(w1[i * TW + j]);
    if (j == 0) xn[4 * g + i] = x;
  }
  if (z1) z1[idx] = acc;
  h1[idx] = silu(acc);
}

// dense layer: z = h W + b over K = TW inputs, M outputs; act = silu or identity
template <bool ACT>
__global__ void tail_dense_kernel(const float *__restrict__ h, int n, int m, const __bf16 *__restrict__ w,
                                  const float *__restrict__ b, float *__restrict__ z, float *__restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int g = idx / m, j = idx % m;
  const float *hr = h + (size_t)g * TW;
  float acc = b[j];
  for (int k = 0; k < TW; ++k) acc += hr[k] * bf2f(w[k * m + j]);
  if (z) z[idx] = acc;
  out[idx] = ACT ? silu(acc) : acc;
}

// ---- head, T U, U^H U, loss terms and d loss / d o ----------------------------------------------
__global__ void tail_head_kernel(const float *__restrict__ o, const float *__restrict__ feat, int n, int rank,
                                 float *__restrict__ d, float2 *__restrict__ u) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const float s = expf(feat[4 * g + 1]);
  const float rs = sqrtf(s);
  d[g] = softplus(o[g * TO]) * s;
  for (int k = 0; k < TR; ++k)
    u[g * TR + k] = k < rank ? make_float2(o[g * TO + 1 + k] * rs, o[g * TO + 1 + TR + k] * rs) : make_float2(0.f, 0.f);
}

// W = T U, one workgroup per row g; also the row's contribution to ||T||^2.
__global__ __launch_bounds__(256) void tail_tu_kernel(const float2 *__restrict__ t, const float2 *__restrict__ u,
                                                      int n, float2 *__restrict__ w, float *__restrict__ trow) {
  const int g = blockIdx.x;
  __shared__ float red[256][2 * TR + 1];
  float acc[2 * TR + 1];
#pragma unroll
  for (int k = 0; k < 2 * TR + 1; ++k) acc[k] = 0.f;
  for (int gp = threadIdx.x; gp < n; gp += 256) {
    const float2 a = t[(size_t)g * n + gp];
    acc[2 * TR] += a.x * a.x + a.y * a.y;
#pragma unroll
    for (int k = 0; k < TR; ++k) {
      const float2 b = u[gp * TR + k];
      acc[2 * k] += a.x * b.x - a.y * b.y;
      acc[2 * k + 1] += a.x * b.y + a.y * b.x;
    }
  }
#pragma unroll
  for (int k = 0; k < 2 * TR + 1; ++k) red[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 2 * TR + 1; ++k) red[threadIdx.x][k] += red[threadIdx.x + s][k];
    __syncthreads();
  }
  if (threadIdx.x < TR) w[g * TR + threadIdx.x] = make_float2(red[0][2 * threadIdx.x], red[0][2 * threadIdx.x + 1]);
  if (threadIdx.x == 0) trow[g] = red[0][2 * TR];
}

// G = U^H U (16 x 16), one workgroup, thread (k, l).
__global__ __launch_bounds__(256) void tail_gram_kernel(const float2 *__restrict__ u, int n, float2 *__restrict__ gm) {
  const int k = threadIdx.x / TR, l = threadIdx.x % TR;
  float2 acc = make_float2(0.f, 0.f);
  for (int g = 0; g < n; ++g) {
    const float2 a = u[g * TR + k], b = u[g * TR + l];      // conj(a) b
    acc.x += a.x * b.x + a.y * b.y;
    acc.y += a.x * b.y - a.y * b.x;
  }
  gm[k * TR + l] = acc;
}

// Per row g: B U = d U + U G + W, B_gg = d + |u|^2 + Re T_gg, the loss terms of row g, and d loss / d o.
// tn (device) is ||T||^2, computed from trow by tail_reduce_kernel before this kernel.
__global__ void tail_grad_o_kernel(const float *__restrict__ o, const float *__restrict__ feat,
                                   const float *__restrict__ d, const float2 *__restrict__ u,
                                   const float2 *__restrict__ w, const float2 *__restrict__ gm,
                                   const float2 *__restrict__ t, int n, int rank, const float *__restrict__ tn,
                                   float *__restrict__ go, float *__restrict__ lrow) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const float s = expf(feat[4 * g + 1]), rs = sqrtf(s);
  const float inv = 1.0f / tn[0];
  const float dg = d[g];
  float u2 = 0.f, uw = 0.f;
  for (int k = 0; k < TR; ++k) {
    const float2 a = u[g * TR + k], b = w[g * TR + k];
    u2 += a.x * a.x + a.y * a.y;
    uw += a.x * b.x + a.y * b.y;          // Re(conj(u) w)
  }
  const float tgg = t[(size_t)g * n + g].x;
  const float bgg = dg + u2 + tgg;
  go[g * TO] = 2.0f * bgg * sigm(o[g * TO]) * s * inv;
  for (int k = 0; k < TR; ++k) {
    float2 bu = make_float2(dg * u[g * TR + k].x + w[g * TR + k].x, dg * u[g * TR + k].y + w[g * TR + k].y);
    for (int l = 0; l < TR; ++l) {
      const float2 a = u[g * TR + l], c = gm[l * TR + k];
      bu.x += a.x * c.x - a.y * c.y;
      bu.y += a.x * c.y + a.y * c.x;
    }
    go[g * TO + 1 + k] = k < rank ? 4.0f * bu.x * rs * inv : 0.f;        // unused columns: no gradient
    go[g * TO + 1 + TR + k] = k < rank ? 4.0f * bu.y * rs * inv : 0.f;
  }
  lrow[g] = dg * dg + 2.0f * dg * tgg + 2.0f * dg * u2 + 2.0f * uw;
}

// sum of v[0..n) into out[0] (one workgroup); with add_gram also adds ||G||_F^2 and forms the loss.
__global__ __launch_bounds__(256) void tail_reduce_kernel(const float *__restrict__ v, int n, float *__restrict__ out,
                                                          const float2 *__restrict__ gm, const float *__restrict__ tn) {
  __shared__ float red[256];
  float a = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) a += v[i];
  if (gm)
    for (int i = threadIdx.x; i < TR * TR; i += 256) a += gm[i].x * gm[i].x + gm[i].y * gm[i].y;
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = tn ? (tn[0] + red[0]) / tn[0] : red[0];
}

// ---- MLP backward ----------------------------------------------------------------------------------
// out[i][j] = sum_g a[g][i] b[g][j]   (weight gradient), a: [n][ka], b: [n][kb]
__global__ void tail_wgrad_kernel(const float *__restrict__ a, int ka, const float *__restrict__ b, int kb, int n,
                                  float *__restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ka * kb) return;
  const int i = idx / kb, j = idx % kb;
  float acc = 0.f;
  for (int g = 0; g < n; ++g) acc += a[(size_t)g * ka + i] * b[(size_t)g * kb + j];
  out[idx] = acc;
}

// out[j] = sum_g b[g][j]   (bias gradient)
__global__ void tail_bgrad_kernel(const float *__restrict__ b, int kb, int n, float *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kb) return;
  float acc = 0.f;
  for (int g = 0; g < n; ++g) acc += b[(size_t)g * kb + j];
  out[j] = acc;
}

// dz[g][i] = (sum_j b[g][j] W[i][j]) * silu'(z[g][i])   (back through a layer with TW inputs)
__global__ void tail_back_kernel(const float *__restrict__ b, int m, const __bf16 *__restrict__ w,
                                 const float *__restrict__ z, int n, float *__restrict__ dz) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * TW) return;
  const int g = idx / TW, i = idx % TW;
  float acc = 0.f;
  for (int j = 0; j < m; ++j) acc += b[(size_t)g * m + j] * bf2f(w[i * m + j]);
  dz[idx] = acc * dsilu(z[idx]);
}

// ---- Adam on the FP32 master copy, then the BF16 weights / FP32 biases of the next forward ------
// master layout: W1 [4][128], b1 [128], W2 [128][128], b2 [128], W3 [128][33], b3 [33]
// The step count t comes from device memory (step_dev), so the same launch replays correctly from a graph;
// the bias corrections are 1 - beta^t.
__global__ void tail_adam_kernel(float *__restrict__ master, float *__restrict__ m, float *__restrict__ v,
                                 const float *__restrict__ grad, int np, float lr, float b1, float b2, float eps,
                                 const int *__restrict__ step_dev, __bf16 *__restrict__ wout, float *__restrict__ bout,
                                 int update) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  float p = master[i];
  if (update) {
    const float t = (float)step_dev[0];
    const float c1 = 1.0f - powf(b1, t), c2 = 1.0f - powf(b2, t);
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    master[i] = p;
  }
  // scatter to the weight / bias buffers
  const int o1 = 4 * TW, o2 = o1 + TW, o3 = o2 + TW * TW, o4 = o3 + TW, o5 = o4 + TW * TO;
  if (i < o1) wout[i] = (__bf16)p;
  else if (i < o2) bout[i - o1] = p;
  else if (i < o3) wout[o1 + (i - o2)] = (__bf16)p;
  else if (i < o4) bout[TW + (i - o3)] = p;
  else if (i < o5) wout[o1 + TW * TW + (i - o4)] = (__bf16)p;
  else bout[2 * TW + (i - o5)] = p;
}

// ---- corrected P~ and the training-box check -------------------------------------------------------
// flag[0] = 1 if any raw feature leaves [lo - 5% w, hi + 5% w], w = hi - lo (per feature).
__global__ void tail_box_kernel(const float *__restrict__ feat, int n, const float *__restrict__ norm,
                                int *__restrict__ flag) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  for (int i = 0; i < 4; ++i) {
    const float lo = norm[8 + i], hi = norm[12 + i], m = 0.05f * (hi - lo);
    const float x = feat[4 * g + i];
    if (!(x >= lo - m && x <= hi + m)) flag[0] = 1;
  }
}

// p_corr = p_trunc - (diag(d) + U U^H)
__global__ void tail_apply_kernel(const float2 *__restrict__ p, const float *__restrict__ d,
                                  const float2 *__restrict__ u, int n, float2 *__restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const int g = (int)(idx / n), gp = (int)(idx % n);
  float2 acc = make_float2(g == gp ? d[g] : 0.f, 0.f);
  for (int k = 0; k < TR; ++k) {
    const float2 a = u[g * TR + k], b = u[gp * TR + k];     // a conj(b)
    acc.x += a.x * b.x + a.y * b.y;
    acc.y += a.y * b.x - a.x * b.y;
  }
  const float2 x = p[idx];
  out[idx] = make_float2(x.x - acc.x, x.y - acc.y);
}

// One more Adam step: the device step counter advances by one (first node of a captured training step).
__global__ void tail_step_inc_kernel(int *__restrict__ step_dev) { step_dev[0] += 1; }

// Residual parts of one row g of dP~ - T with dP~ = -(diag(d) + U U^H): one workgroup per row; part[g][0..3] =
// off-diagonal |residual|^2, off-diagonal |T|^2, diagonal |residual|^2, diagonal |T|^2.
__global__ __launch_bounds__(256) void tail_parts_kernel(const float *__restrict__ d, const float2 *__restrict__ u,
                                                         const float2 *__restrict__ t, int n,
                                                         float *__restrict__ part) {
  const int g = blockIdx.x;
  __shared__ float2 ug[TR];
  __shared__ float red[4][256];
  if (threadIdx.x < TR) ug[threadIdx.x] = u[g * TR + threadIdx.x];
  __syncthreads();
  float a[4] = {0.f, 0.f, 0.f, 0.f};
  for (int gp = threadIdx.x; gp < n; gp += 256) {
    float2 c = make_float2(gp == g ? d[g] : 0.f, 0.f);
    for (int k = 0; k < TR; ++k) {
      const float2 x = ug[k], y = u[gp * TR + k];          // x conj(y)
      c.x += x.x * y.x + x.y * y.y;
      c.y += x.y * y.x - x.x * y.y;
    }
    const float2 tv = t[(size_t)g * n + gp];
    const float rx = -c.x - tv.x, ry = -c.y - tv.y;
    const int b = gp == g ? 2 : 0;
    a[b] += rx * rx + ry * ry;
    a[b + 1] += tv.x * tv.x + tv.y * tv.y;
  }
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[4 * g + threadIdx.x] = red[threadIdx.x][0];
}

// Column sums of part [n][4] into out[4] (one workgroup, double accumulation).
__global__ __launch_bounds__(256) void tail_parts_sum_kernel(const float *__restrict__ part, int n,
                                                             float *__restrict__ out) {
  __shared__ double red[4][256];
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int g = threadIdx.x; g < n; g += 256)
    for (int k = 0; k < 4; ++k) a[k] += part[4 * g + k];
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = (float)red[threadIdx.x][0];
}

// Feature statistics over a training set, one system per launch (one workgroup), merged into acc
// (double [16]): pass 0 adds the sums (acc[0..4)) and folds min / max (acc[8..12), acc[12..16)); pass 1
// adds the squared deviations from mean = acc[0..4) / total (acc[4..8)).  The first launch of a pass
// initialises its entries.
__global__ __launch_bounds__(256) void tail_stats_kernel(const float *__restrict__ feat, int n, int pass, int first,
                                                         double total, double *__restrict__ acc) {
  __shared__ double red[12][256];
  double a[12];
  for (int k = 0; k < 4; ++k) {
    a[k] = 0.0;
    a[4 + k] = INFINITY;
    a[8 + k] = -INFINITY;
  }
  for (int g = threadIdx.x; g < n; g += 256)
    for (int k = 0; k < 4; ++k) {
      const double x = feat[4 * g + k];
      if (pass == 0) {
        a[k] += x;
        a[4 + k] = fmin(a[4 + k], x);
        a[8 + k] = fmax(a[8 + k], x);
      } else {
        const double dx = x - acc[k] / total;
        a[k] += dx * dx;
      }
    }
  for (int k = 0; k < 12; ++k) red[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < 4; ++k) {
        red[k][threadIdx.x] += red[k][threadIdx.x + st];
        red[4 + k][threadIdx.x] = fmin(red[4 + k][threadIdx.x], red[4 + k][threadIdx.x + st]);
        red[8 + k][threadIdx.x] = fmax(red[8 + k][threadIdx.x], red[8 + k][threadIdx.x + st]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    if (pass == 0) {
      acc[k] = (first ? 0.0 : acc[k]) + red[k][0];
      acc[8 + k] = first ? red[4 + k][0] : fmin(acc[8 + k], red[4 + k][0]);
      acc[12 + k] = first ? red[8 + k][0] : fmax(acc[12 + k], red[8 + k][0]);
    } else {
      acc[4 + k] = (first ? 0.0 : acc[4 + k]) + red[k][0];
    }
  }
}

// norm = mean[4], std[4] (1 where std <= 1e-12 max(1, |mean|)), min[4], max[4] as floats.
__global__ void tail_stats_final_kernel(const double *__restrict__ acc, double total, float *__restrict__ norm) {
  const int k = threadIdx.x;
  if (k >= 4) return;
  const double mean = acc[k] / total;
  double sd = sqrt(acc[4 + k] / total);
  if (sd <= 1e-12 * fmax(1.0, fabs(mean))) sd = 1.0;
  norm[k] = (float)mean;
  norm[4 + k] = (float)sd;
  norm[8 + k] = (float)acc[8 + k];
  norm[12 + k] = (float)acc[12 + k];
}

// ---- launch sequences ------------------------------------------------------------------------------
#define T_LAUNCH(kernel, total, ...)                                                                      \
  do {                                                                                                    \
    hipLaunchKernelGGL(kernel, dim3((unsigned)(((size_t)(total) + 255) / 256)), dim3(256), 0, s, __VA_ARGS__); \
    hipError_t e_ = hipGetLastError();                                                                    \
    if (e_ != hipSuccess) return e_;                                                                      \
  } while (0)

size_t tail_ws_floats(int n) {
  // xn 4n, z1 h1 z2 h2 4*128n, o go 2*33n, d n, u w 2*(32n), trow lrow 2n, gram 512, scalars 16,
  // dz1 dz2 2*128n
  return (size_t)n * (4 + 6 * TW + 2 * TO + 1 + 4 * TR + 2 + 4) + 2 * TR * TR + 16 + 64;
}

struct TailWs {
  float *xn, *z1, *h1, *z2, *h2, *o, *go, *d, *trow, *lrow, *dz1, *dz2, *part, *sc;
  float2 *u, *w, *gm;
};

static TailWs carve(float *base, int n) {
  TailWs t;
  float *p = base;
  t.xn = p; p += 4 * (size_t)n;
  t.z1 = p; p += (size_t)TW * n;
  t.h1 = p; p += (size_t)TW * n;
  t.z2 = p; p += (size_t)TW * n;
  t.h2 = p; p += (size_t)TW * n;
  t.dz1 = p; p += (size_t)TW * n;
  t.dz2 = p; p += (size_t)TW * n;
  t.o = p; p += (size_t)TO * n;
  t.go = p; p += (size_t)TO * n;
  t.d = p; p += n;
  t.trow = p; p += n;
  t.lrow = p; p += n;
  t.part = p; p += 4 * (size_t)n;
  p = (float *)(((uintptr_t)p + 15) & ~(uintptr_t)15);
  t.u = (float2 *)p; p += 2 * (size_t)TR * n;
  t.w = (float2 *)p; p += 2 * (size_t)TR * n;
  t.gm = (float2 *)p; p += 2 * TR * TR;
  t.sc = p;
  return t;
}

hipError_t tail_features(const float2 *p, int ng, const int *miller, const double *q, double a_bohr, int nc,
                         double e_max, float *feat, hipStream_t s) {
  T_LAUNCH(tail_features_kernel, ng, p, ng, miller, q[0], q[1], q[2], a_bohr, nc, e_max, feat);
  return hipSuccess;
}

hipError_t tail_target(const float2 *full, const float2 *trunc, int ng, float2 *t, hipStream_t s) {
  dim3 grid((ng + 31) / 32, (ng + 31) / 32);
  hipLaunchKernelGGL(tail_target_kernel, grid, dim3(256), 0, s, full, trunc, ng, t);
  return hipGetLastError();
}

static hipError_t forward(const gw_mlp &w, const float *feat, int n, const TailWs &t, float *out, hipStream_t s) {
  const __bf16 *w1 = (const __bf16 *)w.w, *w2 = w1 + 4 * TW, *w3 = w2 + TW * TW;
  const float *b1 = w.b, *b2 = b1 + TW, *b3 = b2 + TW;
  T_LAUNCH(tail_l1_kernel, (size_t)n * TW, feat, n, w1, b1, w.norm, t.xn, t.z1, t.h1);
  T_LAUNCH(tail_dense_kernel<true>, (size_t)n * TW, t.h1, n, TW, w2, b2, t.z2, t.h2);
  T_LAUNCH(tail_dense_kernel<false>, (size_t)n * TO, t.h2, n, TO, w3, b3, (float *)nullptr, out);
  return hipSuccess;
}

hipError_t tail_forward(const gw_mlp &w, const float *feat, int n, float *ws, float *out, hipStream_t s) {
  return forward(w, feat, n, carve(ws, n), out, s);
}

// forward and loss (into loss_out) plus d loss / d o in t.go
static hipError_t loss_and_grad_o(const gw_mlp &w, const float *feat, const float2 *target, int n, const TailWs &t,
                                  float *loss_out, hipStream_t s) {
  hipError_t e = forward(w, feat, n, t, t.o, s);
  if (e != hipSuccess) return e;
  // loss and d loss / d o
  T_LAUNCH(tail_head_kernel, n, t.o, feat, n, w.rank, t.d, t.u);
  hipLaunchKernelGGL(tail_tu_kernel, dim3(n), dim3(256), 0, s, target, t.u, n, t.w, t.trow);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(tail_gram_kernel, dim3(1), dim3(256), 0, s, t.u, n, t.gm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  float *tn = t.sc;
  hipLaunchKernelGGL(tail_reduce_kernel, dim3(1), dim3(256), 0, s, t.trow, n, tn, (const float2 *)nullptr,
                     (const float *)nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  T_LAUNCH(tail_grad_o_kernel, n, t.o, feat, t.d, t.u, t.w, t.gm, target, n, w.rank, tn, t.go, t.lrow);
  hipLaunchKernelGGL(tail_reduce_kernel, dim3(1), dim3(256), 0, s, t.lrow, n, loss_out, t.gm, tn);
  return hipGetLastError();
}

hipError_t tail_loss(const gw_mlp &w, const float *feat, const float2 *target, int n, float *ws, float *loss_out,
                     hipStream_t s) {
  return loss_and_grad_o(w, feat, target, n, carve(ws, n), loss_out, s);
}

// One training step.  The Adam step count lives in step_dev: with set_step >= 0 it is first written (eager
// calls), with set_step < 0 a kernel advances it by one (the form a captured graph replays).
hipError_t tail_train_step(const gw_mlp &w, const gw_adam &a, const float *feat, const float2 *target, int n,
                           float *ws, float *loss_out, int *step_dev, int set_step, hipStream_t s) {
  const TailWs t = carve(ws, n);
  hipError_t e = set_step >= 0 ? launch_fill_int(step_dev, set_step, s) : hipSuccess;
  if (e != hipSuccess) return e;
  if (set_step < 0) {
    hipLaunchKernelGGL(tail_step_inc_kernel, dim3(1), dim3(1), 0, s, step_dev);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  e = loss_and_grad_o(w, feat, target, n, t, loss_out, s);
  if (e != hipSuccess) return e;
  // backward into a.grad (flat master layout)
  const __bf16 *w2 = (const __bf16 *)w.w + 4 * TW, *w3 = w2 + TW * TW;
  float *gw1 = a.grad, *gb1 = gw1 + 4 * TW, *gw2 = gb1 + TW, *gb2 = gw2 + TW * TW, *gw3 = gb2 + TW, *gb3 = gw3 + TW * TO;
  T_LAUNCH(tail_wgrad_kernel, TW * TO, t.h2, TW, t.go, TO, n, gw3);
  T_LAUNCH(tail_bgrad_kernel, TO, t.go, TO, n, gb3);
  T_LAUNCH(tail_back_kernel, (size_t)n * TW, t.go, TO, w3, t.z2, n, t.dz2);
  T_LAUNCH(tail_wgrad_kernel, TW * TW, t.h1, TW, t.dz2, TW, n, gw2);
  T_LAUNCH(tail_bgrad_kernel, TW, t.dz2, TW, n, gb2);
  T_LAUNCH(tail_back_kernel, (size_t)n * TW, t.dz2, TW, w2, t.z1, n, t.dz1);
  T_LAUNCH(tail_wgrad_kernel, 4 * TW, t.xn, 4, t.dz1, TW, n, gw1);
  T_LAUNCH(tail_bgrad_kernel, TW, t.dz1, TW, n, gb1);
  // Adam
  T_LAUNCH(tail_adam_kernel, GW_TAIL_NPARAM, a.master, a.m, a.v, a.grad, GW_TAIL_NPARAM, a.lr, a.beta1, a.beta2, a.eps,
           (const int *)step_dev, (__bf16 *)w.w, w.b, 1);
  return hipSuccess;
}

hipError_t tail_sync_weights(gw_mlp &w, const float *master, hipStream_t s) {
  T_LAUNCH(tail_adam_kernel, GW_TAIL_NPARAM, (float *)master, (float *)nullptr, (float *)nullptr, (const float *)nullptr,
           GW_TAIL_NPARAM, 0.f, 0.f, 0.f, 0.f, (const int *)nullptr, (__bf16 *)w.w, w.b, 0);
  return hipSuccess;
}

hipError_t tail_check_box(const float *feat, int n, const float *norm, int *flag, hipStream_t s) {
  hipError_t e = launch_fill_int(flag, 0, s);
  if (e != hipSuccess) return e;
  T_LAUNCH(tail_box_kernel, n, feat, n, norm, flag);
  return hipSuccess;
}

hipError_t tail_apply(const gw_mlp &w, const float *feat, const float2 *p, int n, float *ws, float2 *out,
                      hipStream_t s) {
  const TailWs t = carve(ws, n);
  hipError_t e = forward(w, feat, n, t, t.o, s);
  if (e != hipSuccess) return e;
  T_LAUNCH(tail_head_kernel, n, t.o, feat, n, w.rank, t.d, t.u);
  T_LAUNCH(tail_apply_kernel, (size_t)n * n, p, t.d, t.u, n, out);
  return hipSuccess;
}

hipError_t tail_residual_parts(const gw_mlp &w, const float *feat, const float2 *target, int n, float *ws,
                               float *parts, hipStream_t s) {
  const TailWs t = carve(ws, n);
  hipError_t e = forward(w, feat, n, t, t.o, s);
  if (e != hipSuccess) return e;
  T_LAUNCH(tail_head_kernel, n, t.o, feat, n, w.rank, t.d, t.u);
  hipLaunchKernelGGL(tail_parts_kernel, dim3(n), dim3(256), 0, s, t.d, t.u, target, n, t.part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(tail_parts_sum_kernel, dim3(1), dim3(256), 0, s, t.part, n, parts);
  return hipGetLastError();
}

hipError_t tail_fit_norm(int nsys, const float *const *feats, const int *ngs, double *acc, float *norm,
                         hipStream_t s) {
  double total = 0.0;
  for (int i = 0; i < nsys; ++i) total += ngs[i];
  for (int pass = 0; pass < 2; ++pass)
    for (int i = 0; i < nsys; ++i) {
      hipLaunchKernelGGL(tail_stats_kernel, dim3(1), dim3(256), 0, s, feats[i], ngs[i], pass, i == 0 ? 1 : 0, total,
                         acc);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  hipLaunchKernelGGL(tail_stats_final_kernel, dim3(1), dim3(64), 0, s, (const double *)acc, total, norm);
  return hipGetLastError();
}

}  // namespace gwi
