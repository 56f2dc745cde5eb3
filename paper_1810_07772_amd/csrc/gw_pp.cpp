// C ABI of the plasmon-pole model (the paper's section on the dynamic inverse dielectric matrix):
// the few most negative eigenpairs of S = sqrt(V)(eps^-1 - I)sqrt(V) by block subspace iteration
// with a Rayleigh-Ritz step per iteration, their frequencies from the Johnson sum rule, and the
// pole-form eps^-1(w).  Kernels in pp.hip; the large products on the FP64 MFMA GEMM.
//
// Iteration (all on the device, one host read of the residual per iteration):
//   Y = -S X;  H = X^H Y;  H = Z diag(theta) Z^H (Jacobi, descending);  X <- X Z, Y <- Y Z
//   stop when max_{a < n_modes} ||Y_a - theta_a X_a|| <= tol * theta_0
//   X <- orthonormal basis of Y (columns to unit length, then X = Y U diag(lambda)^-1/2 from the
//        eigenpairs of Y^H Y: the SVQB orthonormalisation of Stathopoulos and Wu, 2002)
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "gw_internal.h"

using namespace gwi;

namespace {

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

constexpr int kBlock = 32;      // subspace size (the Jacobi kernel's limit)
constexpr int kMaxModes = 24;   // at least 8 guard vectors beyond the wanted modes

enum {
  PP_MILLER = 40, PP_SQRTV, PP_RHO, PP_RHO_T, PP_S, PP_M, PP_X, PP_Y, PP_W, PP_T, PP_SMALL, PP_B, PP_SPLITK
};

struct Small {            // b x b matrices and eigenvalues of the iteration
  double2 *h, *z, *g, *u;
  double *theta, *lam, *res;
  double2 *ws;             // split-K partial products of the thin products
  size_t ws_elems;
};

int upload_sphere(gw_ctx *ctx, const int *miller, int ng, const double *q, double a_bohr, int **dm, double **dsv,
                  hipStream_t s) {
  void *m, *sv;
  GWX_STATUS(api_ws_get(ctx, PP_MILLER, (size_t)ng * 3 * sizeof(int), &m, s));
  GWX_STATUS(api_ws_get(ctx, PP_SQRTV, (size_t)ng * sizeof(double), &sv, s));
  GWX_HIP(ctx, hipMemcpyAsync(m, miller, (size_t)ng * 3 * sizeof(int), hipMemcpyHostToDevice, s));
  GWX_HIP(ctx, launch_sqrtv((const int *)m, ng, q[0], q[1], q[2], a_bohr, (double *)sv, s));
  *dm = (int *)m;
  *dsv = (double *)sv;
  return GW_OK;
}

// x = orthonormal basis of the columns of w (w is overwritten by its column-normalised copy)
int orthonormalize(gw_ctx *ctx, double2 *w, int ng, int b, const Small &sm, double2 *x, hipStream_t s) {
  GWX_HIP(ctx, launch_col_normalize(w, ng, b, b, s));
  GWX_HIP(ctx, launch_zgemm_splitk(b, b, ng, w, b, 1, w, b, 0, sm.g, b, 1.0, 0.0, sm.ws, sm.ws_elems, s));
  GWX_HIP(ctx, launch_herm_jacobi(sm.g, b, b, sm.lam, sm.u, b, s));
  GWX_HIP(ctx, launch_svqb_scale(sm.u, sm.lam, b, 1e-14, s));
  GWX_HIP(ctx, launch_zgemm(ng, b, b, w, b, 0, sm.u, b, 0, x, b, 1.0, 0.0, s));
  return GW_OK;
}

}  // namespace

extern "C" {

int gw_plasmon_pole(gw_ctx *ctx, const gw_c64 *eps_inv, int ng, gw_grid grid, const double *q, const int *g_miller,
                    const gw_c32 *psi_v, int nv, double occupation, int n_modes, double tol, int max_iter,
                    double *sigma, double *omega, gw_c64 *modes, int *iterations, double *residual, void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_CHECK(ctx, eps_inv && psi_v && sigma && omega && modes && iterations && q,
            "eps_inv, psi_v, sigma, omega, modes, iterations and q must not be NULL");
  GWX_STATUS(api_check_grid(ctx, grid));
  const long long nrl = (long long)grid.n1 * grid.n2 * grid.n3;
  GWX_CHECK(ctx, nrl <= (1 << 24), "grid too large");
  GWX_STATUS(api_check_sphere(ctx, grid, g_miller, ng));
  GWX_CHECK(ctx, std::isfinite(q[0]) && std::isfinite(q[1]) && std::isfinite(q[2]), "q must be finite");
  GWX_CHECK(ctx, nv > 0, "nv must be positive");
  GWX_CHECK(ctx, std::isfinite(occupation) && occupation > 0.0, "occupation must be positive");
  GWX_CHECK(ctx, n_modes >= 1 && n_modes <= std::min(kMaxModes, ng), "n_modes must be in [1, min(24, ng)]");
  GWX_CHECK(ctx, std::isfinite(tol) && tol > 0.0, "tol must be positive");
  GWX_CHECK(ctx, max_iter >= 1 && max_iter <= 100000, "max_iter must be in [1, 100000]");
  if (ctx->device < 0) {
    *iterations = 0;
    return GW_OK;
  }
  hipStream_t s = as_stream(stream);
  const int nr = (int)nrl, b = std::min(kBlock, ng);
  int *dm;
  double *sv;
  GWX_STATUS(upload_sphere(ctx, g_miller, ng, q, grid.a_bohr, &dm, &sv, s));
  // density and its transform on the full grid, then S and the sum-rule matrix M
  void *rho, *rho_t, *sp, *mp;
  GWX_STATUS(api_ws_get(ctx, PP_RHO, (size_t)nr * sizeof(double2), &rho, s));
  GWX_STATUS(api_ws_get(ctx, PP_RHO_T, (size_t)nr * sizeof(double2), &rho_t, s));
  GWX_STATUS(api_ws_get(ctx, PP_S, (size_t)ng * ng * sizeof(double2), &sp, s));
  GWX_STATUS(api_ws_get(ctx, PP_M, (size_t)ng * ng * sizeof(double2), &mp, s));
  GWX_HIP(ctx, launch_density((const float2 *)psi_v, nv, nr, occupation, (double2 *)rho, s));
  GWX_HIP(ctx, launch_density_transform((double2 *)rho, (double2 *)rho_t, grid.n1, grid.n2, grid.n3, s));
  double2 *S = (double2 *)sp, *M = (double2 *)mp;
  GWX_HIP(ctx, launch_screening((const double2 *)eps_inv, sv, ng, S, s));
  GWX_HIP(ctx, launch_sum_rule(dm, ng, q, grid.a_bohr, sv, (const double2 *)rho_t, grid.n1, grid.n2, grid.n3, M, s));
  // block buffers
  void *xp, *yp, *wp, *tp, *smp;
  const size_t blk = (size_t)ng * b * sizeof(double2);
  GWX_STATUS(api_ws_get(ctx, PP_X, blk, &xp, s));
  GWX_STATUS(api_ws_get(ctx, PP_Y, blk, &yp, s));
  GWX_STATUS(api_ws_get(ctx, PP_W, blk, &wp, s));
  GWX_STATUS(api_ws_get(ctx, PP_T, blk, &tp, s));
  const size_t bb = (size_t)b * b;
  GWX_STATUS(api_ws_get(ctx, PP_SMALL, 4 * bb * sizeof(double2) + (3 * b + 8) * sizeof(double), &smp, s));
  Small sm;
  sm.h = (double2 *)smp;
  sm.z = sm.h + bb;
  sm.g = sm.z + bb;
  sm.u = sm.g + bb;
  sm.theta = (double *)(sm.u + bb);
  sm.lam = sm.theta + b;
  sm.res = sm.lam + b;
  sm.ws_elems = std::max({zgemm_splitk_ws_elems(ng, b, ng), zgemm_splitk_ws_elems(b, b, ng),
                          zgemm_splitk_ws_elems(ng, n_modes, ng)});
  sm.ws = nullptr;
  if (sm.ws_elems) {
    void *w;
    GWX_STATUS(api_ws_get(ctx, PP_SPLITK, sm.ws_elems * sizeof(double2), &w, s));
    sm.ws = (double2 *)w;
  }
  double2 *X = (double2 *)xp, *Y = (double2 *)yp, *W = (double2 *)wp, *T = (double2 *)tp;
  GWX_HIP(ctx, launch_start_block(T, ng, b, 0x5eedULL, s));
  GWX_STATUS(orthonormalize(ctx, T, ng, b, sm, X, s));
  double res = INFINITY;
  int it = 0;
  for (it = 1; it <= max_iter; ++it) {
    GWX_HIP(ctx, launch_zgemm_splitk(ng, b, ng, S, ng, 0, X, b, 0, Y, b, -1.0, 0.0, sm.ws, sm.ws_elems, s));  // -S X
    GWX_HIP(ctx, launch_zgemm_splitk(b, b, ng, X, b, 1, Y, b, 0, sm.h, b, 1.0, 0.0, sm.ws, sm.ws_elems, s));  // X^H Y
    GWX_HIP(ctx, launch_herm_jacobi(sm.h, b, b, sm.theta, sm.z, b, s));
    GWX_HIP(ctx, launch_zgemm(ng, b, b, X, b, 0, sm.z, b, 0, W, b, 1.0, 0.0, s));   // Ritz vectors
    GWX_HIP(ctx, launch_zgemm(ng, b, b, Y, b, 0, sm.z, b, 0, T, b, 1.0, 0.0, s));   // -S times them
    GWX_HIP(ctx, launch_ritz_residual(W, T, ng, b, sm.theta, n_modes, sm.res, s));
    GWX_HIP(ctx, hipMemcpyAsync(&res, sm.res, sizeof(double), hipMemcpyDeviceToHost, s));
    GWX_HIP(ctx, hipStreamSynchronize(s));
    if (!std::isfinite(res)) break;
    if (res <= tol || b == ng) break;      // converged (a full-space block is exact after one step)
    GWX_STATUS(orthonormalize(ctx, T, ng, b, sm, X, s));
  }
  *iterations = std::min(it, max_iter);
  if (residual) *residual = res;
  // frequencies from the sum rule: t = M A, omega_a^2 = Re(a^H t_a) / theta_a
  GWX_HIP(ctx, launch_zgemm_splitk(ng, n_modes, ng, M, ng, 0, W, b, 0, Y, n_modes, 1.0, 0.0, sm.ws, sm.ws_elems, s));
  GWX_HIP(ctx, launch_pp_frequency(W, b, Y, n_modes, ng, sm.theta, n_modes, sigma, omega, s));
  GWX_HIP(ctx, hipMemcpy2DAsync(modes, (size_t)n_modes * sizeof(double2), W, (size_t)b * sizeof(double2),
                                (size_t)n_modes * sizeof(double2), ng, hipMemcpyDeviceToDevice, s));
  GWX_HIP(ctx, hipStreamSynchronize(s));
  if (!std::isfinite(res)) {
    api_set_err(ctx, "plasmon-pole iteration produced a non-finite residual");
    return GW_E_HIP;
  }
  if (res > tol) {
    char m[200];
    snprintf(m, sizeof(m), "plasmon-pole iteration did not reach tol %.3g in %d iterations (residual %.3g)", tol,
             max_iter, res);
    api_set_err(ctx, m);
    return GW_E_UNSUPPORTED;
  }
  return GW_OK;
}

int gw_pp_eps_inverse(gw_ctx *ctx, const gw_c64 *eps_inv_static, int ng, gw_grid grid, const double *q,
                      const int *g_miller, const gw_c64 *modes, const double *sigma, const double *omega, int n_modes,
                      const double *freqs, int nf, gw_c64 *out, void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_CHECK(ctx, eps_inv_static && modes && sigma && omega && freqs && out && q,
            "eps_inv_static, modes, sigma, omega, freqs, out and q must not be NULL");
  GWX_STATUS(api_check_grid(ctx, grid));
  GWX_STATUS(api_check_sphere(ctx, grid, g_miller, ng));
  GWX_CHECK(ctx, n_modes >= 1 && n_modes <= ng, "n_modes must be in [1, ng]");
  GWX_CHECK(ctx, nf >= 1, "nf must be positive");
  for (int f = 0; f < nf; ++f) GWX_CHECK(ctx, std::isfinite(freqs[f]), "frequencies must be finite");
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  int *dm;
  double *sv;
  GWX_STATUS(upload_sphere(ctx, g_miller, ng, q, grid.a_bohr, &dm, &sv, s));
  void *bp;
  GWX_STATUS(api_ws_get(ctx, PP_B, (size_t)ng * n_modes * sizeof(double2), &bp, s));
  for (int f = 0; f < nf; ++f) {
    double2 *e = (double2 *)out + (size_t)f * ng * ng;
    GWX_HIP(ctx, launch_pp_weight((const double2 *)modes, ng, n_modes, sigma, omega, freqs[f], (double2 *)bp, s));
    GWX_HIP(ctx, launch_zgemm(ng, ng, n_modes, (const double2 *)bp, n_modes, 0, (const double2 *)modes, n_modes, 1, e,
                              ng, 1.0, 0.0, s));
    GWX_HIP(ctx, launch_pp_finish(e, (const double2 *)eps_inv_static, sv, ng, s));
  }
  return GW_OK;
}

}  // extern "C"
