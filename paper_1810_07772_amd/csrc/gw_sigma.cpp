// C ABI of the static self-energy matrix elements in g-space (bare exchange, screened exchange in
// the T and eigen forms of the paper's self-energy section).  Kernels in sigma.hip; the pair
// transforms use the sphere passes of fft.hip and the T product the FP64 MFMA GEMM.
#include <algorithm>
#include <cmath>

#include "gw_internal.h"

using namespace gwi;

namespace {

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// workspace slots of this file (after those of the batched path)
enum { SG_ONES = 512, SG_F, SG_FT, SG_FG, SG_MAP, SG_A1, SG_A2, SG_MILLER, SG_SQRTV, SG_S, SG_FC, SG_T, SG_Z };

int check_common(gw_ctx *ctx, const void *psi_n, int nn, const void *psi_v, int nv, gw_grid grid, const int *miller,
                 int ng) {
  GWX_CHECK(ctx, psi_n && psi_v, "psi_n and psi_v must not be NULL");
  GWX_CHECK(ctx, nn >= 1 && nn <= 256, "nn must be in [1, 256]");
  GWX_CHECK(ctx, nv >= 1, "nv must be positive");
  GWX_STATUS(api_check_grid(ctx, grid));
  const long long nr = (long long)grid.n1 * grid.n2 * grid.n3;
  GWX_CHECK(ctx, nr <= (1 << 24), "grid too large");
  GWX_CHECK(ctx, (long long)nn * nv * nr <= (1LL << 31), "nn * nv * N_r too large for one pass");
  GWX_STATUS(api_check_sphere(ctx, grid, miller, ng));
  GWX_STATUS(api_grid_supported(ctx, grid));
  return GW_OK;
}

// f~ [ng][nn*nv] (complex64, pair index n*nv + v fastest) for the bands and occupied set given
int pair_transform(gw_ctx *ctx, const float2 *psi_n, int nn, const float2 *psi_v, int nv, gw_grid grid,
                   const int *miller, int ng, float2 **ft, hipStream_t s) {
  const int nr = grid.n1 * grid.n2 * grid.n3, B = nn * nv;
  const int ldsc = scale_ld(nv);
  void *ones, *f, *fr, *fg;
  GWX_STATUS(api_ws_get(ctx, SG_ONES, (size_t)nn * ldsc * sizeof(float), &ones, s));
  GWX_HIP(ctx, launch_fill_f32((float *)ones, nn * ldsc, 1.0f, s));
  GWX_STATUS(api_ws_get(ctx, SG_F, (size_t)B * nr * sizeof(float2), &f, s));
  GWX_STATUS(api_ws_get(ctx, SG_FT, (size_t)B * nr * sizeof(float2), &fr, s));
  GWX_STATUS(api_ws_get(ctx, SG_FG, (size_t)B * ng * sizeof(float2), &fg, s));
  // conj(u_n) u_v as rows [n*nv + v][r] (the pair-product kernel with unit scales), then grid-major
  GWX_HIP(ctx, launch_pair_products(psi_n, nn, psi_v, nv, nr, (const float *)ones, ldsc, (float2 *)f, s));
  GWX_HIP(ctx, launch_transpose_c64((const float2 *)f, (float2 *)fr, B, nr, nr, B, s));
  SpherePlan p;
  int *dA, *dB, *dC;
  GWX_STATUS(upload_plan(ctx, grid, miller, ng, SG_MAP, p, &dA, &dB, &dC, s));
  const int bc = std::max(1, std::min(p.bc, B));
  void *a1, *a2;
  GWX_STATUS(api_ws_get(ctx, SG_A1, (size_t)grid.n1 * grid.n2 * p.m3count * bc * sizeof(float2), &a1, s));
  GWX_STATUS(api_ws_get(ctx, SG_A2, (size_t)grid.n1 * p.npair * bc * sizeof(float2), &a2, s));
  GWX_HIP(ctx, transform_rows(p, -1, (const float2 *)fr, B, B, (float2 *)fg, B, (float2 *)a1, (float2 *)a2, bc, dA,
                              dB, dC, s));
  *ft = (float2 *)fg;
  return GW_OK;
}

int sqrtv_on_device(gw_ctx *ctx, const int *miller, int ng, const double *q, double a_bohr, double **sv,
                    hipStream_t s) {
  void *m, *d;
  GWX_STATUS(api_ws_get(ctx, SG_MILLER, (size_t)ng * 3 * sizeof(int), &m, s));
  GWX_STATUS(api_ws_get(ctx, SG_SQRTV, (size_t)ng * sizeof(double), &d, s));
  GWX_HIP(ctx, hipMemcpyAsync(m, miller, (size_t)ng * 3 * sizeof(int), hipMemcpyHostToDevice, s));
  GWX_HIP(ctx, launch_sqrtv((const int *)m, ng, q[0], q[1], q[2], a_bohr, (double *)d, s));
  *sv = (double *)d;
  return GW_OK;
}

}  // namespace

extern "C" {

int gw_sigma_static(gw_ctx *ctx, const gw_c32 *psi_n, int nn, const gw_c32 *psi_v, int nv, gw_grid grid,
                    const double *q, const int *g_miller, int ng, const gw_c64 *eps_inv, gw_c64 *sigma_x,
                    gw_c64 *sigma_sex, void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_STATUS(check_common(ctx, psi_n, nn, psi_v, nv, grid, g_miller, ng));
  GWX_CHECK(ctx, q != nullptr && std::isfinite(q[0]) && std::isfinite(q[1]) && std::isfinite(q[2]),
            "q must be given and finite");
  GWX_CHECK(ctx, sigma_x || sigma_sex, "ask for sigma_x, sigma_sex or both");
  GWX_CHECK(ctx, !sigma_sex || eps_inv, "sigma_sex needs eps_inv");
  if (api_device(ctx) < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  float2 *ft;
  GWX_STATUS(pair_transform(ctx, (const float2 *)psi_n, nn, (const float2 *)psi_v, nv, grid, g_miller, ng, &ft, s));
  double *sv;
  GWX_STATUS(sqrtv_on_device(ctx, g_miller, ng, q, grid.a_bohr, &sv, s));
  const int B = nn * nv;
  if (sigma_x) GWX_HIP(ctx, launch_contract_conj(ft, ft, ng, nv, B, sv, -1.0, nn, (double2 *)sigma_x, s));
  if (sigma_sex) {
    void *sp, *fc, *tp;
    GWX_STATUS(api_ws_get(ctx, SG_S, (size_t)ng * ng * sizeof(double2), &sp, s));
    GWX_STATUS(api_ws_get(ctx, SG_FC, (size_t)ng * B * sizeof(double2), &fc, s));
    GWX_STATUS(api_ws_get(ctx, SG_T, (size_t)ng * B * sizeof(double2), &tp, s));
    GWX_HIP(ctx, launch_screening((const double2 *)eps_inv, sv, ng, (double2 *)sp, s));
    GWX_HIP(ctx, launch_conj_upcast(ft, (size_t)ng * B, (double2 *)fc, s));
    // T = -S conj(f~)
    GWX_HIP(ctx, launch_zgemm(ng, B, ng, (const double2 *)sp, ng, 0, (const double2 *)fc, B, 0, (double2 *)tp, B, -1.0,
                              0.0, s));
    GWX_HIP(ctx, launch_contract_t(ft, (const double2 *)tp, ng, nv, B, 1.0, nn, (double2 *)sigma_sex, s));
  }
  return GW_OK;
}

int gw_sigma_sex_modes(gw_ctx *ctx, const gw_c32 *psi_n, int nn, const gw_c32 *psi_v, int nv, gw_grid grid,
                       const int *g_miller, int ng, const gw_c64 *modes, const double *sigma, int n_modes,
                       gw_c64 *sigma_sex, void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_STATUS(check_common(ctx, psi_n, nn, psi_v, nv, grid, g_miller, ng));
  GWX_CHECK(ctx, modes && sigma && sigma_sex, "modes, sigma and sigma_sex must not be NULL");
  GWX_CHECK(ctx, n_modes >= 1 && n_modes <= ng, "n_modes must be in [1, ng]");
  if (api_device(ctx) < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  float2 *ft;
  GWX_STATUS(pair_transform(ctx, (const float2 *)psi_n, nn, (const float2 *)psi_v, nv, grid, g_miller, ng, &ft, s));
  const int B = nn * nv;
  void *z;
  GWX_STATUS(api_ws_get(ctx, SG_Z, (size_t)B * n_modes * sizeof(double2), &z, s));
  GWX_HIP(ctx, launch_zeta(ft, ng, B, (const double2 *)modes, n_modes, (double2 *)z, s));
  GWX_HIP(ctx, launch_contract_modes((const double2 *)z, n_modes, nv, nn, sigma, (double2 *)sigma_sex, s));
  return GW_OK;
}

}  // extern "C"
