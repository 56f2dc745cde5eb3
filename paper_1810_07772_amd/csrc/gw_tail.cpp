// C ABI of the learned band-tail correction (argument checks, workspace; kernels in tail.hip).
#include <cmath>
#include <cstdio>

#include "gw_internal.h"

using namespace gwi;

namespace {

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

int check_mlp(gw_ctx *ctx, const gw_mlp *w) {
  GWX_CHECK(ctx, w && w->w && w->b && w->norm, "gw_mlp and its buffers must not be NULL");
  return GW_OK;
}

int tail_ws(gw_ctx *ctx, int n, float **ws, hipStream_t s) {
  void *p;
  GWX_STATUS(api_ws_get(ctx, WS_TAIL, tail_ws_floats(n) * sizeof(float), &p, s));
  *ws = (float *)p;
  return GW_OK;
}

}  // namespace

extern "C" {

int gw_tail_init(gw_ctx *ctx, gw_mlp *w, const float *master, void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_STATUS(check_mlp(ctx, w));
  GWX_CHECK(ctx, master != nullptr, "master must not be NULL");
  if (ctx->device < 0) return GW_OK;
  GWX_HIP(ctx, tail_sync_weights(*w, master, as_stream(stream)));
  return GW_OK;
}

int gw_tail_target(gw_ctx *ctx, const gw_c32 *p_full, const gw_c32 *p_trunc, int ng, gw_c32 *target, void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_CHECK(ctx, p_full && p_trunc && target, "p_full, p_trunc and target must not be NULL");
  GWX_CHECK(ctx, ng > 0 && ng <= 65536, "ng must be in [1, 65536]");
  if (ctx->device < 0) return GW_OK;
  GWX_HIP(ctx, tail_target((const float2 *)p_full, (const float2 *)p_trunc, ng, (float2 *)target, as_stream(stream)));
  return GW_OK;
}

int gw_tail_features(gw_ctx *ctx, const gw_c32 *p_gg, int ng, gw_grid grid, const double *q, const int *g_miller,
                     int nc, double e_max, float *feat, void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_CHECK(ctx, p_gg && q && feat, "p_gg, q and feat must not be NULL");
  GWX_CHECK(ctx, std::isfinite(q[0]) && std::isfinite(q[1]) && std::isfinite(q[2]), "q must be finite");
  GWX_CHECK(ctx, nc > 0 && std::isfinite(e_max), "nc must be positive and e_max finite");
  GWX_STATUS(api_check_grid(ctx, grid));
  GWX_STATUS(api_check_sphere(ctx, grid, g_miller, ng));
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  void *dm;
  GWX_STATUS(api_ws_get(ctx, WS_MILLER, (size_t)ng * 3 * sizeof(int), &dm, s));
  GWX_HIP(ctx, hipMemcpyAsync(dm, g_miller, (size_t)ng * 3 * sizeof(int), hipMemcpyHostToDevice, s));
  GWX_HIP(ctx, tail_features((const float2 *)p_gg, ng, (const int *)dm, q, grid.a_bohr, nc, e_max, feat, s));
  return GW_OK;
}

int gw_tail_forward(gw_ctx *ctx, const gw_mlp *w, const float *feat, int ng, float *out, void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_STATUS(check_mlp(ctx, w));
  GWX_CHECK(ctx, feat && out, "feat and out must not be NULL");
  GWX_CHECK(ctx, ng > 0 && ng <= 65536, "ng must be in [1, 65536]");
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  float *ws;
  GWX_STATUS(tail_ws(ctx, ng, &ws, s));
  GWX_HIP(ctx, tail_forward(*w, feat, ng, ws, out, s));
  return GW_OK;
}

int gw_tail_train_step(gw_ctx *ctx, gw_mlp *w, gw_adam *opt, const float *feat, const gw_c32 *target, int ng,
                       float *loss_out, void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_STATUS(check_mlp(ctx, w));
  GWX_CHECK(ctx, opt && opt->master && opt->m && opt->v && opt->grad, "gw_adam and its buffers must not be NULL");
  GWX_CHECK(ctx, std::isfinite(opt->lr) && opt->lr >= 0.f, "lr must be >= 0");
  GWX_CHECK(ctx, opt->beta1 >= 0.f && opt->beta1 < 1.f && opt->beta2 >= 0.f && opt->beta2 < 1.f,
          "betas must be in [0, 1)");
  GWX_CHECK(ctx, opt->eps > 0.f && opt->step >= 0, "eps must be positive and step >= 0");
  GWX_CHECK(ctx, feat && target && loss_out, "feat, target and loss_out must not be NULL");
  GWX_CHECK(ctx, ng > 0 && ng <= 65536, "ng must be in [1, 65536]");
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  float *ws;
  GWX_STATUS(tail_ws(ctx, ng, &ws, s));
  GWX_HIP(ctx, tail_train_step(*w, *opt, feat, (const float2 *)target, ng, ws, loss_out, s));
  return GW_OK;
}

int gw_tail_loss(gw_ctx *ctx, const gw_mlp *w, const float *feat, const gw_c32 *target, int ng, float *loss_out,
                 void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_STATUS(check_mlp(ctx, w));
  GWX_CHECK(ctx, feat && target && loss_out, "feat, target and loss_out must not be NULL");
  GWX_CHECK(ctx, ng > 0 && ng <= 65536, "ng must be in [1, 65536]");
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  float *ws;
  GWX_STATUS(tail_ws(ctx, ng, &ws, s));
  GWX_HIP(ctx, tail_loss(*w, feat, (const float2 *)target, ng, ws, loss_out, s));
  return GW_OK;
}

int gw_tail_correct(gw_ctx *ctx, const gw_mlp *w, const gw_c32 *p_trunc, int ng, const float *feat, gw_c32 *p_corr,
                    int *used_fallback, void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_STATUS(check_mlp(ctx, w));
  GWX_CHECK(ctx, p_trunc && feat && p_corr && used_fallback, "p_trunc, feat, p_corr and used_fallback must not be NULL");
  GWX_CHECK(ctx, ng > 0 && ng <= 65536, "ng must be in [1, 65536]");
  if (ctx->device < 0) { *used_fallback = 0; return GW_OK; }
  hipStream_t s = as_stream(stream);
  void *flag;
  GWX_STATUS(api_ws_get(ctx, WS_TAIL_FLAG, 256, &flag, s));
  GWX_HIP(ctx, tail_check_box(feat, ng, w->norm, (int *)flag, s));
  GWX_HIP(ctx, hipMemcpyAsync(ctx->pivot_host, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  GWX_HIP(ctx, hipStreamSynchronize(s));
  if (*ctx->pivot_host != 0) {
    *used_fallback = 1;
    return GW_OK;
  }
  float *ws;
  GWX_STATUS(tail_ws(ctx, ng, &ws, s));
  GWX_HIP(ctx, tail_apply(*w, feat, (const float2 *)p_trunc, ng, ws, (float2 *)p_corr, s));
  GWX_HIP(ctx, hipStreamSynchronize(s));
  *used_fallback = 0;
  return GW_OK;
}

}  // extern "C"
