// C ABI of the learned band-tail correction (argument checks, workspace, the training-step graphs;
// kernels in tail.hip).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

#include "gw_internal.h"

using namespace gwi;

namespace {

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

int check_mlp(gw_ctx *ctx, const gw_mlp *w) {
  GWX_CHECK(ctx, w && w->w && w->b && w->norm, "gw_mlp and its buffers must not be NULL");
  GWX_CHECK(ctx, w->rank >= 0 && w->rank <= 16, "gw_mlp rank must be in [0, 16]");
  return GW_OK;
}

int check_adam(gw_ctx *ctx, const gw_adam *opt) {
  GWX_CHECK(ctx, opt && opt->master && opt->m && opt->v && opt->grad, "gw_adam and its buffers must not be NULL");
  GWX_CHECK(ctx, std::isfinite(opt->lr) && opt->lr >= 0.f, "lr must be >= 0");
  GWX_CHECK(ctx, opt->beta1 >= 0.f && opt->beta1 < 1.f && opt->beta2 >= 0.f && opt->beta2 < 1.f,
            "betas must be in [0, 1)");
  GWX_CHECK(ctx, opt->eps > 0.f && opt->step >= 0, "eps must be positive and step >= 0");
  return GW_OK;
}

// Small device words of the tail path, one slot of kTailSmallBytes: the training-box flag (int at byte 0),
// the Adam step counter (int at byte 64) and the feature-statistics accumulator (16 doubles at byte 128).
constexpr size_t kTailSmallBytes = 512;
int tail_small(gw_ctx *ctx, char **p, hipStream_t s) {
  void *v;
  GWX_STATUS(api_ws_get(ctx, WS_TAIL_FLAG, kTailSmallBytes, &v, s));
  *p = (char *)v;
  return GW_OK;
}

int tail_ws(gw_ctx *ctx, int n, float **ws, hipStream_t s) {
  void *p;
  GWX_STATUS(api_ws_get(ctx, WS_TAIL, tail_ws_floats(n) * sizeof(float), &p, s));
  *ws = (float *)p;
  return GW_OK;
}

// Cached training-step graphs: one per (model, optimiser, system, workspace) combination.
struct TailGraphs {
  std::map<std::vector<uint64_t>, hipGraphExec_t> execs;
  hipStream_t cs = nullptr;        // private capture stream
};

TailGraphs *tail_graphs(gw_ctx *ctx) {
  if (!ctx->tail_graphs) ctx->tail_graphs = new TailGraphs();
  return static_cast<TailGraphs *>(ctx->tail_graphs);
}

uint64_t fbits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, sizeof u);
  return u;
}

int tail_step_graph(gw_ctx *ctx, const gw_mlp &w, const gw_adam &a, const float *feat, const float2 *target, int ng,
                    float *ws, float *loss, int *step_dev, hipGraphExec_t *out) {
  TailGraphs *tg = tail_graphs(ctx);
  const std::vector<uint64_t> key = {(uint64_t)w.w, (uint64_t)w.b, (uint64_t)w.norm, (uint64_t)w.rank,
                                     (uint64_t)a.master, (uint64_t)a.m, (uint64_t)a.v, (uint64_t)a.grad,
                                     fbits(a.lr), fbits(a.beta1), fbits(a.beta2), fbits(a.eps),
                                     (uint64_t)feat, (uint64_t)target, (uint64_t)ng, (uint64_t)ws, (uint64_t)loss,
                                     (uint64_t)step_dev};
  auto it = tg->execs.find(key);
  if (it != tg->execs.end()) {
    *out = it->second;
    return GW_OK;
  }
  if (!tg->cs) GWX_HIP(ctx, hipStreamCreateWithFlags(&tg->cs, hipStreamNonBlocking));
  GWX_HIP(ctx, hipStreamBeginCapture(tg->cs, hipStreamCaptureModeThreadLocal));
  const hipError_t ce = tail_train_step(w, a, feat, target, ng, ws, loss, step_dev, -1, tg->cs);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(tg->cs, &g);
  if (ce != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    char b[200];
    snprintf(b, sizeof(b), "training-step graph capture failed: %s / %s", hipGetErrorString(ce), hipGetErrorString(ee));
    api_set_err(ctx, b);
    return GW_E_HIP;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  GWX_HIP(ctx, ie);
  tg->execs[key] = exec;
  *out = exec;
  return GW_OK;
}

int tail_graph_count(const gw_ctx *ctx) {
  return ctx && ctx->tail_graphs ? (int)static_cast<const TailGraphs *>(ctx->tail_graphs)->execs.size() : 0;
}

}  // namespace

namespace gwi {
void tail_graphs_release(gw_ctx *ctx) {
  if (!ctx->tail_graphs) return;
  TailGraphs *tg = static_cast<TailGraphs *>(ctx->tail_graphs);
  for (auto &kv : tg->execs) (void)hipGraphExecDestroy(kv.second);
  if (tg->cs) (void)hipStreamDestroy(tg->cs);
  delete tg;
  ctx->tail_graphs = nullptr;
}
}  // namespace gwi

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
  GWX_STATUS(check_adam(ctx, opt));
  GWX_CHECK(ctx, feat && target && loss_out, "feat, target and loss_out must not be NULL");
  GWX_CHECK(ctx, ng > 0 && ng <= 65536, "ng must be in [1, 65536]");
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  float *ws;
  char *small;
  GWX_STATUS(tail_ws(ctx, ng, &ws, s));
  GWX_STATUS(tail_small(ctx, &small, s));
  GWX_HIP(ctx, tail_train_step(*w, *opt, feat, (const float2 *)target, ng, ws, loss_out, (int *)(small + 64),
                               opt->step + 1, s));
  opt->step += 1;
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
  char *flag;
  GWX_STATUS(tail_small(ctx, &flag, s));
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

int gw_tail_residual_parts(gw_ctx *ctx, const gw_mlp *w, const float *feat, const gw_c32 *target, int ng, float *parts,
                           void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_STATUS(check_mlp(ctx, w));
  GWX_CHECK(ctx, feat && target && parts, "feat, target and parts must not be NULL");
  GWX_CHECK(ctx, ng > 0 && ng <= 65536, "ng must be in [1, 65536]");
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  float *ws;
  GWX_STATUS(tail_ws(ctx, ng, &ws, s));
  GWX_HIP(ctx, tail_residual_parts(*w, feat, (const float2 *)target, ng, ws, parts, s));
  return GW_OK;
}

int gw_tail_fit_norm(gw_ctx *ctx, int nsys, const float *const *feats, const int *ngs, float *norm, void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_CHECK(ctx, nsys > 0 && feats && ngs && norm, "nsys must be positive; feats, ngs and norm must not be NULL");
  for (int i = 0; i < nsys; ++i) {
    GWX_CHECK(ctx, feats[i] != nullptr, "every feature array must be non-NULL");
    GWX_CHECK(ctx, ngs[i] > 0 && ngs[i] <= 65536, "every ng must be in [1, 65536]");
  }
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  char *small;
  GWX_STATUS(tail_small(ctx, &small, s));
  GWX_HIP(ctx, tail_fit_norm(nsys, feats, ngs, (double *)(small + 128), norm, s));
  return GW_OK;
}

int gw_tail_train_steps(gw_ctx *ctx, gw_mlp *w, gw_adam *opt, int nsys, const float *const *feats,
                        const gw_c32 *const *targets, const int *ngs, int nsteps, const int *order, float *loss_out,
                        void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_STATUS(check_mlp(ctx, w));
  GWX_STATUS(check_adam(ctx, opt));
  GWX_CHECK(ctx, nsys > 0 && nsteps >= 0, "nsys must be positive and nsteps >= 0");
  GWX_CHECK(ctx, feats && targets && ngs && loss_out && (order || nsteps == 0),
            "feats, targets, ngs, order and loss_out must not be NULL");
  int ngmax = 0;
  for (int j = 0; j < nsys; ++j) {
    GWX_CHECK(ctx, feats[j] && targets[j], "every system's feat and target must be non-NULL");
    GWX_CHECK(ctx, ngs[j] > 0 && ngs[j] <= 65536, "every ng must be in [1, 65536]");
    ngmax = ngs[j] > ngmax ? ngs[j] : ngmax;
  }
  for (int k = 0; k < nsteps; ++k) GWX_CHECK(ctx, order[k] >= 0 && order[k] < nsys, "order entries must be in [0, nsys)");
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  float *ws;
  char *small;
  GWX_STATUS(tail_ws(ctx, ngmax, &ws, s));          // sized for every system before any capture
  GWX_STATUS(tail_small(ctx, &small, s));
  int *step_dev = (int *)(small + 64);
  GWX_HIP(ctx, launch_fill_int(step_dev, opt->step, s));
  for (int k = 0; k < nsteps; ++k) {
    const int j = order[k];
    hipGraphExec_t exec = nullptr;
    GWX_STATUS(tail_step_graph(ctx, *w, *opt, feats[j], (const float2 *)targets[j], ngs[j], ws, loss_out + j, step_dev,
                               &exec));
    GWX_HIP(ctx, hipGraphLaunch(exec, s));
  }
  opt->step += nsteps;
  return GW_OK;
}

int gw_tail_graph_count(const gw_ctx *ctx) { return tail_graph_count(ctx); }

}  // extern "C"
