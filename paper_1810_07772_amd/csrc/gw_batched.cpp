// Batched q-points and the tile autotuner.
//
// Every q-point is an independent build (P^q of Eq.(staticpol) is defined per q): its own
// unoccupied set, pair scales, sphere and Coulomb kernel, sharing the occupied set.  The launch
// sequence of all jobs is captured once into a HIP graph and replayed on later calls with the
// same shapes and buffers.  Two capture streams form a pipeline inside the graph: the update of
// job j+1 (into one of two P buffers) runs while the transforms, eps and the Cholesky inverse of
// job j run on the other P buffer, so the latency-bound FP64 factorisation hides under the next
// update.  Only kernels are captured (no memsets, no allocation, no host copies).
//
// The autotuner times every update tile of the requested precision on a reduced K (the same
// N_r and Nc, at most 8 occupied bands) and caches the fastest per (arch, N_r, Nv, Nc, precision)
// in the context, and in the file named by GW_AUTOTUNE_CACHE when that variable is set.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "gw_internal.h"

using namespace gwi;

namespace {

const char *kArchFallback = "gfx950";

std::string arch_name(gw_ctx *ctx) {
  if (!ctx->arch.empty()) return ctx->arch;
  hipDeviceProp_t prop;
  if (ctx->device >= 0 && hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    ctx->arch = colon == std::string::npos ? a : a.substr(0, colon);
    return ctx->arch;
  }
  return kArchFallback;
}

std::string tune_key(const std::string &arch, int nr, int nv, int nc, int precision) {
  std::ostringstream os;
  os << arch << ' ' << nr << ' ' << nv << ' ' << nc << ' ' << precision;
  return os.str();
}

void load_tune_file(gw_ctx *ctx) {
  if (ctx->tune_loaded) return;
  ctx->tune_loaded = true;
  const char *path = std::getenv("GW_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream f(path);
  std::string arch;
  int nr, nv, nc, prec, tile;
  while (f >> arch >> nr >> nv >> nc >> prec >> tile)
    if (herk_tile_supports(tile, prec)) ctx->tuned[tune_key(arch, nr, nv, nc, prec)] = tile;
}

void store_tune_file(const std::string &key, int tile) {
  const char *path = std::getenv("GW_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::app);
  f << key << ' ' << tile << '\n';
}

// Workspace slots private to the batched path (so a graph's baked-in addresses stay valid).
enum {
  BS_P0 = 64, BS_P1, BS_A1, BS_A2, BS_PH, BS_PHT, BS_Q, BS_EPS, BS_L, BS_X, BS_SMALL, BS_PIVOT, BS_Y1,
  BS_JOB_BASE = 96   // per job: 6 slots each (energies, scale, band exponents, maps, miller, sqrtv)
};
constexpr int kJobSlots = 6;
constexpr int kMaxJobs = 64;

struct Cached {
  std::string key;
  std::vector<void *> ptrs;        // workspace addresses the graph was captured with
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t sa = nullptr, sb = nullptr;
  std::vector<hipEvent_t> events;
  int *pivots_host = nullptr;
  int npiv = 0;
  int captures = 0;                // graphs captured so far (a replay does not count)
};

Cached *cache_of(gw_ctx *ctx) {
  if (!ctx->graph_cache) ctx->graph_cache = new Cached();
  return static_cast<Cached *>(ctx->graph_cache);
}

void drop_graph(Cached *c) {
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->exec = nullptr;
  c->graph = nullptr;
  c->key.clear();
  c->ptrs.clear();
}

uint64_t fnv(const void *p, size_t n, uint64_t h = 1469598103934665603ULL) {
  const unsigned char *b = static_cast<const unsigned char *>(p);
  for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ULL; }
  return h;
}

}  // namespace

namespace gwi {

int tuned_tile(gw_ctx *ctx, int nr, int nv, int nc, int precision) {
  if (!ctx || ctx->device < 0) return -1;
  load_tune_file(ctx);
  auto it = ctx->tuned.find(tune_key(arch_name(ctx), nr, nv, nc, precision));
  return it == ctx->tuned.end() ? -1 : it->second;
}

int autotune_impl(gw_ctx *ctx, const float2 *psi_v, int nv, const float2 *psi_c, int nc, int nr, const double *e_v,
                  const double *e_c, int precision, float2 *p_scratch, int *best, double *times_ms, hipStream_t s) {
  // scales of the tuning sub-problem (the first nt occupied bands)
  const int nt = std::min(nv, 8);
  const int ldsc = scale_ld(nc);
  void *eb, *sb, *bx;
  GWX_STATUS(api_ws_get(ctx, WS_ENERGY, (size_t)(nv + nc) * sizeof(double), &eb, s));
  GWX_STATUS(api_ws_get(ctx, WS_SCALE, scale_table_floats(nv, nc) * sizeof(float), &sb, s));
  GWX_STATUS(api_ws_get(ctx, WS_BSCALE, band_exp_ints(nv, nc) * sizeof(int), &bx, s));
  double *de = (double *)eb;
  GWX_HIP(ctx, hipMemcpyAsync(de, e_v, nt * sizeof(double), hipMemcpyHostToDevice, s));
  GWX_HIP(ctx, hipMemcpyAsync(de + nt, e_c, nc * sizeof(double), hipMemcpyHostToDevice, s));
  GWX_HIP(ctx, launch_scale_table(de, nt, de + nt, nc, 1.0, (float *)sb, ldsc, s));
  GWX_HIP(ctx, launch_band_exponents(psi_v, nt, psi_c, nc, nr, (const float *)sb, ldsc, (int *)bx, s));
  float2 *pb = p_scratch;
  hipEvent_t e0, e1;
  GWX_HIP(ctx, hipEventCreate(&e0));
  GWX_HIP(ctx, hipEventCreate(&e1));
  int bt = -1;
  float bms = 0.f;
  for (int t = 0; t < herk_tile_count(); ++t) {
    if (times_ms) times_ms[t] = -1.0;
    if (!herk_tile_supports(t, precision)) continue;
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {       // first launch warms caches and code
      GWX_HIP(ctx, hipEventRecord(e0, s));
      GWX_HIP(ctx, launch_herk(precision, t, psi_v, psi_c, (const float *)sb, ldsc, (const int *)bx, (float2 *)pb, nr,
                             nt, nc, 0, s));   // writes the whole P scratch
      GWX_HIP(ctx, hipEventRecord(e1, s));
      GWX_HIP(ctx, hipEventSynchronize(e1));
      GWX_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
    }
    if (times_ms) times_ms[t] = ms;
    if (bt < 0 || ms < bms) { bt = t; bms = ms; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (bt < 0) { api_set_err(ctx, "no tile implements this precision"); return GW_E_UNSUPPORTED; }
  load_tune_file(ctx);
  const std::string key = tune_key(arch_name(ctx), nr, nv, nc, precision);
  ctx->tuned[key] = bt;
  store_tune_file(key, bt);
  *best = bt;
  return GW_OK;
}

void batched_release(gw_ctx *ctx) {
  if (!ctx->graph_cache) return;
  Cached *c = static_cast<Cached *>(ctx->graph_cache);
  drop_graph(c);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  if (c->sa) (void)hipStreamDestroy(c->sa);
  if (c->sb) (void)hipStreamDestroy(c->sb);
  if (c->pivots_host) (void)hipHostFree(c->pivots_host);
  delete c;
  ctx->graph_cache = nullptr;
}

}  // namespace gwi

extern "C" {

int gw_autotune(gw_ctx *ctx, const gw_c32 *psi_v, int nv, const gw_c32 *psi_c, int nc, int nr, const double *e_v,
                const double *e_c, int precision, gw_c32 *p_scratch, int *best_tile, double *times_ms, void *stream) {
  GWX_STATUS(api_begin(ctx));
  GWX_CHECK(ctx, psi_v && psi_c && best_tile && p_scratch, "psi_v, psi_c, p_scratch and best_tile must not be NULL");
  GWX_CHECK(ctx, nv > 0 && nc > 0 && nr > 0 && nr <= (1 << 24), "nv, nc, nr out of range");
  gw_opts o;
  gw_opts_default(&o);
  o.precision = precision;
  GWX_STATUS(api_check_opts(ctx, &o));
  GWX_STATUS(api_check_energies(ctx, e_v, nv, e_c, nc));
  if (ctx->device < 0) { *best_tile = -1; return GW_OK; }
  return autotune_impl(ctx, (const float2 *)psi_v, nv, (const float2 *)psi_c, nc, nr, e_v, e_c, precision,
                       (float2 *)p_scratch, best_tile, times_ms, reinterpret_cast<hipStream_t>(stream));
}

int gw_graph_captures(const gw_ctx *ctx) {
  if (!ctx || !ctx->graph_cache) return 0;
  return static_cast<const Cached *>(ctx->graph_cache)->captures;
}

int gw_polarizability_batched(gw_ctx *ctx, const gw_c32 *psi_occ, int nv, const double *e_v, gw_grid grid, int nq,
                              const gw_qjob *jobs, const gw_opts *opts, double head, void *stream) {
  GWX_STATUS(api_begin(ctx));
  gw_opts o;
  gw_opts_default(&o);
  if (opts) o = *opts;
  GWX_CHECK(ctx, nq > 0 && nq <= kMaxJobs, "nq must be in [1, 64]");
  GWX_CHECK(ctx, jobs != nullptr && psi_occ != nullptr && e_v != nullptr, "jobs, psi_occ and e_v must not be NULL");
  GWX_CHECK(ctx, nv > 0, "nv must be positive");
  GWX_CHECK(ctx, o.accumulate == 0, "accumulate is not available for batched builds");
  GWX_STATUS(api_check_opts(ctx, &o));
  GWX_STATUS(api_check_grid(ctx, grid));
  const long long nrl = (long long)grid.n1 * grid.n2 * grid.n3;
  GWX_CHECK(ctx, nrl <= (1 << 24), "grid too large");
  const int nr = (int)nrl;
  if (std::isnan(head)) head = 1.0;
  GWX_CHECK(ctx, std::isfinite(head) && head > 0.0, "head must be positive");
  for (int j = 0; j < nq; ++j) {
    const gw_qjob &jb = jobs[j];
    GWX_CHECK(ctx, jb.psi_unocc && jb.p_gg && jb.e_c && jb.g_miller, "job pointers must not be NULL (eps_inv may be)");
    GWX_CHECK(ctx, jb.nc > 0 && (long long)nv * jb.nc <= (1LL << 31), "job nc out of range");
    GWX_CHECK(ctx, std::isfinite(jb.q[0]) && std::isfinite(jb.q[1]) && std::isfinite(jb.q[2]), "q must be finite");
    GWX_STATUS(api_check_energies(ctx, e_v, nv, jb.e_c, jb.nc));
    GWX_STATUS(api_check_sphere(ctx, grid, jb.g_miller, jb.ng));
  }
  GWX_STATUS(api_grid_supported(ctx, grid));
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);

  // ---- plans, tiles and workspace (all before any capture) ---------------------------------
  std::vector<SpherePlan> plans(nq);
  std::vector<int> tiles(nq);
  size_t a1 = 0, a2 = 0, ngmax = 0, y1 = 0;
  for (int j = 0; j < nq; ++j) {
    build_sphere_plan(grid, jobs[j].g_miller, jobs[j].ng, plans[j]);
    a1 = std::max(a1, plans[j].a1_elems);
    a2 = std::max(a2, plans[j].a2_elems);
    y1 = std::max(y1, plans[j].y1_elems);
    ngmax = std::max(ngmax, (size_t)jobs[j].ng);
  }
  const int np = nq > 1 ? 2 : 1;
  void *pbuf[2] = {nullptr, nullptr};
  std::vector<void *> ptrs;
  for (int b = 0; b < np; ++b) {
    GWX_STATUS(api_ws_get(ctx, BS_P0 + b, (size_t)nr * nr * sizeof(float2), &pbuf[b], s));
    ptrs.push_back(pbuf[b]);
  }
  for (int j = 0; j < nq; ++j) {
    int t = o.tile;
    if (t < 0) t = tuned_tile(ctx, nr, nv, jobs[j].nc, o.precision);
    if (t < 0) {
      GWX_STATUS(autotune_impl(ctx, (const float2 *)psi_occ, nv, (const float2 *)jobs[j].psi_unocc, jobs[j].nc, nr, e_v,
                             jobs[j].e_c, o.precision, (float2 *)pbuf[0], &t, nullptr, s));
    }
    tiles[j] = t;
  }
  void *wa1, *wa2, *wph, *wpht = nullptr, *wq, *weps, *wl, *wx, *wsmall, *wpiv, *wy1 = nullptr;
  GWX_STATUS(api_ws_get(ctx, BS_A1, a1 * sizeof(float2), &wa1, s));
  GWX_STATUS(api_ws_get(ctx, BS_A2, a2 * sizeof(float2), &wa2, s));
  GWX_STATUS(api_ws_get(ctx, BS_PH, ngmax * nr * sizeof(float2), &wph, s));
  // the row-contiguous transform (every job shares the grid, so all or none of the plans use it)
  if (plans[0].plane) GWX_STATUS(api_ws_get(ctx, BS_Y1, y1 * sizeof(float2), &wy1, s));
  else GWX_STATUS(api_ws_get(ctx, BS_PHT, ngmax * nr * sizeof(float2), &wpht, s));
  GWX_STATUS(api_ws_get(ctx, BS_Q, ngmax * ngmax * sizeof(float2), &wq, s));
  GWX_STATUS(api_ws_get(ctx, BS_EPS, ngmax * ngmax * sizeof(double2), &weps, s));
  GWX_STATUS(api_ws_get(ctx, BS_L, ngmax * ngmax * sizeof(double2), &wl, s));
  GWX_STATUS(api_ws_get(ctx, BS_X, ngmax * ngmax * sizeof(double2), &wx, s));
  GWX_STATUS(api_ws_get(ctx, BS_SMALL, chol_small_bytes((int)ngmax), &wsmall, s));
  GWX_STATUS(api_ws_get(ctx, BS_PIVOT, (size_t)nq * 64, &wpiv, s));
  for (void *p : {wa1, wa2, wph, wpht, wq, weps, wl, wx, wsmall, wpiv, wy1}) ptrs.push_back(p);
  struct JobDev { double *energy; float *scale; int *bexp; int *maps; int *miller; double *sqrtv; };
  std::vector<JobDev> jd(nq);
  for (int j = 0; j < nq; ++j) {
    const int nc = jobs[j].nc, ng = jobs[j].ng;
    const SpherePlan &pl = plans[j];
    void *p[kJobSlots];
    const size_t bytes[kJobSlots] = {(size_t)(nv + nc) * sizeof(double), scale_table_floats(nv, nc) * sizeof(float),
                                     band_exp_ints(nv, nc) * sizeof(int),
                                     pl.maps_ints() * sizeof(int),
                                     (size_t)ng * 3 * sizeof(int), (size_t)ng * sizeof(double)};
    for (int k = 0; k < kJobSlots; ++k) {
      GWX_STATUS(api_ws_get(ctx, BS_JOB_BASE + kJobSlots * j + k, bytes[k], &p[k], s));
      ptrs.push_back(p[k]);
    }
    jd[j] = {(double *)p[0], (float *)p[1], (int *)p[2], (int *)p[3], (int *)p[4], (double *)p[5]};
  }

  // ---- host inputs to device (every call; the graph reads these buffers) ----------------------
  for (int j = 0; j < nq; ++j) {
    const gw_qjob &jb = jobs[j];
    const SpherePlan &pl = plans[j];
    GWX_HIP(ctx, hipMemcpyAsync(jd[j].energy, e_v, nv * sizeof(double), hipMemcpyHostToDevice, s));
    GWX_HIP(ctx, hipMemcpyAsync(jd[j].energy + nv, jb.e_c, jb.nc * sizeof(double), hipMemcpyHostToDevice, s));
    int *m = jd[j].maps;
    GWX_HIP(ctx, hipMemcpyAsync(m, pl.mapA.data(), pl.mapA.size() * sizeof(int), hipMemcpyHostToDevice, s));
    m += pl.mapA.size();
    GWX_HIP(ctx, hipMemcpyAsync(m, pl.mapB.data(), pl.mapB.size() * sizeof(int), hipMemcpyHostToDevice, s));
    m += pl.mapB.size();
    GWX_HIP(ctx, hipMemcpyAsync(m, pl.mapC.data(), pl.mapC.size() * sizeof(int), hipMemcpyHostToDevice, s));
    m += pl.mapC.size();
    for (const std::vector<int> *v : {&pl.mapK2, &pl.mapAB, &pl.mapCT}) {
      if (!v->empty()) GWX_HIP(ctx, hipMemcpyAsync(m, v->data(), v->size() * sizeof(int), hipMemcpyHostToDevice, s));
      m += v->size();
    }
    GWX_HIP(ctx, hipMemcpyAsync(jd[j].miller, jb.g_miller, (size_t)jb.ng * 3 * sizeof(int), hipMemcpyHostToDevice, s));
  }

  // ---- graph key: everything baked into the captured launches ---------------------------------
  // (field by field: the option and grid structs have padding bytes whose contents are undefined)
  uint64_t h = fnv(&nv, sizeof nv);
  h = fnv(&grid.n1, sizeof grid.n1, h);
  h = fnv(&grid.n2, sizeof grid.n2, h);
  h = fnv(&grid.n3, sizeof grid.n3, h);
  h = fnv(&grid.a_bohr, sizeof grid.a_bohr, h);
  h = fnv(&nq, sizeof nq, h);
  h = fnv(&o.precision, sizeof o.precision, h);
  h = fnv(&o.prefactor, sizeof o.prefactor, h);
  h = fnv(&o.accumulate, sizeof o.accumulate, h);
  h = fnv(&o.tile, sizeof o.tile, h);
  h = fnv(&head, sizeof head, h);
  h = fnv(&psi_occ, sizeof psi_occ, h);
  h = fnv(tiles.data(), tiles.size() * sizeof(int), h);
  for (int j = 0; j < nq; ++j) {
    const gw_qjob &jb = jobs[j];
    h = fnv(&jb.psi_unocc, sizeof jb.psi_unocc, h);
    h = fnv(&jb.nc, sizeof jb.nc, h);
    h = fnv(jb.q, sizeof jb.q, h);
    h = fnv(&jb.ng, sizeof jb.ng, h);
    h = fnv(jb.g_miller, (size_t)jb.ng * 3 * sizeof(int), h);
    h = fnv(&jb.p_gg, sizeof jb.p_gg, h);
    h = fnv(&jb.eps_inv, sizeof jb.eps_inv, h);
  }
  const std::string key = std::to_string(h);

  Cached *c = cache_of(ctx);
  if (c->key != key || c->ptrs != ptrs || !c->exec) {
    drop_graph(c);
    if (!c->sa) GWX_HIP(ctx, hipStreamCreateWithFlags(&c->sa, hipStreamNonBlocking));
    if (!c->sb) GWX_HIP(ctx, hipStreamCreateWithFlags(&c->sb, hipStreamNonBlocking));
    const size_t nev = 2 + 2 * (size_t)nq;
    while (c->events.size() < nev) {
      hipEvent_t e;
      GWX_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      c->events.push_back(e);
    }
    hipEvent_t ev_fork = c->events[0], ev_join = c->events[1];
    hipEvent_t *ev_herk = &c->events[2], *ev_post = &c->events[2 + nq];
    // the capture hangs off sa; sa waits for the caller's stream so uploads precede the replay
    GWX_HIP(ctx, hipStreamBeginCapture(c->sa, hipStreamCaptureModeThreadLocal));
    hipError_t ce = hipSuccess;
    auto ck = [&](hipError_t e) { if (ce == hipSuccess && e != hipSuccess) ce = e; };
    ck(hipEventRecord(ev_fork, c->sa));
    ck(hipStreamWaitEvent(c->sb, ev_fork, 0));
    for (int j = 0; j < nq && ce == hipSuccess; ++j) {
      const gw_qjob &jb = jobs[j];
      const int nc = jb.nc, ng = jb.ng, ldsc = scale_ld(nc);
      float2 *pj = (float2 *)pbuf[j % np];
      // update chain (sa): P buffer j%2 is free once job j-2's transforms have read it
      if (j >= np) ck(hipStreamWaitEvent(c->sa, ev_post[j - np], 0));
      ck(launch_scale_table(jd[j].energy, nv, jd[j].energy + nv, nc, o.prefactor, jd[j].scale, ldsc, c->sa));
      if (o.precision == GW_SPLIT_FP16_SCALED)
        ck(launch_band_exponents((const float2 *)psi_occ, nv, (const float2 *)jb.psi_unocc, nc, nr, jd[j].scale, ldsc,
                                 jd[j].bexp, c->sa));
      ck(launch_herk(o.precision, tiles[j], (const float2 *)psi_occ, (const float2 *)jb.psi_unocc, jd[j].scale, ldsc,
                     jd[j].bexp, pj, nr, nv, nc, 0, c->sa));
      ck(hipEventRecord(ev_herk[j], c->sa));
      // transform / eps / inverse chain (sb)
      ck(hipStreamWaitEvent(c->sb, ev_herk[j], 0));
      const SpherePlan &pl = plans[j];
      const int *dA = jd[j].maps, *dB = dA + pl.mapA.size(), *dC = dB + pl.mapB.size();
      const int *dK = dC + pl.mapC.size(), *dAB = dK + pl.mapK2.size(), *dCT = dAB + pl.mapAB.size();
      SphereBuffers sbuf{(float2 *)wa1, (float2 *)wa2, (float2 *)wph, (float2 *)wpht, (float2 *)wq, dA, dB, dC,
                         (float2 *)wy1, dK, dAB, dCT};
      ck(enqueue_sphere_transform(pl, sbuf, pj, (float2 *)jb.p_gg, triangle_form_suits(jb.q, jb.g_miller, ng), c->sb));
      if (jb.eps_inv) {
        ck(launch_sqrtv(jd[j].miller, ng, jb.q[0], jb.q[1], jb.q[2], grid.a_bohr, jd[j].sqrtv, c->sb));
        ck(launch_eps_build((const float2 *)jb.p_gg, ng, jd[j].sqrtv, head, (double2 *)weps, c->sb));
        ck(hpd_inverse((double2 *)weps, ng, (double2 *)wl, (double2 *)wx, (double2 *)wsmall,
                       (int *)((char *)wpiv + 64 * j), (double2 *)jb.eps_inv, c->sb));
      }
      ck(hipEventRecord(ev_post[j], c->sb));
    }
    ck(hipStreamWaitEvent(c->sa, ev_post[nq - 1], 0));
    ck(hipEventRecord(ev_join, c->sa));
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(c->sa, &g);
    if (ce != hipSuccess || ee != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      char b[256];
      snprintf(b, sizeof(b), "graph capture failed: %s / %s", hipGetErrorString(ce), hipGetErrorString(ee));
      api_set_err(ctx, b);
      return GW_E_HIP;
    }
    c->graph = g;
    GWX_HIP(ctx, hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0));
    c->key = key;
    c->ptrs = ptrs;
    ++c->captures;
  }
  if (c->npiv < nq) {
    if (c->pivots_host) (void)hipHostFree(c->pivots_host);
    c->pivots_host = nullptr;
    GWX_HIP(ctx, hipHostMalloc((void **)&c->pivots_host, (size_t)nq * sizeof(int), hipHostMallocDefault));
    c->npiv = nq;
  }
  GWX_HIP(ctx, hipGraphLaunch(c->exec, s));
  for (int j = 0; j < nq; ++j) {
    c->pivots_host[j] = 0;
    if (jobs[j].eps_inv)
      GWX_HIP(ctx, hipMemcpyAsync(&c->pivots_host[j], (char *)wpiv + 64 * j, sizeof(int), hipMemcpyDeviceToHost, s));
  }
  GWX_HIP(ctx, hipStreamSynchronize(s));
  for (int j = 0; j < nq; ++j) {
    if (c->pivots_host[j] != 0) {
      char b[160];
      snprintf(b, sizeof(b), "job %d: eps is not positive definite: pivot %d (1-based) is not positive", j,
               c->pivots_host[j]);
      api_set_err(ctx, b);
      return GW_E_NOTPD;
    }
  }
  return GW_OK;
}

}  // extern "C"
