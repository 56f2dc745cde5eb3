// Host side of the C ABI declared in include/gw.h: argument checks, workspace, planning of
// the sphere transforms, and the launch sequences.  No device work is queued before every
// argument check of a call has passed.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <utility>
#include <vector>

#include "gw_internal.h"

using namespace gwi;

namespace {

struct Fail {
  int status;
};

void set_err(gw_ctx *ctx, const char *fmt, ...) {
  if (!ctx) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  ctx->err = buf;
}

#define GW_CHECK(ctx, cond, ...)                 \
  do {                                           \
    if (!(cond)) {                               \
      set_err((ctx), __VA_ARGS__);               \
      return GW_E_INVAL;                         \
    }                                            \
  } while (0)

#define GW_HIP(ctx, call)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      set_err((ctx), "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
      return GW_E_HIP;                                                                        \
    }                                                                                         \
  } while (0)

#define GW_STATUS(expr)            \
  do {                             \
    int st_ = (expr);              \
    if (st_ != GW_OK) return st_;  \
  } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// grow-only workspace slot
int ws_get(gw_ctx *ctx, int slot, size_t bytes, void **out, hipStream_t s) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~(size_t)255;
  if ((int)ctx->slots.size() <= slot) ctx->slots.resize(slot + 1);
  gw_ctx::Slot &sl = ctx->slots[slot];
  if (sl.bytes >= bytes) { *out = sl.ptr; return GW_OK; }
  const size_t next = ctx->held - sl.bytes + bytes;
  if (ctx->cap && next > ctx->cap) {
    set_err(ctx, "workspace cap exceeded: need %zu bytes in total, cap %zu", next, ctx->cap);
    return GW_E_NOMEM;
  }
  if (sl.ptr) {
    GW_HIP(ctx, hipStreamSynchronize(s));
    GW_HIP(ctx, hipFree(sl.ptr));
    ctx->held -= sl.bytes;
    sl.ptr = nullptr;
    sl.bytes = 0;
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_err(ctx, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    return GW_E_NOMEM;
  }
  sl.ptr = p;
  sl.bytes = bytes;
  ctx->held += bytes;
  *out = p;
  return GW_OK;
}

int begin(gw_ctx *ctx) {
  if (!ctx) return GW_E_INVAL;
  ctx->err.clear();
  if (ctx->device >= 0) GW_HIP(ctx, hipSetDevice(ctx->device));
  return GW_OK;
}

int check_energies(gw_ctx *ctx, const double *e_v, int nv, const double *e_c, int nc) {
  GW_CHECK(ctx, e_v && e_c, "energy arrays must not be NULL");
  double vmax = -std::numeric_limits<double>::infinity(), cmin = std::numeric_limits<double>::infinity();
  for (int i = 0; i < nv; ++i) {
    GW_CHECK(ctx, std::isfinite(e_v[i]), "e_v[%d] is not finite", i);
    vmax = std::max(vmax, e_v[i]);
  }
  for (int i = 0; i < nc; ++i) {
    GW_CHECK(ctx, std::isfinite(e_c[i]), "e_c[%d] is not finite", i);
    cmin = std::min(cmin, e_c[i]);
  }
  GW_CHECK(ctx, cmin - vmax > 0.0, "every E_c - E_v must be > 0 (max E_v = %.17g, min E_c = %.17g)", vmax, cmin);
  return GW_OK;
}

int check_bands(gw_ctx *ctx, const void *psi_v, int nv, const void *psi_c, int nc, int nr) {
  GW_CHECK(ctx, nv > 0 && nc > 0 && nr > 0, "nv, nc and nr must be positive (got %d, %d, %d)", nv, nc, nr);
  GW_CHECK(ctx, psi_v && psi_c, "orbital pointers must not be NULL");
  GW_CHECK(ctx, (long long)nv * nc <= (long long)1 << 31, "nv*nc too large");
  GW_CHECK(ctx, nr <= 1 << 24, "nr too large");
  return GW_OK;
}

int check_grid(gw_ctx *ctx, gw_grid g) {
  GW_CHECK(ctx, g.n1 > 0 && g.n2 > 0 && g.n3 > 0, "grid sides must be positive");
  GW_CHECK(ctx, std::isfinite(g.a_bohr) && g.a_bohr > 0.0, "a_bohr must be positive");
  return GW_OK;
}

int check_sphere(gw_ctx *ctx, gw_grid g, const int *miller, int ng) {
  GW_CHECK(ctx, miller != nullptr, "g_miller must not be NULL");
  const long long nr = (long long)g.n1 * g.n2 * g.n3;
  GW_CHECK(ctx, ng > 0 && ng <= nr, "ng must be in [1, nr] (got %d)", ng);
  const size_t nm = (size_t)ng * 3;
  // a sphere that passed before on this grid passes again without the scan (a step checks the same
  // few spheres on every call)
  for (const gw_ctx::SphereSeen &v : ctx->spheres_ok)
    if (v.n1 == g.n1 && v.n2 == g.n2 && v.n3 == g.n3 && v.miller.size() == nm &&
        std::equal(miller, miller + nm, v.miller.begin()))
      return GW_OK;
  const int n[3] = {g.n1, g.n2, g.n3};
  std::vector<std::pair<long long, int>> keys((size_t)ng);
  for (int i = 0; i < ng; ++i) {
    long long key = 0;
    for (int d = 0; d < 3; ++d) {
      const int m = miller[3 * i + d];
      GW_CHECK(ctx, 2LL * std::llabs((long long)m) < n[d], "g_miller[%d][%d] = %d violates |m| < n/2 (n = %d)", i, d, m,
               n[d]);
      key = key * n[d] + (m < 0 ? m + n[d] : m);
    }
    keys[(size_t)i] = {key, i};
  }
  // equal keys sort together in index order; every member of a run after its first repeats an earlier G
  std::sort(keys.begin(), keys.end());
  int first_dup = -1;
  for (size_t j = 1; j < keys.size(); ++j)
    if (keys[j].first == keys[j - 1].first && (first_dup < 0 || keys[j].second < first_dup)) first_dup = keys[j].second;
  GW_CHECK(ctx, first_dup < 0, "g_miller[%d] duplicates an earlier G", first_dup);
  if (ng > (1 << 20)) return GW_OK;   // spheres this large are checked on every call rather than copied
  gw_ctx::SphereSeen &slot = ctx->spheres_ok[ctx->spheres_next];
  ctx->spheres_next = (ctx->spheres_next + 1) % (int)(sizeof(ctx->spheres_ok) / sizeof(ctx->spheres_ok[0]));
  slot.n1 = g.n1;
  slot.n2 = g.n2;
  slot.n3 = g.n3;
  slot.miller.assign(miller, miller + nm);
  return GW_OK;
}

int check_q(gw_ctx *ctx, const double *q) {
  GW_CHECK(ctx, q != nullptr, "q must not be NULL");
  GW_CHECK(ctx, std::isfinite(q[0]) && std::isfinite(q[1]) && std::isfinite(q[2]), "q must be finite");
  return GW_OK;
}

int check_opts(gw_ctx *ctx, const gw_opts *o) {
  GW_CHECK(ctx, o->precision == GW_FP32 || o->precision == GW_SPLIT_BF16 || o->precision == GW_SPLIT_FP16_SCALED,
           "unknown precision %d", o->precision);
  GW_CHECK(ctx, std::isfinite(o->prefactor) && o->prefactor > 0.0, "prefactor must be positive");
  GW_CHECK(ctx, o->accumulate == 0 || o->accumulate == 1, "accumulate must be 0 or 1");
  if (o->tile >= 0)
    GW_CHECK(ctx, herk_tile_supports(o->tile, o->precision), "tile %d does not implement precision %d", o->tile,
             o->precision);
  return GW_OK;
}

}  // namespace

// --------------------------------------------------------------------------------------------
// Sphere-transform plan: output-row maps of the three passes (see fft.hip).
// --------------------------------------------------------------------------------------------
namespace gwi {

void build_sphere_plan(gw_grid g, const int *miller, int ng, SpherePlan &p) {
  p.n1 = g.n1; p.n2 = g.n2; p.n3 = g.n3; p.ng = ng;
  p.m3count = 0; p.npair = 0;
  std::vector<int> idx3(g.n3, -1);
  std::vector<int> k1s(ng), k2s(ng), k3s(ng);
  for (int i = 0; i < ng; ++i) {
    k1s[i] = ((miller[3 * i] % g.n1) + g.n1) % g.n1;
    k2s[i] = ((miller[3 * i + 1] % g.n2) + g.n2) % g.n2;
    k3s[i] = ((miller[3 * i + 2] % g.n3) + g.n3) % g.n3;
  }
  for (int i = 0; i < ng; ++i) idx3[k3s[i]] = 0;
  for (int k = 0; k < g.n3; ++k)
    if (idx3[k] == 0) idx3[k] = p.m3count++;
  // (k2, j3) pairs present in the sphere
  std::vector<int> pair(g.n2 * p.m3count, -1);
  for (int i = 0; i < ng; ++i) pair[k2s[i] * p.m3count + idx3[k3s[i]]] = 0;
  for (size_t i = 0; i < pair.size(); ++i)
    if (pair[i] == 0) pair[i] = p.npair++;
  // pass A: o = (i1, i2) in n1*n2, U = 1, axis n3
  p.mapA.assign((size_t)g.n1 * g.n2 * g.n3, -1);
  for (int o = 0; o < g.n1 * g.n2; ++o)
    for (int k = 0; k < g.n3; ++k)
      if (idx3[k] >= 0) p.mapA[(size_t)o * g.n3 + k] = o * p.m3count + idx3[k];
  // pass B: o = i1, U = m3count, axis n2
  p.mapB.assign((size_t)g.n1 * p.m3count * g.n2, -1);
  for (int o = 0; o < g.n1; ++o)
    for (int u = 0; u < p.m3count; ++u)
      for (int k = 0; k < g.n2; ++k) {
        const int pi = pair[k * p.m3count + u];
        if (pi >= 0) p.mapB[((size_t)o * p.m3count + u) * g.n2 + k] = o * p.npair + pi;
      }
  // pass C: o = 0, U = npair, axis n1 -> sphere index
  p.mapC.assign((size_t)p.npair * g.n1, -1);
  for (int i = 0; i < ng; ++i) {
    const int pi = pair[k2s[i] * p.m3count + idx3[k3s[i]]];
    p.mapC[(size_t)pi * g.n1 + k1s[i]] = i;
  }
  // column chunk of the row passes so that the first intermediate stays near 1 GiB
  const long long nr = (long long)g.n1 * g.n2 * g.n3;
  const long long rowsA = (long long)g.n1 * g.n2 * p.m3count;
  // (smaller chunks that keep the intermediates in the 256 MB last-level cache measured slower: every
  // pass already streams near HBM speed, and more chunks add launches)
  long long bc = std::max<long long>(256, std::min<long long>(nr, (1LL << 27) / std::max<long long>(1, rowsA)));
  bc = std::min<long long>(nr, (bc + 255) / 256 * 256);      // whole 256-lane blocks
  p.bc = (int)std::min<long long>(bc, nr);
  p.a1_elems = (size_t)rowsA * p.bc;
  p.a2_elems = (size_t)g.n1 * p.npair * p.bc;
  // row-contiguous form: the k2 values with sphere pairs, (k2, k3) -> pair slot, (k1, pair) -> sphere index
  p.mapK2.clear(); p.mapAB.clear(); p.mapCT.clear();
  p.plane = plane_path_supported(g.n2, g.n3);
  p.nk2 = 0;
  p.y1_elems = 0;
  if (p.plane) {
    for (int k2 = 0; k2 < g.n2; ++k2) {
      bool any = false;
      for (int j = 0; j < p.m3count; ++j) any = any || pair[k2 * p.m3count + j] >= 0;
      if (any) p.mapK2.push_back(k2);
    }
    p.nk2 = (int)p.mapK2.size();
    p.mapK2.resize((size_t)p.nk2 + g.n2, -1);                  // then the slot of each k2 (-1: no pair)
    for (int sl = 0; sl < p.nk2; ++sl) p.mapK2[(size_t)p.nk2 + p.mapK2[sl]] = sl;
    p.mapAB.assign((size_t)p.nk2 * g.n3, -1);
    for (int sl = 0; sl < p.nk2; ++sl)
      for (int k3 = 0; k3 < g.n3; ++k3)
        if (idx3[k3] >= 0) p.mapAB[(size_t)sl * g.n3 + k3] = pair[p.mapK2[sl] * p.m3count + idx3[k3]];
    p.mapCT.assign((size_t)g.n1 * p.npair, -1);
    for (int pi = 0; pi < p.npair; ++pi)
      for (int k1 = 0; k1 < g.n1; ++k1) p.mapCT[(size_t)k1 * p.npair + pi] = p.mapC[(size_t)pi * g.n1 + k1];
    p.y1_elems = (size_t)nr * g.n1 * p.npair;
  }
}

// One 3-D transform over the row index of `in` ([nr][B], row stride ld_in) to `out` ([ng][B],
// row stride ld_out), in column chunks of at most bc.
hipError_t transform_rows(const SpherePlan &p, int sign, const float2 *in, long long ld_in, int B, float2 *out,
                                 long long ld_out, float2 *a1, float2 *a2, int bc, const int *dA, const int *dB,
                                 const int *dC, hipStream_t s) {
  for (int b0 = 0; b0 < B; b0 += bc) {
    const int w = std::min(bc, B - b0);
    hipError_t e;
    if ((e = launch_fft_pass(p.n3, sign, in + b0, a1, p.n1 * p.n2, 1, w, ld_in, w, dA, s)) != hipSuccess) return e;
    if ((e = launch_fft_pass(p.n2, sign, a1, a2, p.n1, p.m3count, w, w, w, dB, s)) != hipSuccess) return e;
    if ((e = launch_fft_pass(p.n1, sign, a2, out + b0, 1, p.npair, w, w, ld_out, dC, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t enqueue_sphere_transform(const SpherePlan &p, const SphereBuffers &b, const float2 *p_rr, float2 *p_gg,
                                    bool herm, hipStream_t s) {
  const int nr = p.n1 * p.n2 * p.n3, ng = p.ng;
  hipError_t e;
  if (p.plane && b.y1) {
    // rows of M (P itself, or for a Hermitian P its upper triangle with half the diagonal), contiguous:
    // Y[r][g'] = sum_r' M(r, r') exp(+i G'.r')
    if ((e = launch_plane_ab(p.n3, herm, p_rr, nr, nr, p.n1, b.dK2 + p.nk2, p.nk2, b.dAB, p.npair, b.y1, s)) !=
        hipSuccess)
      return e;
    if ((e = launch_plane_c(p.n1, herm, b.y1, nr, p.n2 * p.n3, p.npair, b.dCT, ng, b.ph, ng, s)) != hipSuccess)
      return e;
    // X(g, g') = sum_r exp(-i G.r) Y[r][g'], then P~ = X (general P) or X + X^H (P = M + M^H)
    float2 *x = herm ? b.q : p_gg;
    if ((e = transform_rows(p, -1, b.ph, ng, ng, x, ng, b.a1, b.a2, std::min(p.bc, ng), b.dA, b.dB, b.dC, s)) !=
        hipSuccess)
      return e;
    return herm ? launch_add_adjoint(b.q, ng, p_gg, s) : hipSuccess;
  }
  // rows: P^(g, r') = sum_r exp(-i G.r) P(r, r')
  if ((e = transform_rows(p, -1, p_rr, nr, nr, b.ph, nr, b.a1, b.a2, p.bc, b.dA, b.dB, b.dC, s)) != hipSuccess) return e;
  // columns: transpose, then Q(g', g) = sum_r' exp(+i G'.r') P^T(r', g), and p_gg = Q^T
  if ((e = launch_transpose_c64(b.ph, b.pht, ng, nr, nr, ng, s)) != hipSuccess) return e;
  if ((e = transform_rows(p, +1, b.pht, ng, ng, b.q, ng, b.a1, b.a2, std::min(p.bc, ng), b.dA, b.dB, b.dC, s)) !=
      hipSuccess)
    return e;
  return launch_transpose_c64(b.q, p_gg, ng, ng, ng, ng, s);
}

// The plan's sizes and the device addresses of its maps in `map_slot`.  A call with the grid, Miller
// list and stream of the slot's previous upload reuses the device maps: no host rebuild, and no
// pageable copy that would stall the stream.  `p` receives the plan's sizes (its host maps stay empty).
int upload_plan(gw_ctx *ctx, gw_grid g, const int *miller, int ng, int map_slot, SpherePlan &p, int **dA, int **dB,
                int **dC, hipStream_t s, const int **extra) {
  std::unique_ptr<PlanCacheEntry> &e = ctx->plans[map_slot];
  const size_t nm = (size_t)ng * 3;
  const bool same = e && e->g.n1 == g.n1 && e->g.n2 == g.n2 && e->g.n3 == g.n3 && e->miller.size() == nm &&
                    std::equal(miller, miller + nm, e->miller.begin()) && e->stream == (void *)s;
  if (!same) {
    e.reset(new (std::nothrow) PlanCacheEntry());
    if (!e) {
      set_err(ctx, "out of host memory for the sphere plan");
      return GW_E_NOMEM;
    }
    build_sphere_plan(g, miller, ng, e->plan);
    e->g = g;
    e->miller.assign(miller, miller + nm);
    e->stream = (void *)s;
  }
  const SpherePlan &pl = e->plan;
  const size_t nA = pl.mapA.size(), nB = pl.mapB.size(), nC = pl.mapC.size();
  const size_t nK = pl.mapK2.size(), nAB = pl.mapAB.size(), nCT = pl.mapCT.size();
  void *maps;
  GW_STATUS(ws_get(ctx, map_slot, pl.maps_ints() * sizeof(int), &maps, s));
  *dA = (int *)maps;
  *dB = *dA + nA;
  *dC = *dB + nB;
  int *dK = *dC + nC, *dAB = dK + nK, *dCT = dAB + nAB;
  if (!same || maps != e->maps) {
    e->maps = nullptr;   // not valid until every copy below is queued
    GW_HIP(ctx, hipMemcpyAsync(*dA, pl.mapA.data(), nA * sizeof(int), hipMemcpyHostToDevice, s));
    GW_HIP(ctx, hipMemcpyAsync(*dB, pl.mapB.data(), nB * sizeof(int), hipMemcpyHostToDevice, s));
    GW_HIP(ctx, hipMemcpyAsync(*dC, pl.mapC.data(), nC * sizeof(int), hipMemcpyHostToDevice, s));
    if (nK) GW_HIP(ctx, hipMemcpyAsync(dK, pl.mapK2.data(), nK * sizeof(int), hipMemcpyHostToDevice, s));
    if (nAB) GW_HIP(ctx, hipMemcpyAsync(dAB, pl.mapAB.data(), nAB * sizeof(int), hipMemcpyHostToDevice, s));
    if (nCT) GW_HIP(ctx, hipMemcpyAsync(dCT, pl.mapCT.data(), nCT * sizeof(int), hipMemcpyHostToDevice, s));
    e->maps = maps;
  }
  if (extra) {
    extra[0] = dK;
    extra[1] = dAB;
    extra[2] = dCT;
  }
  p.n1 = pl.n1; p.n2 = pl.n2; p.n3 = pl.n3; p.ng = pl.ng;
  p.m3count = pl.m3count; p.npair = pl.npair;
  p.bc = pl.bc; p.a1_elems = pl.a1_elems; p.a2_elems = pl.a2_elems;
  p.plane = pl.plane; p.nk2 = pl.nk2; p.y1_elems = pl.y1_elems;
  return GW_OK;
}

}  // namespace gwi

namespace {

// The triangle form P~ = X + X^H (X from the upper triangle of P) forms the row and column of a sphere
// vector with |q+G| -> 0 as the difference of two large partial sums (only the whole P's column sums
// cancel, the triangle's do not), and the Coulomb factor sqrt(V) ~ 1/|q+G| carries that rounding into
// eps.  Builds whose sphere holds a vector with 0 < |q+m| < kTriangleMinQ (crystal units) use the
// full-matrix form; at |q+m| = 0 the head rule removes that row from eps.
constexpr double kTriangleMinQ = 1e-2;
}  // namespace

bool gwi::triangle_form_suits(const double *q, const int *miller, int ng) {
  for (int i = 0; i < ng; ++i) {
    const double x = miller[3 * i] + q[0], y = miller[3 * i + 1] + q[1], z = miller[3 * i + 2] + q[2];
    const double d = std::sqrt(x * x + y * y + z * z);
    if (d > 0.0 && d < kTriangleMinQ) return false;
  }
  return true;
}

namespace {

int sphere_transform_impl(gw_ctx *ctx, const float2 *p_rr, gw_grid g, const int *miller, int ng, float2 *p_gg,
                          bool herm, hipStream_t s) {
  SpherePlan plan;
  int *dA, *dB, *dC;
  const int *extra[3] = {nullptr, nullptr, nullptr};
  GW_STATUS(upload_plan(ctx, g, miller, ng, WS_FFT_MAP, plan, &dA, &dB, &dC, s, extra));
  const int nr = g.n1 * g.n2 * g.n3;
  void *a1, *a2, *ph, *pht = nullptr, *q, *y1 = nullptr;
  GW_STATUS(ws_get(ctx, WS_FFT_A, plan.a1_elems * sizeof(float2), &a1, s));
  GW_STATUS(ws_get(ctx, WS_FFT_B, plan.a2_elems * sizeof(float2), &a2, s));
  GW_STATUS(ws_get(ctx, WS_COUNT_BASE + 0, (size_t)ng * nr * sizeof(float2), &ph, s));
  if (plan.plane) GW_STATUS(ws_get(ctx, WS_COUNT_BASE + 2, plan.y1_elems * sizeof(float2), &y1, s));
  else GW_STATUS(ws_get(ctx, WS_COUNT_BASE + 1, (size_t)ng * nr * sizeof(float2), &pht, s));
  GW_STATUS(ws_get(ctx, WS_PGG_T, (size_t)ng * ng * sizeof(float2), &q, s));
  SphereBuffers b{(float2 *)a1, (float2 *)a2, (float2 *)ph, (float2 *)pht, (float2 *)q, dA, dB, dC,
                  (float2 *)y1, extra[0], extra[1], extra[2]};
  GW_HIP(ctx, enqueue_sphere_transform(plan, b, p_rr, p_gg, herm, s));
  return GW_OK;
}

int upload_scales(gw_ctx *ctx, const double *e_v, int nv, const double *e_c, int nc, double prefactor, float **scale,
                  hipStream_t s) {
  void *eb, *sb;
  const int ldsc = scale_ld(nc);
  GW_STATUS(ws_get(ctx, WS_ENERGY, (size_t)(nv + nc) * sizeof(double), &eb, s));
  GW_STATUS(ws_get(ctx, WS_SCALE, scale_table_floats(nv, nc) * sizeof(float), &sb, s));
  double *de = (double *)eb;
  GW_HIP(ctx, hipMemcpyAsync(de, e_v, nv * sizeof(double), hipMemcpyHostToDevice, s));
  GW_HIP(ctx, hipMemcpyAsync(de + nv, e_c, nc * sizeof(double), hipMemcpyHostToDevice, s));
  GW_HIP(ctx, launch_scale_table(de, nv, de + nv, nc, prefactor, (float *)sb, ldsc, s));
  *scale = (float *)sb;
  return GW_OK;
}

int polarizability_r_impl(gw_ctx *ctx, const float2 *psi_v, int nv, const float2 *psi_c, int nc, int nr,
                          const double *e_v, const double *e_c, const gw_opts &o, float2 *p_rr, hipStream_t s) {
  float *scale = nullptr;
  GW_STATUS(upload_scales(ctx, e_v, nv, e_c, nc, o.prefactor, &scale, s));
  int *bexp = nullptr;
  if (o.precision == GW_SPLIT_FP16_SCALED) {
    void *b;
    GW_STATUS(ws_get(ctx, WS_BSCALE, band_exp_ints(nv, nc) * sizeof(int), &b, s));
    bexp = (int *)b;
    GW_HIP(ctx, launch_band_exponents(psi_v, nv, psi_c, nc, nr, scale, scale_ld(nc), bexp, s));
  }
  int tile = o.tile;
  if (tile < 0) tile = tuned_tile(ctx, nr, nv, nc, o.precision);   // -1 when nothing is tuned: the default
  GW_HIP(ctx, launch_herk(o.precision, tile, psi_v, psi_c, scale, scale_ld(nc), bexp, p_rr, nr, nv, nc, o.accumulate, s));
  return GW_OK;
}

int grid_supported(gw_ctx *ctx, gw_grid g) {
  if (!fft_size_supported(g.n1) || !fft_size_supported(g.n2) || !fft_size_supported(g.n3)) {
    set_err(ctx, "grid %dx%dx%d: every side must be one of the built transform lengths", g.n1, g.n2, g.n3);
    return GW_E_UNSUPPORTED;
  }
  return GW_OK;
}

int eps_build_impl(gw_ctx *ctx, const float2 *p_gg, int ng, gw_grid g, const double *q, const int *miller,
                   double head, double2 *eps, hipStream_t s) {
  void *dm, *dsv;
  GW_STATUS(ws_get(ctx, WS_MILLER, (size_t)ng * 3 * sizeof(int), &dm, s));
  GW_STATUS(ws_get(ctx, WS_SQRTV, (size_t)ng * sizeof(double), &dsv, s));
  GW_HIP(ctx, hipMemcpyAsync(dm, miller, (size_t)ng * 3 * sizeof(int), hipMemcpyHostToDevice, s));
  GW_HIP(ctx, launch_sqrtv((const int *)dm, ng, q[0], q[1], q[2], g.a_bohr, (double *)dsv, s));
  GW_HIP(ctx, launch_eps_build(p_gg, ng, (const double *)dsv, head, eps, s));
  return GW_OK;
}

int hpd_inverse_impl(gw_ctx *ctx, double2 *a, int n, double2 *out, hipStream_t s) {
  void *l, *x, *sm, *piv;
  GW_STATUS(ws_get(ctx, WS_CHOL_L, (size_t)n * n * sizeof(double2), &l, s));
  GW_STATUS(ws_get(ctx, WS_CHOL_X, (size_t)n * n * sizeof(double2), &x, s));
  GW_STATUS(ws_get(ctx, WS_CHOL_SMALL, chol_small_bytes(n) + 256, &sm, s));
  piv = (char *)sm + chol_small_bytes(n);
  GW_HIP(ctx, hpd_inverse(a, n, (double2 *)l, (double2 *)x, (double2 *)sm, (int *)piv, out, s));
  GW_HIP(ctx, hipMemcpyAsync(ctx->pivot_host, piv, sizeof(int), hipMemcpyDeviceToHost, s));
  GW_HIP(ctx, hipStreamSynchronize(s));
  if (*ctx->pivot_host != 0) {
    set_err(ctx, "matrix is not positive definite: pivot %d (1-based) is not positive", *ctx->pivot_host);
    return GW_E_NOTPD;
  }
  return GW_OK;
}

}  // namespace

// ============================================================================================
// Exported entry points
// ============================================================================================
extern "C" {

void gw_opts_default(gw_opts *o) {
  if (!o) return;
  o->precision = GW_FP32;
  o->prefactor = 1.0;
  o->accumulate = 0;
  o->tile = -1;
}

int gw_version(void) { return 10000; }

const char *gw_status_string(int st) {
  switch (st) {
    case GW_OK: return "GW_OK";
    case GW_E_INVAL: return "GW_E_INVAL: invalid argument";
    case GW_E_NOMEM: return "GW_E_NOMEM: workspace cap or device memory exceeded";
    case GW_E_HIP: return "GW_E_HIP: HIP runtime error";
    case GW_E_NOTPD: return "GW_E_NOTPD: matrix not positive definite";
    case GW_E_UNSUPPORTED: return "GW_E_UNSUPPORTED: request not supported by this build";
  }
  return "unknown status";
}

int gw_create(gw_ctx **ctx, int hip_device, size_t cap) {
  if (!ctx) return GW_E_INVAL;
  *ctx = nullptr;
  if (hip_device < -1) return GW_E_INVAL;
  gw_ctx *c = new (std::nothrow) gw_ctx();
  if (!c) return GW_E_NOMEM;
  c->device = hip_device;
  c->cap = cap;
  if (hip_device >= 0) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || hip_device >= count) {
      (void)hipGetLastError();
      delete c;
      return GW_E_HIP;
    }
    if (hipSetDevice(hip_device) != hipSuccess ||
        hipHostMalloc((void **)&c->pivot_host, sizeof(int), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      delete c;
      return GW_E_HIP;
    }
    *c->pivot_host = 0;
    // the allocation-free update's scratch array: this device's address, resolved with the device current
    if (gwi::noalloc_resolve(hip_device) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipHostFree(c->pivot_host);
      delete c;
      return GW_E_HIP;
    }
  }
  *ctx = c;
  return GW_OK;
}

int gw_destroy(gw_ctx *ctx) {
  if (!ctx) return GW_E_INVAL;
  int st = GW_OK;
  if (ctx->device >= 0) {
    if (hipSetDevice(ctx->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) st = GW_E_HIP;
    gwi::batched_release(ctx);
    gwi::tail_graphs_release(ctx);
    for (auto &sl : ctx->slots)
      if (sl.ptr) (void)hipFree(sl.ptr);
    if (ctx->pivot_host) (void)hipHostFree(ctx->pivot_host);
  }
  delete ctx;
  return st;
}

const char *gw_last_error(const gw_ctx *ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

size_t gw_workspace_bytes(const gw_ctx *ctx) { return ctx ? ctx->held : 0; }

int gw_tile_count(void) { return herk_tile_count(); }
const char *gw_tile_name(int t) { return herk_tile_name(t); }
int gw_default_tile(int precision, int nr) { return herk_default_tile(precision, nr); }

int gw_mfma_rate(gw_ctx *ctx, const uint32_t *words, int n_iter, int grid, float *out, void *stream) {
  GW_STATUS(begin(ctx));
  GW_CHECK(ctx, words != nullptr && out != nullptr, "words and out must not be NULL");
  GW_CHECK(ctx, n_iter >= 1 && grid >= 1 && grid <= (1 << 24), "n_iter must be >= 1 and grid in [1, 2^24]");
  if (ctx->device < 0) return GW_OK;
  GW_HIP(ctx, launch_mfma_rate(words, n_iter, grid, out, as_stream(stream)));
  return GW_OK;
}

int gw_pair_products(gw_ctx *ctx, const gw_c32 *psi_v, int nv, const gw_c32 *psi_c, int nc, int nr,
                     const double *e_v, const double *e_c, double prefactor, gw_c32 *f_out, void *stream) {
  GW_STATUS(begin(ctx));
  GW_STATUS(check_bands(ctx, psi_v, nv, psi_c, nc, nr));
  GW_CHECK(ctx, f_out != nullptr, "f_out must not be NULL");
  GW_CHECK(ctx, std::isfinite(prefactor) && prefactor > 0.0, "prefactor must be positive");
  GW_CHECK(ctx, (nc + 7) / 8 <= 65535, "nc too large for the pair-product grid");
  GW_STATUS(check_energies(ctx, e_v, nv, e_c, nc));
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  float *scale = nullptr;
  GW_STATUS(upload_scales(ctx, e_v, nv, e_c, nc, prefactor, &scale, s));
  GW_HIP(ctx, launch_pair_products((const float2 *)psi_v, nv, (const float2 *)psi_c, nc, nr, scale, scale_ld(nc),
                                   (float2 *)f_out, s));
  return GW_OK;
}

int gw_polarizability_r(gw_ctx *ctx, const gw_c32 *psi_v, int nv, const gw_c32 *psi_c, int nc, int nr,
                        const double *e_v, const double *e_c, const gw_opts *opts, gw_c32 *p_rr, void *stream) {
  GW_STATUS(begin(ctx));
  gw_opts o;
  gw_opts_default(&o);
  if (opts) o = *opts;
  GW_STATUS(check_bands(ctx, psi_v, nv, psi_c, nc, nr));
  GW_CHECK(ctx, p_rr != nullptr, "p_rr must not be NULL");
  GW_STATUS(check_opts(ctx, &o));
  GW_STATUS(check_energies(ctx, e_v, nv, e_c, nc));
  if (ctx->device < 0) return GW_OK;
  return polarizability_r_impl(ctx, (const float2 *)psi_v, nv, (const float2 *)psi_c, nc, nr, e_v, e_c, o,
                               (float2 *)p_rr, as_stream(stream));
}

int gw_sphere_transform(gw_ctx *ctx, const gw_c32 *p_rr, gw_grid grid, const int *g_miller, int ng, gw_c32 *p_gg,
                        void *stream) {
  GW_STATUS(begin(ctx));
  GW_CHECK(ctx, p_rr && p_gg, "p_rr and p_gg must not be NULL");
  GW_STATUS(check_grid(ctx, grid));
  GW_STATUS(check_sphere(ctx, grid, g_miller, ng));
  GW_STATUS(grid_supported(ctx, grid));
  if (ctx->device < 0) return GW_OK;
  return sphere_transform_impl(ctx, (const float2 *)p_rr, grid, g_miller, ng, (float2 *)p_gg, false, as_stream(stream));
}

int gw_sphere_transform_herm(gw_ctx *ctx, const gw_c32 *p_rr, gw_grid grid, const int *g_miller, int ng,
                             gw_c32 *p_gg, void *stream) {
  GW_STATUS(begin(ctx));
  GW_CHECK(ctx, p_rr && p_gg, "p_rr and p_gg must not be NULL");
  GW_STATUS(check_grid(ctx, grid));
  GW_STATUS(check_sphere(ctx, grid, g_miller, ng));
  GW_STATUS(grid_supported(ctx, grid));
  if (ctx->device < 0) return GW_OK;
  return sphere_transform_impl(ctx, (const float2 *)p_rr, grid, g_miller, ng, (float2 *)p_gg, true, as_stream(stream));
}

int gw_orbitals_to_grid(gw_ctx *ctx, const gw_c32 *coeff, int nb, int npw, gw_grid grid, const int *pw_miller,
                        gw_c32 *psi, void *stream) {
  GW_STATUS(begin(ctx));
  GW_CHECK(ctx, coeff && psi, "coeff and psi must not be NULL");
  GW_CHECK(ctx, nb > 0, "nb must be positive (got %d)", nb);
  GW_STATUS(check_grid(ctx, grid));
  const long long nrl = (long long)grid.n1 * grid.n2 * grid.n3;
  GW_CHECK(ctx, nrl <= (1 << 24), "grid too large");
  GW_STATUS(check_sphere(ctx, grid, pw_miller, npw));
  GW_STATUS(grid_supported(ctx, grid));
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  const int nr = (int)nrl;
  SpherePlan p;
  int *dA, *dB, *dC;
  const int *extra[3] = {nullptr, nullptr, nullptr};   // k2 list + slot table, (k2, k3) pair slots, (k1, pair) map
  GW_STATUS(upload_plan(ctx, grid, pw_miller, npw, WS_ORB_MAP, p, &dA, &dB, &dC, s, extra));
  const float scale = (float)(1.0 / std::sqrt((double)nr));
  const float2 *c = (const float2 *)coeff;
  float2 *out = (float2 *)psi;
  if (p.plane) {
    // row-contiguous: y [w][n1][npair] per chunk of w bands (near 1 GiB), then the planes of each band
    const size_t per_band = (size_t)p.n1 * p.npair;
    const int w = (int)std::min<long long>(nb, std::max<long long>(1, (1LL << 27) / (long long)per_band));
    void *y;
    GW_STATUS(ws_get(ctx, WS_ORB_A1, per_band * w * sizeof(float2), &y, s));
    for (int b0 = 0; b0 < nb; b0 += w) {
      const int bw = std::min(w, nb - b0);
      GW_HIP(ctx, launch_orb_c(p.n1, c + (size_t)b0 * npw, npw, bw, extra[2], p.npair, scale, (float2 *)y, s));
      GW_HIP(ctx, launch_orb_plane(p.n3, (const float2 *)y, bw, p.n1, extra[0] + p.nk2, p.nk2, extra[1], p.npair,
                                   out + (size_t)b0 * nr, nr, s));
    }
    return GW_OK;
  }
  // band chunk: an intermediate of [nr][w] elements would stay near 1 GiB
  const int w = (int)std::min<long long>(nb, std::max<long long>(64, (1LL << 27) / nr));
  const size_t rows1 = (size_t)p.n1 * p.n2 * p.m3count, rows2 = (size_t)p.n1 * p.npair;
  void *ct, *a1, *a2;
  GW_STATUS(ws_get(ctx, WS_ORB_T, (size_t)npw * w * sizeof(float2), &ct, s));
  GW_STATUS(ws_get(ctx, WS_ORB_A1, rows1 * w * sizeof(float2), &a1, s));
  GW_STATUS(ws_get(ctx, WS_ORB_A2, rows2 * w * sizeof(float2), &a2, s));
  for (int b0 = 0; b0 < nb; b0 += w) {
    const int bw = std::min(w, nb - b0);
    float2 *t = (float2 *)ct, *x1 = (float2 *)a1, *x2 = (float2 *)a2;
    GW_HIP(ctx, launch_transpose_c64(c + (size_t)b0 * npw, t, bw, npw, npw, bw, s));
    // sphere -> (i1, pair) along axis 1; -> (i1, i2, m3) along axis 2; -> grid along axis 3
    GW_HIP(ctx, launch_fft_gather_pass(p.n1, +1, t, x2, 1, p.npair, bw, bw, bw, dC, scale, s));
    GW_HIP(ctx, launch_fft_gather_pass(p.n2, +1, x2, x1, p.n1, p.m3count, bw, bw, bw, dB, 1.0f, s));
    // the last axis writes the band-major orbitals directly
    GW_HIP(ctx, launch_fft_gather_pass_t(p.n3, +1, x1, out + (size_t)b0 * nr, p.n1 * p.n2, bw, bw, nr, dA, 1.0f, s));
  }
  return GW_OK;
}

int gw_polarizability(gw_ctx *ctx, const gw_c32 *psi_occ, int nv, const gw_c32 *psi_unocc, int nc, const double *e_v,
                      const double *e_c, gw_grid grid, const double *q, const int *g_miller, int ng,
                      const gw_opts *opts, gw_c32 *p_rr, gw_c32 *p_gg, void *stream) {
  GW_STATUS(begin(ctx));
  gw_opts o;
  gw_opts_default(&o);
  if (opts) o = *opts;
  GW_STATUS(check_grid(ctx, grid));
  const long long nrl = (long long)grid.n1 * grid.n2 * grid.n3;
  GW_CHECK(ctx, nrl <= (1 << 24), "grid too large");
  const int nr = (int)nrl;
  GW_STATUS(check_bands(ctx, psi_occ, nv, psi_unocc, nc, nr));
  GW_STATUS(check_q(ctx, q));
  GW_CHECK(ctx, p_gg != nullptr, "p_gg must not be NULL");
  GW_CHECK(ctx, !(o.accumulate && !p_rr), "accumulate needs the caller's p_rr buffer");
  GW_STATUS(check_opts(ctx, &o));
  GW_STATUS(check_energies(ctx, e_v, nv, e_c, nc));
  GW_STATUS(check_sphere(ctx, grid, g_miller, ng));
  GW_STATUS(grid_supported(ctx, grid));
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  float2 *prr = (float2 *)p_rr;
  if (!prr) {
    void *w;
    GW_STATUS(ws_get(ctx, WS_PRR, (size_t)nr * nr * sizeof(float2), &w, s));
    prr = (float2 *)w;
  }
  GW_STATUS(polarizability_r_impl(ctx, (const float2 *)psi_occ, nv, (const float2 *)psi_unocc, nc, nr, e_v, e_c, o,
                                  prr, s));
  // the update writes a Hermitian P (with accumulate the caller's earlier contents are part of it)
  return sphere_transform_impl(ctx, prr, grid, g_miller, ng, (float2 *)p_gg,
                               !o.accumulate && triangle_form_suits(q, g_miller, ng), s);
}

int gw_epsilon(gw_ctx *ctx, const gw_c32 *p_gg, int ng, gw_grid grid, const double *q, const int *g_miller,
               double head, gw_c64 *eps_out, void *stream) {
  GW_STATUS(begin(ctx));
  GW_CHECK(ctx, p_gg && eps_out, "p_gg and eps_out must not be NULL");
  GW_STATUS(check_q(ctx, q));
  GW_STATUS(check_grid(ctx, grid));
  GW_STATUS(check_sphere(ctx, grid, g_miller, ng));
  if (std::isnan(head)) head = 1.0;
  GW_CHECK(ctx, std::isfinite(head) && head > 0.0, "head must be positive");
  if (ctx->device < 0) return GW_OK;
  return eps_build_impl(ctx, (const float2 *)p_gg, ng, grid, q, g_miller, head, (double2 *)eps_out, as_stream(stream));
}

int gw_eps_inverse(gw_ctx *ctx, const gw_c32 *p_gg, int ng, gw_grid grid, const double *q, const int *g_miller,
                   double head, gw_c64 *eps_inv, void *stream) {
  GW_STATUS(begin(ctx));
  GW_CHECK(ctx, p_gg && eps_inv, "p_gg and eps_inv must not be NULL");
  GW_STATUS(check_q(ctx, q));
  GW_STATUS(check_grid(ctx, grid));
  GW_STATUS(check_sphere(ctx, grid, g_miller, ng));
  if (std::isnan(head)) head = 1.0;
  GW_CHECK(ctx, std::isfinite(head) && head > 0.0, "head must be positive");
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  void *e;
  GW_STATUS(ws_get(ctx, WS_EPS, (size_t)ng * ng * sizeof(double2), &e, s));
  GW_STATUS(eps_build_impl(ctx, (const float2 *)p_gg, ng, grid, q, g_miller, head, (double2 *)e, s));
  return hpd_inverse_impl(ctx, (double2 *)e, ng, (double2 *)eps_inv, s);
}

int gw_hpd_inverse(gw_ctx *ctx, const gw_c64 *a, int n, gw_c64 *out, void *stream) {
  GW_STATUS(begin(ctx));
  GW_CHECK(ctx, a && out, "a and out must not be NULL");
  GW_CHECK(ctx, n > 0 && n <= 65536, "n must be in [1, 65536]");
  if (ctx->device < 0) return GW_OK;
  hipStream_t s = as_stream(stream);
  void *e;
  GW_STATUS(ws_get(ctx, WS_EPS, (size_t)n * n * sizeof(double2), &e, s));
  GW_HIP(ctx, hipMemcpyAsync(e, a, (size_t)n * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
  return hpd_inverse_impl(ctx, (double2 *)e, n, (double2 *)out, s);
}

int gw_newton_inverse(gw_ctx *ctx, const gw_c64 *a, int n, double tol, int max_iter, gw_c64 *out, int *iterations,
                      double *history, void *stream) {
  GW_STATUS(begin(ctx));
  GW_CHECK(ctx, a && out && iterations, "a, out and iterations must not be NULL");
  GW_CHECK(ctx, n > 0 && n <= 65536, "n must be in [1, 65536]");
  GW_CHECK(ctx, std::isfinite(tol) && tol > 0.0, "tol must be positive");
  GW_CHECK(ctx, max_iter > 0 && max_iter <= 10000, "max_iter must be in [1, 10000]");
  if (ctx->device < 0) { *iterations = 0; return GW_OK; }
  hipStream_t s = as_stream(stream);
  void *w;
  GW_STATUS(ws_get(ctx, WS_NEWTON, newton_ws_bytes(n), &w, s));
  const size_t nn = (size_t)n * n;
  double2 *x = (double2 *)w, *t = x + nn, *xn = t + nn;
  double *sc = (double *)(xn + nn);
  GW_HIP(ctx, newton_start((const double2 *)a, n, x, t, sc, s));
  double diff = 0.0;
  int it = 0;
  for (it = 1; it <= max_iter; ++it) {
    GW_HIP(ctx, newton_step((const double2 *)a, n, x, t, xn, sc, s));
    GW_HIP(ctx, hipMemcpyAsync(&diff, sc + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    GW_HIP(ctx, hipStreamSynchronize(s));
    if (history) history[it - 1] = diff;
    std::swap(x, xn);
    if (!(diff >= tol)) break;     // converged (or NaN: stop and report)
  }
  *iterations = std::min(it, max_iter);
  GW_HIP(ctx, hipMemcpyAsync(out, x, nn * sizeof(double2), hipMemcpyDeviceToDevice, s));
  GW_HIP(ctx, hipStreamSynchronize(s));
  if (!std::isfinite(diff)) {
    set_err(ctx, "Newton iteration diverged (max change is not finite)");
    return GW_E_NOTPD;
  }
  if (diff >= tol) {
    set_err(ctx, "Newton iteration did not reach tol %.3g in %d iterations (last max change %.3g)", tol, max_iter,
            diff);
    return GW_E_UNSUPPORTED;
  }
  return GW_OK;
}

int gw_eps_inverse_newton(gw_ctx *ctx, const gw_c32 *p_gg, int ng, gw_grid grid, const double *q, const int *g_miller,
                          double head, double tol, int max_iter, gw_c64 *eps_inv, int *iterations, double *history,
                          void *stream) {
  GW_STATUS(begin(ctx));
  GW_CHECK(ctx, p_gg && eps_inv && iterations, "p_gg, eps_inv and iterations must not be NULL");
  GW_STATUS(check_q(ctx, q));
  GW_STATUS(check_grid(ctx, grid));
  GW_STATUS(check_sphere(ctx, grid, g_miller, ng));
  if (std::isnan(head)) head = 1.0;
  GW_CHECK(ctx, std::isfinite(head) && head > 0.0, "head must be positive");
  GW_CHECK(ctx, std::isfinite(tol) && tol > 0.0, "tol must be positive");
  GW_CHECK(ctx, max_iter > 0 && max_iter <= 10000, "max_iter must be in [1, 10000]");
  if (ctx->device < 0) { *iterations = 0; return GW_OK; }
  hipStream_t s = as_stream(stream);
  void *e;
  GW_STATUS(ws_get(ctx, WS_EPS, (size_t)ng * ng * sizeof(double2), &e, s));
  GW_STATUS(eps_build_impl(ctx, (const float2 *)p_gg, ng, grid, q, g_miller, head, (double2 *)e, s));
  return gw_newton_inverse(ctx, (const gw_c64 *)e, ng, tol, max_iter, eps_inv, iterations, history, stream);
}

}  // extern "C"

// Batched q (gw_batched.cpp) reuses the pieces above.
namespace gwi {
int api_ws_get(gw_ctx *ctx, int slot, size_t bytes, void **out, hipStream_t s) { return ws_get(ctx, slot, bytes, out, s); }
int api_check_energies(gw_ctx *ctx, const double *e_v, int nv, const double *e_c, int nc) {
  return check_energies(ctx, e_v, nv, e_c, nc);
}
int api_check_sphere(gw_ctx *ctx, gw_grid g, const int *m, int ng) { return check_sphere(ctx, g, m, ng); }
int api_check_opts(gw_ctx *ctx, const gw_opts *o) { return check_opts(ctx, o); }
int api_check_grid(gw_ctx *ctx, gw_grid g) { return check_grid(ctx, g); }
int api_grid_supported(gw_ctx *ctx, gw_grid g) { return grid_supported(ctx, g); }
int api_begin(gw_ctx *ctx) { return begin(ctx); }
void api_set_err(gw_ctx *ctx, const char *msg) { set_err(ctx, "%s", msg); }
int api_device(gw_ctx *ctx) { return ctx->device; }
}  // namespace gwi
