// Internal declarations shared by the host ABI (gw_api.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdio>
#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/gw.h"

namespace gwi {
struct PlanCacheEntry;
}

struct gw_ctx {
  int device = -1;            // -1: dry-run context (argument checks only)
  size_t cap = 0;             // workspace cap in bytes (0: none)
  size_t held = 0;            // bytes currently allocated in slots
  std::string err;            // text of the last failure
  struct Slot { void *ptr = nullptr; size_t bytes = 0; };
  std::vector<Slot> slots;    // grow-only named workspace buffers
  int *pivot_host = nullptr;  // pinned host word for the Cholesky pivot flag
  void *graph_cache = nullptr;  // batched-q graphs (owned; see gw_batched.cpp)
  void *tail_graphs = nullptr;  // training-step graphs of the learned tail (owned; see gw_tail.cpp)
  std::map<std::string, int> tuned;   // autotuned update tiles, keyed by arch and shape
  bool tune_loaded = false;           // the autotune cache file has been read
  std::string arch;                   // device architecture name (cached)
  // the sphere plan last uploaded into each map slot, reused while grid, Miller list and stream match
  std::map<int, std::unique_ptr<gwi::PlanCacheEntry>> plans;
  // the last spheres (grid and Miller list) that passed the argument checks, reused round-robin
  struct SphereSeen { int n1 = 0, n2 = 0, n3 = 0; std::vector<int> miller; };
  SphereSeen spheres_ok[4];
  int spheres_next = 0;
};

namespace gwi {

// Workspace slots (each a grow-only device buffer owned by the context).
enum SlotId {
  WS_SCALE = 0,   // float [nv][nc] pair scales
  WS_ENERGY,      // double [nv + nc] energies
  WS_PRR,         // complex64 [nr][nr] internal P(r,r')
  WS_FFT_A,       // FFT intermediates
  WS_FFT_B,
  WS_FFT_MAP,     // int output-row maps of the FFT passes
  WS_MILLER,      // int [ng][3]
  WS_SQRTV,       // double [ng]
  WS_EPS,         // complex128 [n][n] eps / working matrix
  WS_CHOL_L,      // complex128 [n][n] Cholesky factor
  WS_CHOL_X,      // complex128 [n][n] L^-1
  WS_CHOL_SMALL,  // diagonal-block inverses + pivot flag
  WS_BSCALE,      // per-band power-of-two exponents (FP16 path)
  WS_PGG_T,       // complex64 [ng][ng] transposed sphere result
  WS_TAIL,        // learned-tail intermediates
  WS_TAIL_FLAG,   // training-box flag
  WS_NEWTON,      // Newton iteration buffers
  WS_ORB_T,       // plane-wave coefficients, transposed [npw][nb]
  WS_ORB_A1,      // orbital transform intermediates
  WS_ORB_A2,
  WS_ORB_MAP,     // int maps of the orbital transform
  WS_COUNT_BASE
};

// Kernel launchers.  All return hipSuccess or the launch error; all run on `s`.
// Pair scales s_vc = sqrt(p / (E_c - E_v)) as float [nv][ldsc], zero for nc <= c < ldsc.
int scale_ld(int nc);
size_t scale_table_floats(int nv, int nc);   // s table, then s^2 table, each [nv][scale_ld(nc)]
hipError_t launch_scale_table(const double *e_v, int nv, const double *e_c, int nc, double prefactor,
                              float *scale, int ldsc, hipStream_t s);
hipError_t launch_pair_products(const float2 *psi_v, int nv, const float2 *psi_c, int nc, int nr,
                                const float *scale, int ldsc, float2 *f, hipStream_t s);

// Rank-K update P = -F^H F with the pair products formed in-kernel.
// precision: enum gw_precision; tile: index into the tile table (-1 default).
int herk_tile_count();
const char *herk_tile_name(int tile);
bool herk_tile_supports(int tile, int precision);
int herk_default_tile(int precision, int nr);
hipError_t launch_herk(int precision, int tile, const float2 *psi_v, const float2 *psi_c, const float *scale, int ldsc,
                       const int *band_exp, float2 *p, int nr, int nv, int nc, int accumulate, hipStream_t s);
hipError_t launch_band_exponents(const float2 *psi_v, int nv, const float2 *psi_c, int nc, int nr,
                                 const float *scale, int ldsc, int *band_exp, hipStream_t s);
// ints needed by launch_band_exponents' buffer (exponents, band order, sorted exponents, row maxima)
size_t band_exp_ints(int nv, int nc);
// MFMA-only rate kernel (4096 uint32 operand words, grid workgroups of 512 threads).
hipError_t launch_mfma_rate(const unsigned *words, int n_iter, int grid, float *out, hipStream_t s);

// FFT helpers.
bool fft_size_supported(int n);
// One pass along an axis of length n: in element ((o*n + i)*U + u)*ld_in + b, out element
// map[(o*U + u)*n + k]*ld_out + b for every k with map >= 0.  sign -1: exp(-i..), +1: exp(+i..).
hipError_t launch_fft_pass(int n, int sign, const float2 *in, float2 *out, int O, int U, int B, long long ld_in,
                           long long ld_out, const int *map, hipStream_t s);
// Gather pass: rows of `in` read through `map` (-1 reads zero) and scaled, outputs to rows (o*n + k)*U + u.
// The gather pass along the last axis (U = 1) writing out[b][o n + k] directly (band-major output).
hipError_t launch_fft_gather_pass_t(int n, int sign, const float2 *in, float2 *out, int O, int B, long long ld_in,
                                    long long ld_out, const int *map, float scale, hipStream_t s);
hipError_t launch_fft_gather_pass(int n, int sign, const float2 *in, float2 *out, int O, int U, int B, long long ld_in,
                                  long long ld_out, const int *map, float scale, hipStream_t s);
hipError_t launch_transpose_c64(const float2 *in, float2 *out, int rows, int cols, long long ld_in,
                                long long ld_out, hipStream_t s);

// eps and the FP64 Hermitian inverse.
hipError_t launch_sqrtv(const int *miller, int ng, double q0, double q1, double q2, double a_bohr, double *sv,
                        hipStream_t s);
hipError_t launch_eps_build(const float2 *p_gg, int ng, const double *sv, double head, double2 *eps,
                            hipStream_t s);
// Cholesky-based inverse of a Hermitian PD matrix (lower triangle of a read).  a is overwritten.
// l, x: n*n workspaces; small: workspace of at least chol_small_bytes(n); pivot_dev: device int.
size_t chol_small_bytes(int n);
hipError_t hpd_inverse(double2 *a, int n, double2 *l, double2 *x, double2 *small, int *pivot_dev, double2 *out,
                       hipStream_t s);
hipError_t launch_fill_int(int *p, int value, hipStream_t s);
// C = alpha op(A) op(B) + beta C, complex128, op = identity (0) or conjugate transpose (1); row-major.
hipError_t launch_zgemm(int M, int N, int K, const double2 *A, long long lda, int transA, const double2 *B,
                        long long ldb, int transB, double2 *C, long long ldc, double alpha, double beta,
                        hipStream_t s);
// The same for thin outputs (fewer than 256 output tiles): K is split over workgroups into partial
// products in ws (zgemm_splitk_ws_elems(M, N, K) complex128 elements; 0 means no split is used) and
// summed by a second kernel.  Falls back to the plain product when ws is too small.
size_t zgemm_splitk_ws_elems(int M, int N, int K);
hipError_t launch_zgemm_splitk(int M, int N, int K, const double2 *A, long long lda, int transA, const double2 *B,
                               long long ldb, int transB, double2 *C, long long ldc, double alpha, double beta,
                               double2 *ws, size_t ws_elems, hipStream_t s);
// Plasmon-pole kernels (pp.hip)
hipError_t launch_density(const float2 *psi, int nv, int nr, double occ, double2 *rho, hipStream_t s);
hipError_t launch_density_transform(double2 *rho, double2 *tmp, int n1, int n2, int n3, hipStream_t s);
hipError_t launch_screening(const double2 *ei, const double *sv, int ng, double2 *out, hipStream_t s);
hipError_t launch_sum_rule(const int *miller, int ng, const double *q, double a_bohr, const double *sv,
                           const double2 *rho_g, int n1, int n2, int n3, double2 *m, hipStream_t s);
hipError_t launch_start_block(double2 *x, int ng, int b, unsigned long long seed, hipStream_t s);
hipError_t launch_herm_jacobi(const double2 *h, int b, int ldh, double *evals, double2 *z, int ldz, hipStream_t s);
hipError_t launch_col_normalize(double2 *w, int rows, int ld, int cols, hipStream_t s);
hipError_t launch_svqb_scale(double2 *u, const double *lam, int b, double rel, hipStream_t s);
hipError_t launch_ritz_residual(const double2 *x, const double2 *y, int ng, int ld, const double *theta, int nm,
                                double *out, hipStream_t s);
hipError_t launch_pp_frequency(const double2 *a, int lda, const double2 *t, int ldt, int ng, const double *theta,
                               int nm, double *sigma, double *omega, hipStream_t s);
hipError_t launch_pp_weight(const double2 *modes, int ng, int nm, const double *sigma, const double *omega, double w,
                            double2 *out, hipStream_t s);
hipError_t launch_pp_finish(double2 *e, const double2 *ei_static, const double *sv, int ng, hipStream_t s);
hipError_t launch_sqrtv(const int *miller, int ng, double q0, double q1, double q2, double a_bohr, double *sv,
                        hipStream_t s);
// Static self-energy kernels (sigma.hip)
hipError_t launch_fill_f32(float *p, int n, float v, hipStream_t s);
hipError_t launch_conj_upcast(const float2 *in, size_t n, double2 *out, hipStream_t s);
hipError_t launch_contract_conj(const float2 *a, const float2 *b, int ng, int nv, long long ld, const double *sv,
                                double scale, int nn, double2 *out, hipStream_t s);
hipError_t launch_contract_t(const float2 *a, const double2 *t, int ng, int nv, long long ld, double scale, int nn,
                             double2 *out, hipStream_t s);
hipError_t launch_zeta(const float2 *f, int ng, int npair, const double2 *modes, int nm, double2 *zeta, hipStream_t s);
hipError_t launch_contract_modes(const double2 *zeta, int nm, int nv, int nn, const double *sigma, double2 *out,
                                 hipStream_t s);
// Newton iteration for the inverse: workspace of newton_ws_bytes(n) holds x, t, xn and the scalars.
size_t newton_ws_bytes(int n);
hipError_t newton_start(const double2 *a, int n, double2 *x, double2 *t, double *scratch, hipStream_t s);
hipError_t newton_step(const double2 *a, int n, const double2 *x, double2 *t, double2 *xn, double *scratch,
                       hipStream_t s);

// Learned band-tail correction (tail.hip).
size_t tail_ws_floats(int n);
hipError_t tail_features(const float2 *p, int ng, const int *miller, const double *q, double a_bohr, int nc,
                         double e_max, float *feat, hipStream_t s);
hipError_t tail_target(const float2 *full, const float2 *trunc, int ng, float2 *t, hipStream_t s);
hipError_t tail_forward(const gw_mlp &w, const float *feat, int n, float *ws, float *out, hipStream_t s);
hipError_t tail_train_step(const gw_mlp &w, const gw_adam &a, const float *feat, const float2 *target, int n,
                           float *ws, float *loss_out, int *step_dev, int set_step, hipStream_t s);
void tail_graphs_release(gw_ctx *ctx);
hipError_t tail_residual_parts(const gw_mlp &w, const float *feat, const float2 *target, int n, float *ws,
                               float *parts, hipStream_t s);
hipError_t tail_fit_norm(int nsys, const float *const *feats, const int *ngs, double *acc, float *norm,
                         hipStream_t s);
hipError_t tail_sync_weights(gw_mlp &w, const float *master, hipStream_t s);
hipError_t tail_loss(const gw_mlp &w, const float *feat, const float2 *target, int n, float *ws, float *loss_out,
                     hipStream_t s);
hipError_t tail_check_box(const float *feat, int n, const float *norm, int *flag, hipStream_t s);
hipError_t tail_apply(const gw_mlp &w, const float *feat, const float2 *p, int n, float *ws, float2 *out,
                      hipStream_t s);

// Releases the batched-q graphs a context holds.
void batched_release(gw_ctx *ctx);

// ---- sphere-transform plan (host) and its launch sequence (kernels only) -----------------------
struct SpherePlan {
  int n1 = 0, n2 = 0, n3 = 0, ng = 0;
  int m3count = 0, npair = 0;
  std::vector<int> mapA, mapB, mapC;
  int bc = 0;                      // column chunk of the row passes
  size_t a1_elems = 0, a2_elems = 0;
  // row-contiguous form (plane_ab_kernel / plane_c_kernel; only when n2 == n3, see plane_path_supported)
  bool plane = false;
  int nk2 = 0;                     // k2 values that occur in a sphere pair
  std::vector<int> mapK2;          // [nk2] those k2 (grid indices 0 .. n2-1), then [n2] the slot of each k2 or -1
  std::vector<int> mapAB;          // [nk2][n3] pair slot of (k2, k3) or -1
  std::vector<int> mapCT;          // [n1][npair] sphere index of (k1, pair) or -1
  size_t y1_elems = 0;             // [nr][n1][npair] intermediate
  size_t maps_ints() const { return mapA.size() + mapB.size() + mapC.size() + mapK2.size() + mapAB.size() + mapCT.size(); }
};
void build_sphere_plan(gw_grid g, const int *miller, int ng, SpherePlan &p);
struct PlanCacheEntry {
  gw_grid g{};
  std::vector<int> miller;   // [ng][3], the list the plan was built from
  void *stream = nullptr;    // stream the maps were uploaded on
  void *maps = nullptr;      // device copy of the maps (the slot's buffer at upload)
  SpherePlan plan;
};
struct SphereBuffers {
  float2 *a1, *a2, *ph, *pht, *q;  // pass intermediates, P^ [ng][nr], its transpose, Q [ng][ng]
  const int *dA, *dB, *dC;         // device copies of the plan's maps
  float2 *y1 = nullptr;            // row-contiguous form: [nr][n1][npair] (plan.y1_elems)
  const int *dK2 = nullptr, *dAB = nullptr, *dCT = nullptr;   // dK2: the k2 list, then the slot table
};
// P~ from P(r,r') [nr][nr].  herm: P is Hermitian (as the update writes it), so only its upper
// triangle is read.  The row-contiguous form runs where the plan allows it (b.y1 set), else the
// strided passes.
hipError_t enqueue_sphere_transform(const SpherePlan &p, const SphereBuffers &b, const float2 *p_rr, float2 *p_gg,
                                    bool herm, hipStream_t s);
bool plane_path_supported(int n2, int n3);
// Whether the triangle (Hermitian) form of the transforms suits a build at q with this sphere: no vector
// with 0 < |q+m| < 1e-2 (crystal units), whose Coulomb factor would amplify that form's head-row rounding.
bool triangle_form_suits(const double *q, const int *miller, int ng);
hipError_t launch_plane_ab(int n, bool herm, const float2 *p, long long ldp, int nr, int n1, const int *k2s, int nk2,
                           const int *mapab, int npair, float2 *y1, hipStream_t s);
hipError_t launch_plane_c(int n1, bool herm, const float2 *y1, int nr, int plane, int npair, const int *mapct, int ng,
                          float2 *y, long long ldy, hipStream_t s);
// orbitals, row-contiguous (n2 == n3): y[b][i1][pair] = sum_k1 of the band's sphere coefficients over k1 (scaled), then
// the planes of psi[b] (row stride ldpsi) from y
hipError_t launch_orb_c(int n1, const float2 *coeff, int npw, int nb, const int *mapct, int npair, float scale,
                        float2 *y, hipStream_t s);
hipError_t launch_orb_plane(int n, const float2 *y, int nb, int n1, const int *k2s, int nk2, const int *mapab,
                            int npair, float2 *psi, long long ldpsi, hipStream_t s);
hipError_t launch_add_adjoint(const float2 *x, int n, float2 *out, hipStream_t s);
// One 3-D transform over the row index of `in` ([nr][B], row stride ld_in) to the sphere rows of
// `out` ([ng][B], row stride ld_out), in column chunks of at most bc (a1, a2 hold rowsA*bc and
// n1*npair*bc elements).
hipError_t transform_rows(const SpherePlan &p, int sign, const float2 *in, long long ld_in, int B, float2 *out,
                          long long ld_out, float2 *a1, float2 *a2, int bc, const int *dA, const int *dB,
                          const int *dC, hipStream_t s);
// Build the sphere plan and copy its maps into workspace slot `map_slot` (all six maps, in the order
// A, B, C, K2, AB, CT; `extra`, if given, receives the device addresses of K2, AB and CT).
int upload_plan(gw_ctx *ctx, gw_grid g, const int *miller, int ng, int map_slot, SpherePlan &p, int **dA, int **dB,
                int **dC, hipStream_t s, const int **extra = nullptr);

// ---- shared host helpers of gw_api.cpp used by the batched path ---------------------------------
int api_ws_get(gw_ctx *ctx, int slot, size_t bytes, void **out, hipStream_t s);
int api_check_energies(gw_ctx *ctx, const double *e_v, int nv, const double *e_c, int nc);
int api_check_sphere(gw_ctx *ctx, gw_grid g, const int *m, int ng);
int api_check_opts(gw_ctx *ctx, const gw_opts *o);
int api_check_grid(gw_ctx *ctx, gw_grid g);
int api_grid_supported(gw_ctx *ctx, gw_grid g);
int api_begin(gw_ctx *ctx);
void api_set_err(gw_ctx *ctx, const char *msg);
int api_device(gw_ctx *ctx);

// ---- allocation-free update (noalloc.hip) ------------------------------------------------------------
// Resolve this device's address of the fixed scratch array (call with `device` current).
hipError_t noalloc_resolve(int device);
size_t noalloc_scratch_bytes(int nv, int nc, int precision);
size_t noalloc_scratch_limit();

// ---- tile autotuner --------------------------------------------------------------------------------
// Tuned tile for (nr, nv, nc, precision) on the context's device, or -1 if none is cached.
int tuned_tile(gw_ctx *ctx, int nr, int nv, int nc, int precision);
int autotune_impl(gw_ctx *ctx, const float2 *psi_v, int nv, const float2 *psi_c, int nc, int nr, const double *e_v,
                  const double *e_c, int precision, float2 *p_scratch, int *best, double *times_ms, hipStream_t s);

}  // namespace gwi

// Error macros of the host files other than gw_api.cpp (they report through api_set_err).
#define GWX_CHECK(ctx, cond, msg)    \
  do {                               \
    if (!(cond)) {                   \
      gwi::api_set_err((ctx), (msg)); \
      return GW_E_INVAL;             \
    }                                \
  } while (0)

#define GWX_HIP(ctx, call)                                                                                    \
  do {                                                                                                        \
    hipError_t e_ = (call);                                                                                   \
    if (e_ != hipSuccess) {                                                                                   \
      char b_[320];                                                                                           \
      snprintf(b_, sizeof(b_), "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__);  \
      gwi::api_set_err((ctx), b_);                                                                            \
      return GW_E_HIP;                                                                                        \
    }                                                                                                         \
  } while (0)

#define GWX_STATUS(expr)           \
  do {                             \
    int st_ = (expr);              \
    if (st_ != GW_OK) return st_;  \
  } while (0)
