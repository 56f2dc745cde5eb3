/*
 * gw.h - C ABI of the MI355X (gfx950) static polarizability library.
 *
 * The library builds the static polarizability of a plane-wave GW
 * calculation in real space (paper: "Scalable GW software for quasiparticle
 * properties using OpenAtom", Sec. 4.1 and Sec. 5.1):
 *
 *   f_vc(r)   = conj(u_v(r)) u_c(r) sqrt(p / (E_c - E_v))              Eq.(fdef)
 *   P(r,r')   = - sum_vc conj(f_vc(r)) f_vc(r')                        outer product below Eq.(fdef), N_k = 1
 *   P^(g,r')  = sum_r  exp(-i G_g.r)   P(r,r')                         first transform, Sec. 4.1
 *   P~(g,g')  = sum_r' P^(g,r') exp(+i G_g'.r')                        second transform, Sec. 4.1
 *   eps(g,g') = delta - sqrt(V(q+g)) P~(g,g') sqrt(V(q+g'))            Sec. 5.1
 *   V(q+g)    = 4 pi / (Omega |q+g|^2)                                 Sec. 5.1, Hartree atomic units
 *   eps^-1                                                             Sec. 5.1 (here: FP64 Cholesky)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array arguments are DEVICE pointers unless marked (host).  Arrays are
 *   row-major.  Complex numbers are interleaved {re, im}.
 * - Orbitals: psi[n][nr], grid-normalised (sum_r |psi|^2 = 1), with grid index
 *   r = (i1*n2 + i2)*n3 + i3.
 * - Energies are float64 in Hartree.  Every E_c - E_v must be > 0.
 * - The G-sphere is an ordered host list of Miller triples g_miller[ng][3]
 *   (int32) with |m_d| < n_d/2 and no duplicates; outputs indexed by g follow
 *   that order.  q (host, [3], finite; GW_E_INVAL otherwise) is in crystal units;
 *   the cell is cubic with side a_bohr.
 * - Where |q+G| < 1e-10 * 2pi/a, sqrt(V) is taken as 0 and eps(g,g) is set to
 *   the caller's `head` value (the wings become 0).
 * - Ownership: the caller owns every buffer it passes and the library never
 *   frees them.  The context owns its device workspace, bounded by the cap
 *   given at creation.  Host arrays are read during the call only.
 * - Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *   asynchronous on that stream unless stated otherwise.
 * - Errors: every call returns a gw_status; no exception crosses the ABI.  All
 *   argument checks run on the host before any device work is queued; on a
 *   failed check nothing is launched and gw_last_error(ctx) describes it.
 *   A context is not thread-safe: use one per host thread.
 * - Dry-run contexts (gw_create with hip_device = -1) run every argument
 *   check and return GW_OK without touching any device; they exist so that
 *   callers can validate arguments on machines without a GPU.
 */
#ifndef GW_H
#define GW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gw_ctx gw_ctx;
typedef struct { float re, im; } gw_c32;
typedef struct { double re, im; } gw_c64;
typedef struct { int n1, n2, n3; double a_bohr; } gw_grid;

enum gw_status {
  GW_OK = 0,
  GW_E_INVAL = 1,        /* bad argument (shape, pointer, energy order, sphere) */
  GW_E_NOMEM = 2,        /* the workspace cap or the device memory is exceeded */
  GW_E_HIP = 3,          /* a HIP runtime call or kernel launch failed */
  GW_E_NOTPD = 4,        /* eps is not positive definite (pivot index in gw_last_error) */
  GW_E_UNSUPPORTED = 5   /* valid request this build cannot serve (e.g. a grid size) */
};

enum gw_precision {
  GW_FP32 = 0,               /* FP32 operands on FP32 MFMA, FP32 accumulation */
  GW_SPLIT_BF16 = 1,         /* f = hi + lo in BF16 (RNE); hi*hi + hi*lo + lo*hi on BF16 MFMA */
  GW_SPLIT_FP16_SCALED = 2   /* as split BF16 in FP16, each occupied band scaled by a power of two */
};

typedef struct {
  int precision;      /* enum gw_precision */
  double prefactor;   /* p of f_vc = conj(u_v) u_c sqrt(p/(E_c - E_v)); 1 by default, 2 is the paper's spin factor */
  int accumulate;     /* 0: P(r,r') := result; 1: P(r,r') += result (p_rr must be the caller's buffer) */
  int tile;           /* -1: the tuned or default tile of the update kernel; otherwise an index from gw_tile_count() */
} gw_opts;

/* Fills opts with {GW_FP32, 1.0, 0, -1}. */
void gw_opts_default(gw_opts *opts);

/* Library version as 10000*major + 100*minor + patch. */
int gw_version(void);

/* Human-readable name of a status code (static storage). */
const char *gw_status_string(int status);

/* Create a context on HIP device `hip_device` (or a dry-run context for -1).
 * workspace_cap_bytes bounds the device memory the context may allocate for
 * its own scratch (0 = no bound).  On success *ctx is set and GW_OK returned. */
int gw_create(gw_ctx **ctx, int hip_device, size_t workspace_cap_bytes);

/* Release the context and its workspace.  Waits for the context's pending work. */
int gw_destroy(gw_ctx *ctx);

/* Text of the last failure on this context ("" if none).  Valid until the next call on ctx. */
const char *gw_last_error(const gw_ctx *ctx);

/* Bytes of device workspace the context currently holds. */
size_t gw_workspace_bytes(const gw_ctx *ctx);

/* Number of tile configurations of the rank-k update kernel, the name of one, and the one used
 * for `precision` at grid size nr when gw_opts.tile is -1 (-1 for an unknown precision). */
int gw_tile_count(void);
const char *gw_tile_name(int tile);
int gw_default_tile(int precision, int nr);

/* Rate reference for the split-precision update (not a step of the method; for benchmarks that
 * compare the update with what the matrix cores reach on this device).  Launches `grid`
 * workgroups of 512 threads; each of the 8 waves runs n_iter iterations of twelve BF16
 * 32x32x16 MFMAs (12 * 32768 flop) whose operands come from 16 KB of LDS copied from `words`.
 * The executed flop count is grid * 8 * n_iter * 393216; the caller times the launch on `stream`.
 *   words  device, 4096 uint32 (2048 BF16 pairs; finite values keep the sums finite), read only
 *   out    device, grid * 512 floats: one sum per thread, written so the products stay live
 * Errors: GW_E_INVAL for NULL pointers, n_iter < 1 or grid outside [1, 2^24]. */
int gw_mfma_rate(gw_ctx *ctx, const uint32_t *words, int n_iter, int grid, float *out, void *stream);

/* ---------------------------------------------------------------------------
 * Orbitals on the grid from their plane-wave coefficients (Sec. 4.1, the
 * transform of the wavefunctions to real space that precedes the pair
 * products; Table 1's first row):
 *   psi[n][r] = N_r^(-1/2) sum_m coeff[n][m] exp(+2 pi i (m1 i1/n1 + m2 i2/n2 + m3 i3/n3)),
 *   r = (i1*n2 + i2)*n3 + i3, so grid-orthonormal orbitals come from orthonormal
 *   coefficient vectors.
 *   coeff [nb][npw] complex64 (device, read only); pw_miller host [npw][3]
 *   distinct Miller triples with |m_d| < n_d/2; psi [nb][N_r] complex64
 *   (device), written entirely.  FP32 transform: three pruned 1-D passes.
 *   Grid sides as for gw_sphere_transform (else GW_E_UNSUPPORTED).
 * ------------------------------------------------------------------------- */
int gw_orbitals_to_grid(gw_ctx *ctx, const gw_c32 *coeff, int nb, int npw, gw_grid grid, const int *pw_miller,
                        gw_c32 *psi, void *stream);

/* ---------------------------------------------------------------------------
 * Pair products, Eq.(fdef):  f_out[v*nc + c][r] = conj(psi_v[v][r]) psi_c[c][r] sqrt(p/(E_c - E_v)).
 *   psi_v [nv][nr], psi_c [nc][nr] complex64; e_v[nv], e_c[nc] (host, Hartree);
 *   f_out [nv*nc][nr] complex64, written entirely.  FP32 product of the FP32
 *   inputs with the scale rounded once from FP64.
 * ------------------------------------------------------------------------- */
int gw_pair_products(gw_ctx *ctx, const gw_c32 *psi_v, int nv, const gw_c32 *psi_c, int nc, int nr,
                     const double *e_v, const double *e_c, double prefactor, gw_c32 *f_out, void *stream);

/* ---------------------------------------------------------------------------
 * Real-space polarizability (pair products fused into the Hermitian rank-K
 * update, K = nv*nc):  P(r,r') = -sum_vc conj(f_vc(r)) f_vc(r')  (+ P if accumulate).
 *   p_rr [nr][nr] complex64, both triangles written (P is Hermitian).
 *   The pair products are formed inside the update kernel and never stored.
 * ------------------------------------------------------------------------- */
int gw_polarizability_r(gw_ctx *ctx, const gw_c32 *psi_v, int nv, const gw_c32 *psi_c, int nc, int nr,
                        const double *e_v, const double *e_c, const gw_opts *opts, gw_c32 *p_rr,
                        void *stream);

/* ---------------------------------------------------------------------------
 * The same update as gw_polarizability_r, allocating nothing: for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Inputs, output, options and results
 * are those of gw_polarizability_r, except that opts->tile = -1 means the default
 * tile of the precision (no autotuner lookup).  The energies, the pair-scale table
 * and the FP16 band exponents go to a fixed 8 MiB device array that each GPU holds
 * for the life of the process (its address is resolved once per device by
 * gw_create): calls needing more than 8 MiB, i.e. about
 * 8 (nv + nc) + 8 nv ceil32(nc) (+ 4 (5 nv + nc) for FP16) bytes, return
 * GW_E_INVAL with the figure in gw_last_error.  Every call on one GPU shares that
 * array, so calls that overlap on one GPU (different streams or host threads)
 * race; calls on one stream are ordered.  No hipMalloc, hipFree or other
 * allocating call is made.
 * ------------------------------------------------------------------------- */
int gw_polarizability_r_noalloc(gw_ctx *ctx, const gw_c32 *psi_v, int nv, const gw_c32 *psi_c, int nc, int nr,
                                const double *e_v, const double *e_c, const gw_opts *opts, gw_c32 *p_rr,
                                void *stream);

/* ---------------------------------------------------------------------------
 * Both transforms of Sec. 4.1 restricted to the sphere:
 *   p_gg[g][g'] = sum_{r,r'} exp(-i G_g.r) p_rr[r][r'] exp(+i G_g'.r').
 *   p_rr [nr][nr] complex64 (read only), g_miller host [ng][3], p_gg [ng][ng] complex64.
 *   Grid sides n_d must be in {4, 5, 6, 8, 9, 10, 12, 15, 16, 18, 20, 24, 27, 30, 32, 36, 40, 48}
 *   (else GW_E_UNSUPPORTED).
 * ------------------------------------------------------------------------- */
int gw_sphere_transform(gw_ctx *ctx, const gw_c32 *p_rr, gw_grid grid, const int *g_miller, int ng,
                        gw_c32 *p_gg, void *stream);

/* The same transforms for a Hermitian P(r,r') (as gw_polarizability_r writes it): P~ is formed
 * from P's upper triangle alone, P = M + M^H with M the strict upper triangle plus half the real
 * diagonal, so only that half of p_rr is read; P~ = F M F^H + (F M F^H)^H.  Entries below the
 * diagonal and the imaginary part of the diagonal are then ignored.  This form needs n2 = n3 (each
 * row's i1 planes are transformed over (i2, i3) by one wave); on other grids the strided transform of
 * the whole p_rr runs, so p_rr must hold both triangles.  Arguments as gw_sphere_transform. */
int gw_sphere_transform_herm(gw_ctx *ctx, const gw_c32 *p_rr, gw_grid grid, const int *g_miller, int ng,
                             gw_c32 *p_gg, void *stream);

/* ---------------------------------------------------------------------------
 * The whole build from orbitals to P~(g,g') (a rank-K update then both transforms).
 *   psi_occ [nv][nr], psi_unocc [nc][nr] with nr = n1*n2*n3; q (host) [3] enters
 *   only the sphere, the Coulomb step and the choice of transform: P is Hermitian, so
 *   the transforms use its upper triangle (as gw_sphere_transform_herm) unless
 *   accumulate is set or the sphere holds a vector with 0 < |q+m| < 0.01 (crystal
 *   units), whose Coulomb weight would magnify that form's rounding of the head row;
 *   then all of P is transformed.
 *   p_rr: [nr][nr] buffer that receives P(r,r'), or NULL to use workspace.
 *   p_gg: [ng][ng] complex64 output.
 * ------------------------------------------------------------------------- */
int gw_polarizability(gw_ctx *ctx, const gw_c32 *psi_occ, int nv, const gw_c32 *psi_unocc, int nc,
                      const double *e_v, const double *e_c, gw_grid grid, const double *q,
                      const int *g_miller, int ng, const gw_opts *opts, gw_c32 *p_rr, gw_c32 *p_gg,
                      void *stream);

/* ---------------------------------------------------------------------------
 * eps of Sec. 5.1 in FP64:  eps[g][g'] = delta - sv(g) * H(g,g') * sv(g'), with
 * sv = sqrt(4 pi / (Omega |q+G|^2)) (0 where |q+G| vanishes; then eps[g][g] = head)
 * and H the Hermitian part (P~ + P~^H)/2 of the single-precision input.
 *   p_gg [ng][ng] complex64, eps_out [ng][ng] complex128.
 * ------------------------------------------------------------------------- */
int gw_epsilon(gw_ctx *ctx, const gw_c32 *p_gg, int ng, gw_grid grid, const double *q, const int *g_miller,
               double head, gw_c64 *eps_out, void *stream);

/* ---------------------------------------------------------------------------
 * eps^-1 in FP64: builds eps as gw_epsilon does, factors eps = L L^H (Cholesky,
 * eps is Hermitian positive definite because P~ is negative semidefinite),
 * then eps^-1 = L^-H L^-1.  head: NaN means 1.0.
 *   eps_inv [ng][ng] complex128 output.
 * Synchronises `stream` to read the pivot flag; returns GW_E_NOTPD (pivot in
 * gw_last_error) if a pivot is not positive.
 * ------------------------------------------------------------------------- */
int gw_eps_inverse(gw_ctx *ctx, const gw_c32 *p_gg, int ng, gw_grid grid, const double *q, const int *g_miller,
                   double head, gw_c64 *eps_inv, void *stream);

/* Inverse of a Hermitian positive definite complex128 matrix a[n][n] (lower
 * triangle read) by the same Cholesky path; out [n][n].  Synchronises `stream`. */
int gw_hpd_inverse(gw_ctx *ctx, const gw_c64 *a, int n, gw_c64 *out, void *stream);

/* ---------------------------------------------------------------------------
 * Inverse by the Newton iteration of Sec. 5.1, for any nonsingular complex128
 * a[n][n]:  X_{n+1} = X_n (2I - A X_n), X_0 = alpha A^H with
 * alpha = 1 / max_i sum_j |(A A^H)_ij| (absolute values, so that the iteration
 * converges); stops when max_ij |X_{n+1} - X_n| < tol.  Every product runs on
 * the FP64 MFMA GEMM.  *iterations (host) receives the iteration count and
 * history (host, optional, [max_iter]) the max change of each iteration.
 * Synchronises `stream` once per iteration.  Returns GW_E_UNSUPPORTED if tol is
 * not reached in max_iter iterations (out then holds the last iterate) and
 * GW_E_NOTPD if the iteration diverges.
 * ------------------------------------------------------------------------- */
int gw_newton_inverse(gw_ctx *ctx, const gw_c64 *a, int n, double tol, int max_iter, gw_c64 *out, int *iterations,
                      double *history, void *stream);

/* eps^-1 as gw_eps_inverse, but by the Newton iteration above (the paper's method). */
int gw_eps_inverse_newton(gw_ctx *ctx, const gw_c32 *p_gg, int ng, gw_grid grid, const double *q, const int *g_miller,
                          double head, double tol, int max_iter, gw_c64 *eps_inv, int *iterations, double *history,
                          void *stream);

/* ---------------------------------------------------------------------------
 * Plasmon-pole model (the paper's section on the dynamic inverse dielectric
 * matrix, vdLH-type poles on the polarization part of W):
 *   S = sqrt(V) (eps^-1 - I) sqrt(V),  S = A diag(sigma) A^H   (Eq.(eigdecomp)),
 *   omega_a^2 = (A^H M A)_aa / |sigma_a|,                        (Eq.(ppfreq))
 *   M(g,g') = V(q+g) V(q+g') [(q+g).(q+g')] rho_{g-g'},
 *   rho(r) = occupation * sum_v |psi_v(r)|^2,  rho_g = sum_r rho(r) exp(-i G.r)
 * (grid-normalised orbitals, so rho_0 is the electron count; differences g-g'
 * are taken modulo the grid).  The printed Eq.(ppfreq) divides by sigma_a; since
 * S is negative semidefinite and M positive semidefinite, |sigma_a| is used,
 * which is what the sum rule gives through the retarded pole form.
 * The n_modes most negative sigma (n_modes <= min(24, ng)) come from a block
 * subspace iteration on -S (block of 32, Rayleigh-Ritz every iteration, FP64)
 * stopped when max_a ||S a_a - sigma_a a_a|| <= tol |sigma_0|.
 *   eps_inv [ng][ng] complex128 (device), q host [3] crystal units, g_miller
 *   host [ng][3], psi_v [nv][N_r] complex64 (device);
 *   sigma, omega [n_modes] float64 (device), ascending sigma (most negative
 *   first); modes [ng][n_modes] complex128 (device), column a = A_a (unit norm,
 *   arbitrary phase); iterations and residual (optional) on the host.
 * Synchronises `stream` once per iteration.  GW_E_UNSUPPORTED if tol is not
 * reached in max_iter iterations (the outputs then hold the last Ritz pairs).
 * ------------------------------------------------------------------------- */
int gw_plasmon_pole(gw_ctx *ctx, const gw_c64 *eps_inv, int ng, gw_grid grid, const double *q, const int *g_miller,
                    const gw_c32 *psi_v, int nv, double occupation, int n_modes, double tol, int max_iter,
                    double *sigma, double *omega, gw_c64 *modes, int *iterations, double *residual, void *stream);

/* Pole form Eq.(ppform) turned back into the dynamic inverse dielectric matrix:
 *   out[f] = I + V^-1/2 S(w_f) V^-1/2,  S(w) = sum_a A_a sigma_a omega_a^2 / (omega_a^2 - w^2) A_a^H,
 * for each host frequency freqs[f] (Hartree); rows and columns with sqrt(V) = 0 take
 * their values from eps_inv_static.  modes/sigma/omega as returned by
 * gw_plasmon_pole (device); out [nf][ng][ng] complex128 (device).  A frequency
 * equal to some omega_a gives infinities (the pole). */
int gw_pp_eps_inverse(gw_ctx *ctx, const gw_c64 *eps_inv_static, int ng, gw_grid grid, const double *q,
                      const int *g_miller, const gw_c64 *modes, const double *sigma, const double *omega, int n_modes,
                      const double *freqs, int nf, gw_c64 *out, void *stream);

/* ---------------------------------------------------------------------------
 * Static self-energy matrix elements in g-space (the paper's self-energy
 * section, one q, N_k = 1), for a band list n (psi_n [nn][N_r]) and the
 * occupied set v (psi_v [nv][N_r]), both complex64 on the device:
 *   f~_g^{nv} = sum_r exp(-i G_g.r) conj(u_n(r)) u_v(r)         (FP32 transform)
 *   sigma_x[n][n']   = -sum_g V(q+g) sum_v f~_g^{nv} conj(f~_g^{n'v})
 *   sigma_sex[n][n'] = -sum_v sum_{g,g'} f~_g^{nv} S(g,g') conj(f~_g'^{n'v}),
 *                      S = sqrt(V) (eps^-1 - I) sqrt(V)           (T form)
 * with FP64 contractions (the T = S conj(f~) product on the FP64 MFMA GEMM).
 *   eps_inv [ng][ng] complex128 (device; may be NULL when sigma_sex is NULL);
 *   sigma_x, sigma_sex [nn][nn] complex128 (device), either may be NULL.
 *   nn <= 256; grid sides as for gw_sphere_transform.
 * ------------------------------------------------------------------------- */
int gw_sigma_static(gw_ctx *ctx, const gw_c32 *psi_n, int nn, const gw_c32 *psi_v, int nv, gw_grid grid,
                    const double *q, const int *g_miller, int ng, const gw_c64 *eps_inv, gw_c64 *sigma_x,
                    gw_c64 *sigma_sex, void *stream);

/* Screened exchange in the eigen form: zeta_a^{nv} = sum_g f~_g^{nv} A(g,a),
 *   sigma_sex[n][n'] = -sum_a sigma_a sum_v zeta_a^{nv} conj(zeta_a^{n'v}),
 * with modes [ng][n_modes] complex128 and sigma [n_modes] float64 as returned by
 * gw_plasmon_pole (device). */
int gw_sigma_sex_modes(gw_ctx *ctx, const gw_c32 *psi_n, int nn, const gw_c32 *psi_v, int nv, gw_grid grid,
                       const int *g_miller, int ng, const gw_c64 *modes, const double *sigma, int n_modes,
                       gw_c64 *sigma_sex, void *stream);

/* ---------------------------------------------------------------------------
 * Batched q-points (P^q is defined per q, Eq.(staticpol)): each job j runs the
 * whole build and eps^-1 for its own unoccupied set, energies, q and sphere,
 * sharing the occupied set.  The launch sequence of all jobs (kernels only) is
 * captured into one HIP graph, cached in the context and replayed while the
 * shapes, pointers, q, sphere lists, head and options stay the same; energies
 * are re-read on every call.  Inside the graph the update of job j+1 overlaps
 * the transforms and inverse of job j (two P(r,r') workspace buffers).  Tiles:
 * opts->tile if >= 0, else the tuned tile, tuning first where none is cached.
 *   nq in [1, 64]; jobs (host) [nq]; job pointers are device pointers except
 *   e_c and g_miller (host).  accumulate must be 0.
 *   Synchronises `stream`; GW_E_NOTPD names the first job whose eps failed.
 * ------------------------------------------------------------------------- */
typedef struct {
  const gw_c32 *psi_unocc;   /* [nc][nr] */
  int nc;
  const double *e_c;         /* host [nc] */
  double q[3];
  const int *g_miller;       /* host [ng][3] */
  int ng;
  gw_c32 *p_gg;              /* [ng][ng] out */
  gw_c64 *eps_inv;           /* [ng][ng] out, or NULL to skip the inverse */
} gw_qjob;

int gw_polarizability_batched(gw_ctx *ctx, const gw_c32 *psi_occ, int nv, const double *e_v, gw_grid grid,
                              int nq, const gw_qjob *jobs, const gw_opts *opts, double head, void *stream);

/* Number of batched-q graphs this context has captured so far (a replay of a cached graph does not
 * count; a call whose shapes, pointers, q, spheres, head or options differ from the cached graph's
 * captures a new one).  0 for NULL or a context that never ran a batch. */
int gw_graph_captures(const gw_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Tile autotuner of the rank-K update: times every tile of `precision` on the
 * first min(nv, 8) occupied bands of these inputs (same N_r and Nc) and caches
 * the fastest for (device arch, nr, nv, nc, precision) in the context (and
 * appends it to the file named by the environment variable GW_AUTOTUNE_CACHE
 * when set; that file is read back by later contexts).  Calls with tile = -1
 * then use the tuned tile.  p_scratch: device [nr][nr] complex64 the timing
 * launches overwrite.  best_tile (host) receives the choice; times_ms (host,
 * [gw_tile_count()], optional) the time of each tile (-1 where the tile does
 * not implement the precision).  Synchronises `stream`.
 * ------------------------------------------------------------------------- */
int gw_autotune(gw_ctx *ctx, const gw_c32 *psi_v, int nv, const gw_c32 *psi_c, int nc, int nr, const double *e_v,
                const double *e_c, int precision, gw_c32 *p_scratch, int *best_tile, double *times_ms, void *stream);

/* ===========================================================================
 * Learned band-tail correction of the truncated unoccupied-band sum (the band
 * truncation the paper lists as the first technical issue of Eq.(Pstatic)).
 *   features x_G = (|q+G| [1/Bohr], log|Re P~_Nc(G,G)|, Nc/N_g, E_max [Ha]),
 *   o_G = MLP(x_G): 4 -> 128 -> 128 -> 33, SiLU, BF16 weights, FP32 arithmetic,
 *         inputs normalised by the stored mean and std,
 *   s_G = |Re P~_Nc(G,G)|, d_G = softplus(o_G0) s_G, u_Gk = (o_G,1+k + i o_G,17+k) sqrt(s_G) for
 *   k < rank (zero for k >= rank; rank <= 16 is a model setting, chosen on validation systems),
 *   dP~ = -(diag(d) + U U^H)  (negative semidefinite, like the missing tail),
 *   training loss ||dP~ - T||_F^2 / ||T||_F^2 with T = H(P~_4Nc) - H(P~_Nc), H(X) = (X + X^H)/2,
 *   minimised with Adam on an FP32 master copy of the parameters.
 * ========================================================================= */
#define GW_TAIL_NWEIGHT 21120  /* 4*128 + 128*128 + 128*33 BF16 weights                       */
#define GW_TAIL_NBIAS 289      /* 128 + 128 + 33 FP32 biases                                  */
#define GW_TAIL_NPARAM 21409   /* master layout: W1[4][128] b1 W2[128][128] b2 W3[128][33] b3  */

typedef struct {
  void *w;        /* device BF16 [GW_TAIL_NWEIGHT]: W1, W2, W3, each [inputs][outputs] row-major   */
  float *b;       /* device FP32 [GW_TAIL_NBIAS]: b1, b2, b3                                      */
  float *norm;    /* device FP32 [16]: feature mean[4], std[4], training box lo[4], hi[4] (raw)   */
  int rank;       /* columns of U in use, 0..16 (0: diagonal correction only); outputs of the other */
                  /* columns are ignored and receive no gradient                                    */
} gw_mlp;

typedef struct {
  float *master;  /* device FP32 [GW_TAIL_NPARAM] parameters (master copy)                        */
  float *m, *v;   /* device FP32 [GW_TAIL_NPARAM] Adam moments (zero-initialised by the caller)     */
  float *grad;    /* device FP32 [GW_TAIL_NPARAM] gradient of the last step (written)             */
  int step;       /* steps taken so far; each train step increments it (bias corrections 1 - beta^step) */
  float lr, beta1, beta2, eps;
} gw_adam;

/* Writes w->w (BF16, round to nearest even) and w->b from an FP32 master copy [GW_TAIL_NPARAM]. */
int gw_tail_init(gw_ctx *ctx, gw_mlp *w, const float *master, void *stream);

/* Training target T = H(p_full) - H(p_trunc), all [ng][ng] complex64. */
int gw_tail_target(gw_ctx *ctx, const gw_c32 *p_full, const gw_c32 *p_trunc, int ng, gw_c32 *target, void *stream);

/* Raw features [ng][4] of the truncated build p_gg (nc unoccupied bands, highest energy e_max in
 * Hartree) on the sphere g_miller (host) around q (host). */
int gw_tail_features(gw_ctx *ctx, const gw_c32 *p_gg, int ng, gw_grid grid, const double *q, const int *g_miller,
                     int nc, double e_max, float *feat, void *stream);

/* MLP outputs o [ng][33] for raw features feat [ng][4]. */
int gw_tail_forward(gw_ctx *ctx, const gw_mlp *w, const float *feat, int ng, float *out, void *stream);

/* One training step on one system: forward, loss (written to the device float *loss_out),
 * gradient (opt->grad), Adam update of opt->master and refresh of w->w, w->b; opt->step += 1.
 * target [ng][ng] must be Hermitian (as gw_tail_target makes it). */
int gw_tail_train_step(gw_ctx *ctx, gw_mlp *w, gw_adam *opt, const float *feat, const gw_c32 *target, int ng,
                       float *loss_out, void *stream);

/* Training steps replayed from captured HIP graphs: step k trains on system j = order[k] exactly as
 * gw_tail_train_step would (feats[j] [ngs[j]][4] and targets[j] [ngs[j]][ngs[j]] are device arrays;
 * feats, targets, ngs and order are host arrays) and writes that step's loss to loss_out[j] (device
 * FP32 [nsys]).  The launch sequence of one step on one system is captured once into a graph, cached
 * in the context while the model, optimiser, system, workspace and hyperparameters stay the same, and
 * launched once per step; the Adam step count is kept on the device inside the graphs.
 * opt->step += nsteps.  Only kernels are captured (no memsets, no allocation). */
int gw_tail_train_steps(gw_ctx *ctx, gw_mlp *w, gw_adam *opt, int nsys, const float *const *feats,
                        const gw_c32 *const *targets, const int *ngs, int nsteps, const int *order, float *loss_out,
                        void *stream);

/* Number of training-step graphs cached in the context (0 for NULL). */
int gw_tail_graph_count(const gw_ctx *ctx);

/* Feature statistics of a training set into norm (device FP32 [16]): mean[4] and population std[4]
 * (1 where a feature is constant to 1e-12 of max(1, |mean|)) over all rows of the nsys feature
 * arrays feats[i] [ngs[i]][4] (device pointers in a host array), then the training box min[4],
 * max[4].  Accumulated in FP64. */
int gw_tail_fit_norm(gw_ctx *ctx, int nsys, const float *const *feats, const int *ngs, float *norm, void *stream);

/* Parts of the training loss of the current weights on one system, into parts (device FP32 [4]):
 * ||offdiag(dP~ - T)||_F^2, ||offdiag(T)||_F^2, ||diag(dP~ - T)||^2, ||diag(T)||^2, so that
 * loss = (parts[0] + parts[2]) / (parts[1] + parts[3]).  Used to judge the rank on validation. */
int gw_tail_residual_parts(gw_ctx *ctx, const gw_mlp *w, const float *feat, const gw_c32 *target, int ng, float *parts,
                           void *stream);

/* The training loss of the current weights on one system, into the device float *loss_out
 * (forward and loss only; no gradient, no update). */
int gw_tail_loss(gw_ctx *ctx, const gw_mlp *w, const float *feat, const gw_c32 *target, int ng, float *loss_out,
                 void *stream);

/* Corrected build p_corr = p_trunc + dP~ [ng][ng].  If any feature lies outside the training box
 * widened by 5% of its width on each side, *used_fallback (host) is set to 1, p_corr is not
 * written, and the caller runs the plain larger-Nc build instead; otherwise *used_fallback = 0.
 * Synchronises `stream`. */
int gw_tail_correct(gw_ctx *ctx, const gw_mlp *w, const gw_c32 *p_trunc, int ng, const float *feat, gw_c32 *p_corr,
                    int *used_fallback, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GW_H */
