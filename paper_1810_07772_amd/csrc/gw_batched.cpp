// Batched q-points (placeholder until the graph path lands).
#include "gw_internal.h"

void gwi::batched_release(gw_ctx *ctx) { (void)ctx; }

extern "C" int gw_polarizability_batched(gw_ctx *ctx, const gw_c32 *psi_occ, int nv, const double *e_v, gw_grid grid,
                                         int nq, const gw_qjob *jobs, const gw_opts *opts, double head, void *stream) {
  (void)psi_occ; (void)nv; (void)e_v; (void)grid; (void)nq; (void)jobs; (void)opts; (void)head; (void)stream;
  if (!ctx) return GW_E_INVAL;
  return GW_E_UNSUPPORTED;
}
