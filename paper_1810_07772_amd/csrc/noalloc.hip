// Allocation-free variant of the rank-K update entry point (P(r,r') = -sum conj(f) f^T with the pair
// products of Eq.(fdef) formed in-kernel), for callers that cannot allocate device memory: code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
//
// The only device memory the update needs beyond its inputs and output is small: the energies
// (nv + nc doubles), the pair-scale table ([nv][ldsc] floats) and, for the scaled FP16 path, the
// per-band exponents.  Here they live in one file-scope device array of fixed size.  Each GPU holds its
// own copy of that array (at its own address) for the life of the process; its device address is
// looked up once per device at context creation, with that device current, and only that address is
// ever passed to copies and kernels.  Every call on one GPU shares the array and overwrites it, so
// calls that overlap on one GPU race; calls on one stream are ordered and safe.
#include <mutex>

#include "gw_internal.h"

namespace gwi {

constexpr size_t kNoallocScratchBytes = size_t(8) << 20;   // 8 MiB per GPU
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kNoallocMaxDevices = 64;
static void *g_scratch_addr[kNoallocMaxDevices];
static std::mutex g_scratch_mu;

hipError_t noalloc_resolve(int device) {
  if (device < 0 || device >= kNoallocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_addr[device] = p;
  return hipSuccess;
}

static void *noalloc_addr(int device) {
  if (device < 0 || device >= kNoallocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_addr[device];
}

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Bytes of scratch one call needs: energies, the scale table, the band exponents (FP16 only).
size_t noalloc_scratch_bytes(int nv, int nc, int precision) {
  size_t b = round256((size_t)(nv + nc) * sizeof(double));
  b += round256(scale_table_floats(nv, nc) * sizeof(float));
  if (precision == GW_SPLIT_FP16_SCALED) b += round256(band_exp_ints(nv, nc) * sizeof(int));
  return b;
}

size_t noalloc_scratch_limit() { return kNoallocScratchBytes; }

}  // namespace gwi

using namespace gwi;

extern "C" int gw_polarizability_r_noalloc(gw_ctx *ctx, const gw_c32 *psi_v, int nv, const gw_c32 *psi_c, int nc,
                                           int nr, const double *e_v, const double *e_c, const gw_opts *opts,
                                           gw_c32 *p_rr, void *stream) {
  GWX_STATUS(api_begin(ctx));
  gw_opts o;
  gw_opts_default(&o);
  if (opts) o = *opts;
  GWX_CHECK(ctx, nv > 0 && nc > 0 && nr > 0, "nv, nc and nr must be positive");
  GWX_CHECK(ctx, psi_v && psi_c && p_rr, "psi_v, psi_c and p_rr must not be NULL");
  GWX_CHECK(ctx, (long long)nv * nc <= (long long)1 << 31 && nr <= 1 << 24, "nv*nc or nr too large");
  GWX_STATUS(api_check_opts(ctx, &o));
  GWX_STATUS(api_check_energies(ctx, e_v, nv, e_c, nc));
  const size_t need = noalloc_scratch_bytes(nv, nc, o.precision);
  if (need > kNoallocScratchBytes) {
    char b[200];
    snprintf(b, sizeof(b), "the allocation-free update needs %zu bytes of scratch for nv = %d, nc = %d; the limit is %zu",
             need, nv, nc, kNoallocScratchBytes);
    api_set_err(ctx, b);
    return GW_E_INVAL;
  }
  if (api_device(ctx) < 0) return GW_OK;
  unsigned char *base = static_cast<unsigned char *>(noalloc_addr(api_device(ctx)));
  GWX_CHECK(ctx, base != nullptr, "the scratch array's device address was not resolved for this device");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double *energy = reinterpret_cast<double *>(base);
  size_t off = round256((size_t)(nv + nc) * sizeof(double));
  float *scale = reinterpret_cast<float *>(base + off);
  const int ldsc = scale_ld(nc);
  off += round256(scale_table_floats(nv, nc) * sizeof(float));
  int *bexp = o.precision == GW_SPLIT_FP16_SCALED ? reinterpret_cast<int *>(base + off) : nullptr;
  GWX_HIP(ctx, hipMemcpyAsync(energy, e_v, (size_t)nv * sizeof(double), hipMemcpyHostToDevice, s));
  GWX_HIP(ctx, hipMemcpyAsync(energy + nv, e_c, (size_t)nc * sizeof(double), hipMemcpyHostToDevice, s));
  GWX_HIP(ctx, launch_scale_table(energy, nv, energy + nv, nc, o.prefactor, scale, ldsc, s));
  if (bexp)
    GWX_HIP(ctx, launch_band_exponents((const float2 *)psi_v, nv, (const float2 *)psi_c, nc, nr, scale, ldsc, bexp, s));
  const int tile = o.tile >= 0 ? o.tile : herk_default_tile(o.precision, nr);
  GWX_HIP(ctx, launch_herk(o.precision, tile, (const float2 *)psi_v, (const float2 *)psi_c, scale, ldsc, bexp,
                           (float2 *)p_rr, nr, nv, nc, o.accumulate, s));
  return GW_OK;
}
