"""MI355X (gfx950) library for the real-space static polarizability build of plane-wave GW.

The computation runs in libgw.so (hand-written HIP kernels, C ABI in include/gw.h); this
package only marshals arguments to it.  There is no CPU fallback: if the library is not
built, every entry point raises."""
from ._lib import (GwError, Context, context, load, tile_names, default_tile_name, pair_products, polarizability_r,
                   polarizability_r_noalloc,  # noqa: F401
                   sphere_transform, polarizability, epsilon, eps_inverse, hpd_inverse, polarizability_batched, autotune,
                   EXPORTS, LIB_PATH, TailModel, tail_target, tail_features, tail_fit_norm, newton_inverse, eps_inverse_newton,
                   orbitals_to_grid, plasmon_pole, pp_eps_inverse, sigma_static,
                   sigma_sex_modes, mfma_rate)
