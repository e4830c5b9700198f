// lbm_host.hpp -- host-side helpers shared by the simulation context and the
// serving engine.
#pragma once

#include <string>

#include "lbm.h"
#include "lbm_common.hpp"

namespace lbm {

// Validate the arguments of one simulation (as lbm_create documents them) and
// fill geometry (sizes, pitch, tile) and FP32 physics constants.  kp.types is
// left null.  Returns LBM_OK or LBM_EINVAL with err set.
lbm_status setup_params(const lbm_grid* grid, const uint8_t* flags, double tau, const lbm_bc* bc, KParams& kp,
                        std::string& err);

// Stored populations per lattice for a geometry and layout.
int64_t lattice_elems(const Geometry& g, int layout);

// Fluid + outlet nodes of a flag array.
int64_t count_updated(const lbm_grid* grid, const uint8_t* flags, const lbm_bc* bc);

} // namespace lbm
