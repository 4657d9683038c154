// Device code of the MI355X (gfx950) lattice Boltzmann elasticity library:
// lbm_common.hpp (descriptor, storage, collision, layouts, reductions),
// lbm_step.hpp (single steps), lbm_fused.hpp (several steps per launch),
// lbm_util.hpp (per-lattice helpers), lbm_small.hpp (whole solves of small
// lattices in one workgroup).
#pragma once

#include "lbm_common.hpp"
#include "lbm_step.hpp"
#include "lbm_fused.hpp"
#include "lbm_wave.hpp"
#include "lbm_util.hpp"
#include "lbm_small.hpp"
