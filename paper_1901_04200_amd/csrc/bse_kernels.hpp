// Launch entry points of the Black-Scholes passes with the Euler scheme on S
// (bse_kernels.hip; internal to the library, the public boundary is
// include/mcaad.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mc_kernels.hpp"

namespace mcaad {

// Pass 1: partial[k][b] = sum over workgroup b's paths of the payoff of
// date-sorted instrument k; store: the spot every K steps into ckpt [nseg][P].
hipError_t launch_bse_pass1(const DevProblem &pb, bool fp64, bool store, const double *theta, double *partial,
                            void *ckpt, int64_t nblocks, hipStream_t stream);
// Pass 2: partial[0][b] = workgroup b's sum of dG/dsigma over its paths, seeded
// with lamD (lambda_i D_i / P, date-sorted); from_ckpt: segments start from
// ckpt, else the forward sweep runs again and writes it.
hipError_t launch_bse_pass2(const DevProblem &pb, bool fp64, bool from_ckpt, const double *theta, const void *lamD,
                            double *partial, void *ckpt, int64_t nblocks, hipStream_t stream);

}  // namespace mcaad
