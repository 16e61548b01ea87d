// SAI least-squares problems solved on the current HIP device (setup.hip).
#pragma once

#include <vector>

#include "host.hpp"

namespace ldgmg {

// Solves the problems (each min || C X - E ||_F of Section 2.3.3) in FP64 on the
// GPU; returns per problem whether its X was written (declined problems are
// solved by the host).  Allocates and frees its own device workspace; one
// rocBLAS handle per device is kept for the life of the process.
std::vector<char> gpu_sai_solve(SaiBatch& batch);

}  // namespace ldgmg
