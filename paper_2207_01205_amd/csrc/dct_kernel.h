// Internal interface of the DCT-basis kernels (fofse_dct.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fofse_kernel.h"

namespace fofse {

// Grid sizes T of the DCT-basis path (the grid is T x T): 16, 32 and 64.
bool dct_size_supported(int T);

// Forward iterations with the orthonormal DCT-II basis for n blocks.  Blocks
// of one support mask share a workgroup (up to 2 kGroup of them, one wavefront each);
// g holds the grouping workspace when p.known is not null.  cosm is the
// device table cos(pi k (2m+1) / (2T)) at [m * T + k], m, k < T.  The model on
// B is written to p.out and the selection record to p.sel / p.coef.
hipError_t launch_dct(const KParams& p, const GroupArgs& g, const double* cosm, int n_cu,
                      hipStream_t stream, const Timing& tm);

}  // namespace fofse
