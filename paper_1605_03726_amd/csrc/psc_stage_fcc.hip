// psc_stage_fcc.hip -- walk-stage kernels of the face-centred cubic lattice.
#include "psc_stage_impl.h"

namespace psc {

template hipError_t launch_stage_lat<1>(const LatDev *dL, uint32_t g, int grid, int items,
                                        bool disp, hipStream_t s);
template hipError_t launch_stage_direct_lat<1>(const LatDev &L, uint32_t c, uint64_t e,
                                               uint64_t due, uint32_t cmax_next, int grid,
                                               int items, bool disp, hipStream_t s);

}  // namespace psc
