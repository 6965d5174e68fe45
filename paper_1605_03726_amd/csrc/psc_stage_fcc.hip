// psc_stage_fcc.hip -- walk-stage kernels of the face-centred cubic lattice.
#include "psc_stage_impl.h"

namespace psc {

template hipError_t launch_stage_lat<1>(const LatDev *dL, uint32_t g, int grid, int items,
                                        bool disp, hipStream_t s);

}  // namespace psc
