// psc_stage_impl.h -- the single-lattice walk-stage kernel and its launcher,
// instantiated per lattice kind by psc_stage_hcp.hip and psc_stage_fcc.hip
// (separate translation units so that they compile in parallel).
#pragma once

#include "psc_device.h"

namespace psc {

template <int ITEMS, int DM, int LAT>
__global__ void __launch_bounds__(kStageThreads) k_stage(const LatDev *__restrict__ Lp, uint32_t g) {
  __shared__ StageShared S;
  __shared__ StageStaging<ITEMS> T;
  const LatDev &L = *Lp;
  const uint4 d = L.sdesc[g];  // empty when the lattice does not run this event
  const uint64_t e = d.z | ((uint64_t)d.w << 32);
  const uint32_t c = d.x, n = d.y;
  const uint64_t chunk = (uint64_t)kStageThreads * ITEMS;
  for (uint64_t base = (uint64_t)blockIdx.x * chunk; base < n; base += (uint64_t)gridDim.x * chunk)
    stage_chunk<ITEMS, DM, LAT>(L, e, c, base, n, S, T);
}

template <int DM, int LAT>
static void launch_stage_dm(const LatDev *dL, uint32_t g, int grid, int items, hipStream_t s) {
  const dim3 G(grid), B(kStageThreads);
  switch (items) {
  case 1: hipLaunchKernelGGL((k_stage<1, DM, LAT>), G, B, 0, s, dL, g); break;
  case 2: hipLaunchKernelGGL((k_stage<2, DM, LAT>), G, B, 0, s, dL, g); break;
  case 8: hipLaunchKernelGGL((k_stage<8, DM, LAT>), G, B, 0, s, dL, g); break;
  case 16: hipLaunchKernelGGL((k_stage<16, DM, LAT>), G, B, 0, s, dL, g); break;
  default: hipLaunchKernelGGL((k_stage<4, DM, LAT>), G, B, 0, s, dL, g); break;
  }
}

template <int LAT>
hipError_t launch_stage_lat(const LatDev *dL, uint32_t g, int grid, int items, bool disp,
                            hipStream_t s) {
  if (disp) launch_stage_dm<1, LAT>(dL, g, grid, items, s);
  else launch_stage_dm<0, LAT>(dL, g, grid, items, s);
  return hipGetLastError();
}

}  // namespace psc
