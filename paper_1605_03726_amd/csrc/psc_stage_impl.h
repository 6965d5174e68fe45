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
  __shared__ uint32_t s_tab[kStageTabWordsMax];
  const LatDev &L = *Lp;
  const uint4 d = L.sdesc[g];  // empty when the lattice does not run this event
  const uint64_t e = d.z | ((uint64_t)d.w << 32);
  const uint32_t c = d.x, n = d.y;
  const uint64_t chunk = (uint64_t)kStageThreads * ITEMS;
  if ((uint64_t)blockIdx.x * chunk >= n) return;
  const uint64_t due = due_of(L, e);
  const uint32_t cmax_next = cmax_after(L, e);
  const RxTabLds tab{s_tab, stage_tab_layout(L.n_species, L.n_rx)};
  for (uint64_t base = (uint64_t)blockIdx.x * chunk; base < n; base += (uint64_t)gridDim.x * chunk)
    stage_chunk<ITEMS, DM, LAT>(L, e, c, base, n, due, cmax_next, tab,
                                base == (uint64_t)blockIdx.x * chunk ? s_tab : nullptr, S, T);
}

// The direct form, for launches made one event at a time from the host: the
// lattice record, the stage's colour, the event and its two tape words
// arrive as arguments (the host draws the stage order as k_begin does and
// holds the tape), and the first chunk's entries are read alongside the
// bin's count.  Its chain of dependent reads before the entries is one
// (the arguments) instead of four (record pointer, stage descriptor, count,
// tape).  PAR is the event's parity, so that every field of the record
// that the stage reads sits at an offset known when compiling and all are
// read in one round.
template <int ITEMS, int DM, int LAT, int PAR>
__global__ void __launch_bounds__(kStageThreads) k_stage_direct(const LatDev L, uint32_t c,
                                                                 uint64_t e_arg, uint64_t due,
                                                                 uint32_t cmax_next) {
  __shared__ StageShared S;
  __shared__ StageStaging<ITEMS> T;
  __shared__ uint32_t s_tab[kStageTabWordsMax];
  const uint64_t e = (e_arg & ~1ull) | (uint64_t)PAR;  // = e_arg
  const uint64_t chunk = (uint64_t)kStageThreads * ITEMS;
  const uint64_t base0 = (uint64_t)blockIdx.x * chunk;
  const RxTabLds tab{s_tab, stage_tab_layout(L.n_species, L.n_rx)};
  stage_chunk<ITEMS, DM, LAT, true>(L, e, c, base0, 0, due, cmax_next, tab, s_tab, S, T);
  const uint32_t n = (uint32_t)min((uint64_t)L.bins[e & 1].count[c], L.cap);
  for (uint64_t base = base0 + (uint64_t)gridDim.x * chunk; base < n; base += (uint64_t)gridDim.x * chunk)
    stage_chunk<ITEMS, DM, LAT>(L, e, c, base, n, due, cmax_next, tab, nullptr, S, T);
}

template <int DM, int LAT, int PAR>
static void launch_stage_direct_par(const LatDev &L, uint32_t c, uint64_t e, uint64_t due,
                                    uint32_t cmax_next, int grid, int items, hipStream_t s) {
  const dim3 G(grid), B(kStageThreads);
  switch (items) {
  case 1: hipLaunchKernelGGL((k_stage_direct<1, DM, LAT, PAR>), G, B, 0, s, L, c, e, due, cmax_next); break;
  case 2: hipLaunchKernelGGL((k_stage_direct<2, DM, LAT, PAR>), G, B, 0, s, L, c, e, due, cmax_next); break;
  default: hipLaunchKernelGGL((k_stage_direct<4, DM, LAT, PAR>), G, B, 0, s, L, c, e, due, cmax_next); break;
  }
}

// items: 1, 2 or 4 (the shapes the host picks for single lattices; larger
// chunks take the descriptor form)
template <int LAT>
hipError_t launch_stage_direct_lat(const LatDev &L, uint32_t c, uint64_t e, uint64_t due,
                                   uint32_t cmax_next, int grid, int items, bool disp,
                                   hipStream_t s) {
  if (disp) {
    if (e & 1) launch_stage_direct_par<1, LAT, 1>(L, c, e, due, cmax_next, grid, items, s);
    else launch_stage_direct_par<1, LAT, 0>(L, c, e, due, cmax_next, grid, items, s);
  } else {
    if (e & 1) launch_stage_direct_par<0, LAT, 1>(L, c, e, due, cmax_next, grid, items, s);
    else launch_stage_direct_par<0, LAT, 0>(L, c, e, due, cmax_next, grid, items, s);
  }
  return hipGetLastError();
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
