// psc_stage_multi.hip -- the batched walk-stage kernel of an ensemble.
#include "psc_device.h"

namespace psc {

// Stage g of every member lattice of an ensemble in one launch: the chunks of
// all members' stage bins form one work list (prefix over members, built in
// LDS by every workgroup), so lattices of any size share the GPU evenly.
constexpr uint32_t kMaxMembers = 4096;

template <int ITEMS>
__global__ void __launch_bounds__(kStageThreads) k_stage_multi(const LatDev *__restrict__ lats,
                                                               uint32_t R, uint32_t g) {
  __shared__ StageShared S;
  __shared__ StageStaging<ITEMS> T;
  __shared__ uint32_t s_pre[kMaxMembers + 1];
  __shared__ uint32_t s_part[kStageThreads];
  __shared__ uint32_t s_tab[kStageTabWordsMax];  // the tables of the chunk's member
  const int tid = threadIdx.x;
  const uint64_t chunk = (uint64_t)kStageThreads * ITEMS;
  // chunks per member (contiguous slices of members per thread), then an
  // exclusive scan over the slices
  const uint32_t per = (R + kStageThreads - 1) / kStageThreads;
  const uint32_t lo = min((uint32_t)tid * per, R), hi = min(lo + per, R);
  uint32_t run = 0;
  for (uint32_t r = lo; r < hi; ++r) {
    const uint32_t n = lats[r].sdesc[g].y;
    s_pre[r] = run;
    run += (uint32_t)((n + chunk - 1) / chunk);
  }
  s_part[tid] = run;
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (int t = 0; t < kStageThreads; ++t) {
      const uint32_t x = s_part[t];
      s_part[t] = acc;
      acc += x;
    }
    s_pre[R] = acc;
  }
  __syncthreads();
  for (uint32_t r = lo; r < hi; ++r) s_pre[r] += s_part[tid];
  __syncthreads();
  const uint32_t total = s_pre[R];
  uint32_t tab_member = ~0u;  // whose tables s_tab holds
  for (uint32_t q = blockIdx.x; q < total; q += gridDim.x) {
    // member owning chunk q: last r with s_pre[r] <= q
    uint32_t a = 0, b = R;
    while (b - a > 1) {
      const uint32_t m = (a + b) >> 1;
      if (s_pre[m] <= q) a = m;
      else b = m;
    }
    const LatDev &L = lats[a];
    const uint4 d = L.sdesc[g];
    const uint64_t e = d.z | ((uint64_t)d.w << 32);
    const uint64_t due = due_of(L, e);
    const uint32_t cmax_next = cmax_after(L, e);
    const uint64_t base = (uint64_t)(q - s_pre[a]) * chunk;
    const RxTabLds tab{s_tab, stage_tab_layout(L.n_species, L.n_rx)};
    uint32_t *fill = tab_member == a ? nullptr : s_tab;  // a new member: load its tables
    tab_member = a;
    if (L.geo.fcc) stage_chunk<ITEMS, 2, 1>(L, e, d.x, base, d.y, due, cmax_next, tab, fill, S, T);
    else stage_chunk<ITEMS, 2, 0>(L, e, d.x, base, d.y, due, cmax_next, tab, fill, S, T);
  }
}

hipError_t launch_stage_multi(const LatDev *lats, uint32_t R, uint32_t g, int grid, int items,
                              hipStream_t s) {
  switch (items) {
  case 1: hipLaunchKernelGGL(k_stage_multi<1>, dim3(grid), dim3(kStageThreads), 0, s, lats, R, g); break;
  case 2: hipLaunchKernelGGL(k_stage_multi<2>, dim3(grid), dim3(kStageThreads), 0, s, lats, R, g); break;
  case 8: hipLaunchKernelGGL(k_stage_multi<8>, dim3(grid), dim3(kStageThreads), 0, s, lats, R, g); break;
  default: hipLaunchKernelGGL(k_stage_multi<4>, dim3(grid), dim3(kStageThreads), 0, s, lats, R, g); break;
  }
  return hipGetLastError();
}

uint32_t max_members() { return kMaxMembers; }

}  // namespace psc
