// psc_stage_multi.hip -- the batched walk-stage kernel of an ensemble.
#include "psc_device.h"

namespace psc {

// Stage g of every member lattice of an ensemble in one launch: the chunks of
// all members' stage bins form one work list, so lattices of any size share
// the GPU evenly.  The list's prefix over members (chunks before member r,
// R + 1 entries per stage) is computed once per event by k_multi_prefix,
// after the member records.
constexpr uint32_t kMaxMembers = 4096;

__device__ __forceinline__ uint32_t *chunk_prefix(const LatDev *lats, uint32_t R, uint32_t g) {
  return (uint32_t *)(lats + R) + (size_t)g * (R + 1);
}

// one workgroup per stage: chunks per member (contiguous slices of members
// per thread), then an exclusive scan over the slices
__global__ void __launch_bounds__(kStageThreads) k_multi_prefix(const LatDev *__restrict__ lats,
                                                                uint32_t R, uint32_t chunk) {
  __shared__ uint32_t s_part[kStageThreads];
  const uint32_t g = blockIdx.x, tid = threadIdx.x;
  uint32_t *pre = chunk_prefix(lats, R, g);
  const uint32_t per = (R + kStageThreads - 1) / kStageThreads;
  const uint32_t lo = min(tid * per, R), hi = min(lo + per, R);
  uint32_t run = 0;
  for (uint32_t r = lo; r < hi; ++r) run += (lats[r].sdesc[g].y + chunk - 1) / chunk;
  s_part[tid] = run;
  __syncthreads();
  for (uint32_t d = 1; d < kStageThreads; d <<= 1) {
    const uint32_t add = tid >= d ? s_part[tid - d] : 0u;
    __syncthreads();
    s_part[tid] += add;
    __syncthreads();
  }
  uint32_t acc = s_part[tid] - run;
  for (uint32_t r = lo; r < hi; ++r) {
    pre[r] = acc;
    acc += (lats[r].sdesc[g].y + chunk - 1) / chunk;
  }
  if (tid == kStageThreads - 1) pre[R] = s_part[tid];
}

// The one- and two-item forms ask for four waves per SIMD: the two-item
// form then fits in 128 VGPRs (four of its workgroups per compute unit
// instead of three).  The larger forms need more registers than that.
template <int ITEMS>
__global__ void __launch_bounds__(kStageThreads, ITEMS <= 2 ? 4 : 1)
    k_stage_multi(const LatDev *__restrict__ lats, uint32_t R, uint32_t g) {
  __shared__ StageShared S;
  __shared__ StageStaging<ITEMS> T;
  __shared__ uint32_t s_pre[kMaxMembers + 1];
  __shared__ uint32_t s_tab[kStageTabWordsMax];  // the tables of the chunk's member
  const int tid = threadIdx.x;
  const uint64_t chunk = (uint64_t)kStageThreads * ITEMS;
  const uint32_t *pre = chunk_prefix(lats, R, g);
  for (uint32_t r = tid; r <= R; r += kStageThreads) s_pre[r] = pre[r];
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

hipError_t launch_multi_prefix(const LatDev *lats, uint32_t R, uint32_t stages, int items,
                               hipStream_t s) {
  const int it = items == 1 || items == 2 || items == 8 ? items : 4;  // as launch_stage_multi
  hipLaunchKernelGGL(k_multi_prefix, dim3(stages), dim3(kStageThreads), 0, s, lats, R,
                     (uint32_t)(kStageThreads * it));
  return hipGetLastError();
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
