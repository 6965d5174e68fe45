// psc_kernels.hip -- gfx950 kernels of the lattice walk.
//
// One diffusion event e of a lattice is four kinds of launch, in order:
//   k_begin   one workgroup: the event's random stage order, the first-order
//             reactions over the interval since the previous event (2.4.1),
//             and id assignment + binning of their newborns;
//   k_stage   16 launches, one per colour stage in the event's order: every
//             molecule whose voxel has that colour attempts one hop (2.3) and
//             fires a collision reaction with a registered partner (2.4.2);
//             survivors are appended to the next event's colour bins;
//   k_end     one workgroup: clears the reacted flags, advances the event.
// Same-colour voxels are >= 3 hops apart, so the molecules of one stage touch
// disjoint closed neighbourhoods: a stage needs no locks or atomics on the
// lattice, and its result does not depend on the order of its molecules.
//
// The device path is integer only: every probability arrives as a 32-bit
// threshold fixed on the host.
#include "psc_device.h"

namespace psc {

// =============================================================================
// initial first-order candidate scan (before the first event after a load)
// =============================================================================
__global__ void __launch_bounds__(kStageThreads) k_scan_candidates(const LatDev *__restrict__ Lp) {
  const LatDev &L = *Lp;
  const uint64_t e = *L.ev;
  if (L.n_fo == 0 || e >= L.tape_horizon) return;
  const uint32_t cmax = L.tape_cmax[e];
  if (cmax == 0) return;
  const Bins &in = L.bins[e & 1];
  const uint32_t cb = (uint32_t)(e & 1);
  for (uint32_t c = 0; c < L.ncol; ++c) {
    const uint32_t n = min(in.count[c], (uint32_t)L.cap);
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
      const uint32_t id = in.id[c * L.cap + i];
      if (id == kDeadId) continue;
      const U4 r = philox((uint32_t)e, id, kPhaseFirst, 0, L.key0, L.key1);
      if (r.x < cmax) {
        const uint32_t slot = atomicAdd(&L.cand_count[cb], 1u);
        if (slot < L.cand_cap) {
          L.cand_pos[cb][slot] = (uint32_t)i;
          L.cand_id[cb][slot] = id;
          L.cand_col[cb][slot] = (uint8_t)c;
        } else {
          set_error(L, kErrCandOverflow);
        }
      }
    }
  }
}

// =============================================================================
// k_begin: stage order, first-order pass, newborn ids
// =============================================================================
constexpr uint32_t kSortLds = 2048;  // newborn keys ranked in LDS up to this count
// fire lists up to this long test overlaps voxel by voxel in LDS
constexpr uint32_t kFewFirings = 8;

__device__ __forceinline__ void bitonic_sort_keys(uint64_t *keys, uint32_t n2, int tid, int nthreads) {
  for (uint32_t k = 2; k <= n2; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t q = tid; q < n2; q += nthreads) {
        const uint32_t p = q ^ j;
        if (p > q) {
          const uint64_t a = keys[q], b = keys[p];
          const bool up = (q & k) == 0;
          if ((a > b) == up) {
            keys[q] = b;
            keys[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// For each of the nb distinct keys in LDS, f(true, key, rank) with rank =
// the number of smaller keys.  Each thread holds up to PER keys (PER *
// nthreads >= nb) and reads the list once.  Every thread of the workgroup
// calls f PER times (f(false, ...) past the end), so f may reserve bin
// space for the whole workgroup at once.
template <int PER, class F>
__device__ __forceinline__ void for_each_ranked(const uint64_t *keys, uint32_t nb, uint32_t tid,
                                                uint32_t nthreads, F f) {
  uint64_t mine[PER];
  uint32_t rank[PER];
#pragma unroll
  for (int a = 0; a < PER; ++a) {
    const uint32_t q = tid + a * nthreads;
    mine[a] = q < nb ? keys[q] : ~0ull;
    rank[a] = 0;
  }
  // eight LDS reads in flight per step
#pragma unroll 8
  for (uint32_t j = 0; j < nb; ++j) {
    const uint64_t k = keys[j];
#pragma unroll
    for (int a = 0; a < PER; ++a) rank[a] += k < mine[a] ? 1u : 0u;
  }
#pragma unroll
  for (int a = 0; a < PER; ++a) f(tid + a * nthreads < nb, mine[a], rank[a]);
}

// ---- workgroup-wide reservations in global counters.  Every thread of the
// workgroup calls these together, and each counter takes one atomic per
// workgroup: atomics from many workgroups on one cache line are serialised
// in L2 (about 10 ns each), so an event's tens of thousands of firings or
// newborns appended one atomic each would cost a few hundred microseconds
// per counter. ----
struct WgBins {
  uint32_t cnt[kMaxColours];
  uint32_t base[kMaxColours];
};

// a position in colour c's bin, counted in count[c], for each thread that
// wants one (the others get 0)
__device__ __forceinline__ uint32_t wg_reserve_bins(uint32_t *count, bool want, uint32_t c,
                                                    WgBins &s) {
  if (threadIdx.x < (uint32_t)kMaxColours) s.cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t local = want ? atomicAdd(&s.cnt[c], 1u) : 0u;
  __syncthreads();
  if (threadIdx.x < (uint32_t)kMaxColours && s.cnt[threadIdx.x])
    s.base[threadIdx.x] = atomicAdd(&count[threadIdx.x], s.cnt[threadIdx.x]);
  __syncthreads();
  return want ? s.base[c] + local : 0u;
}

struct WgSlots {
  uint32_t cnt, base;
};

// n consecutive slots of *counter for each thread (n may be 0)
__device__ __forceinline__ uint32_t wg_reserve(uint32_t *counter, uint32_t n, WgSlots &s) {
  if (threadIdx.x == 0) s.cnt = 0;
  __syncthreads();
  const uint32_t local = n ? atomicAdd(&s.cnt, n) : 0u;
  __syncthreads();
  if (threadIdx.x == 0 && s.cnt) s.base = atomicAdd(counter, s.cnt);
  __syncthreads();
  return n ? s.base + local : 0u;
}

// The first-order pass's statistics, tallied in LDS by its workgroup and
// added to the lattice's counters once at its end: thousands of firings in
// one workgroup would otherwise queue their 64-bit atomics on one line.
struct FirstOrderTally {
  int32_t dsp[64];                  // live molecules per species, change
  uint32_t fired[kMaxReactions];
  uint32_t fail;                    // placement failures
};

// One first-order firing of the molecule at (colour c, position pos): the
// first product stays in place, the others go to distinct vacant neighbours
// of its compartment chosen by the placement words; too few vacant
// neighbours: no change.  Planned first (reads only), then committed with
// the first of its newborns' slots, so that a workgroup can reserve the
// slots of all its firings at once in between: the firings of one stage
// touch disjoint closed neighbourhoods, so no firing's commit changes what
// another's plan read.
struct FoPlan {
  uint64_t at;          // bin entry
  uint32_t v, w0, rx, id, m;
  bool ok;              // false: a placement failure
  // stencil direction of the neighbour product a + 1 takes, 4 bits each (a
  // register word rather than an indexed array, which would live in scratch)
  uint64_t dirs;
};

// the number of newborns the firing will have (its slots to reserve); v:
// the molecule's voxel (its bin entry's, recorded in the fire list)
template <class Tab>
__device__ __forceinline__ uint32_t plan_first_order(const LatDev &L, const Tab &tab, uint64_t e,
                                                     uint32_t c, uint32_t pos, uint32_t id,
                                                     uint32_t rx, uint32_t v, FoPlan &p) {
  p.at = c * L.cap + pos;
  p.v = v;
  p.rx = rx;
  p.id = id;
  p.m = tab.nprod(rx);
  p.w0 = L.occ[p.v];
  p.ok = true;
  p.dirs = 0;
  if (p.m <= 1) return 0;
  const uint32_t comp = p.w0 & kCompBits;
  // vacant neighbours of the same compartment, as a mask in stencil order
  uint32_t vmask = 0;
  const Coord cv = coord_of(L.geo, p.v);
  for (uint32_t n = 0; n < 12; ++n) {
    Coord ct;
    if (!step_target(L.geo, cv, n, ct)) continue;  // beyond a wall
    if (L.occ[index_of(L.geo, ct)] == comp) vmask |= 1u << n;
  }
  if (__popc(vmask) < (int)(p.m - 1)) {
    p.ok = false;
    return 0;
  }
  // product a + 1 takes the x-th of the vacancies left, in stencil order
  const U4 r = philox((uint32_t)e, id, kPhaseFirst, 0, L.key0, L.key1);
  for (uint32_t a = 0; a + 1 < p.m; ++a) {
    uint32_t x = scale32(placement_word(L, e, id, r, (int)a), (uint32_t)__popc(vmask));
    uint32_t n = 0;
    for (;; ++n) {
      if (!((vmask >> n) & 1u)) continue;
      if (x == 0) break;
      --x;
    }
    vmask &= ~(1u << n);
    p.dirs |= (uint64_t)n << (4 * a);
  }
  return p.m - 1;
}

// b0: the first of the plan's newborn slots
template <class Tab>
__device__ __forceinline__ void commit_first_order(const LatDev &L, const Tab &tab, const Bins &in,
                                                   const FoPlan &p, uint32_t b0,
                                                   FirstOrderTally *T) {
  const uint32_t sp0 = p.w0 & kSpeciesBits;
  const uint32_t comp = p.w0 & kCompBits;  // every product stays in this compartment
  if (!p.ok) {
    atomicAdd(&T->fail, 1u);
    return;
  }
  atomicAdd(&T->fired[p.rx], 1u);
  atomicSub(&T->dsp[sp0], 1);
  if (p.m == 0) {
    L.occ[p.v] = (uint16_t)comp;
    in.id[p.at] = kDeadId;
    return;
  }
  const uint32_t prod0 = tab.prod(p.rx, 0);
  L.occ[p.v] = (uint16_t)(prod0 | comp);
  in.sp[p.at] = (uint16_t)(prod0 | comp);  // the entry stays; its cached word follows
  atomicAdd(&T->dsp[prod0 & 63u], 1);
  const Coord cv = coord_of(L.geo, p.v);
  for (uint32_t a = 0; a + 1 < p.m; ++a) {
    Coord ct;
    step_target(L.geo, cv, (uint32_t)(p.dirs >> (4 * a)) & 15u, ct);
    const uint32_t dest = index_of(L.geo, ct);
    const uint32_t pa = tab.prod(p.rx, a + 1);
    L.occ[dest] = (uint16_t)(pa | comp);
    atomicAdd(&T->dsp[pa & 63u], 1);
    const uint32_t b = b0 + a;
    if (b < L.birth_cap) {
      L.birth_key[b] = ((uint64_t)p.id << 31) | ((uint64_t)(a + 1) << 27) | b;
      L.birth_vox[b] = dest;
      L.birth_sp[b] = (uint16_t)(pa | comp);
    } else {
      atomicOr(L.error, kErrBirthOverflow);
    }
  }
}

// plan and commit at once, newborn slots from *s_nb (LDS: one workgroup)
__device__ __forceinline__ void apply_first_order(const LatDev &L, uint64_t e, const Bins &in,
                                                  uint32_t c, uint32_t pos, uint32_t id,
                                                  uint32_t rx, uint32_t v, uint32_t *s_nb,
                                                  FirstOrderTally *T) {
  const RxTabGlobal tab{L};
  FoPlan p;
  const uint32_t nb = plan_first_order(L, tab, e, c, pos, id, rx, v, p);
  commit_first_order(L, tab, in, p, nb ? atomicAdd(s_nb, nb) : 0u, T);
}

// First-order newborns (key = parent id << 31 | product index << 27 | slot)
// join the bins of the running event with their voxel's word (newborns of
// the first-order pass walk in the same event): thread with `valid` bins the
// newborn of key `key` with id `id`.  Called by the whole workgroup.
__device__ __forceinline__ void bin_first_order_births(const LatDev &L, const Bins &in, bool valid,
                                                       uint64_t key, uint32_t id, WgBins &wb) {
  const uint32_t src = (uint32_t)(key & ((1u << 27) - 1u));
  const uint32_t v = valid ? L.birth_vox[src] : 0u;
  const uint32_t c = valid ? colour_of_voxel(L.geo, v) : 0u;
  const uint32_t pos = wg_reserve_bins(in.count, valid, c, wb);
  if (!valid) return;
  if (pos < L.cap) {
    const uint64_t at = c * L.cap + pos;
    in.vox[at] = v;
    in.id[at] = id;
    in.sp[at] = L.birth_sp[src];
    if (in.disp) {
      in.disp[(0 * L.ncol + c) * L.cap + pos] = 0;
      in.disp[(1 * L.ncol + c) * L.cap + pos] = 0;
      in.disp[(2 * L.ncol + c) * L.cap + pos] = 0;
    }
  } else {
    set_error(L, kErrBinOverflow);
  }
}

// The last of the grid's workgroups to call this returns true (counted in
// *done, which it resets); after a device-scope fence it sees the others'
// atomics.
__device__ __forceinline__ bool last_workgroup(uint32_t *done) {
  __shared__ uint32_t s_last;
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(done, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  if (threadIdx.x == 0) *done = 0;
  return true;
}

// ---- ranking of many distinct keys over the grid.  A key's owner id (key
// >> shift) deals it into one of nbk buckets that split [0, id_end) into
// equal ranges, so the buckets follow the key order, and a key's rank (the
// number of smaller keys) is its bucket's offset plus the number of smaller
// keys in its bucket.  Owner ids spread over the range, and nbk is the power
// of two at least nb / 4 (at most kRankBucketsMax): a few keys per bucket.
// Three launches: k_rank_count (whose last workgroup turns the counts into
// offsets), k_rank_deal, then the numbering kernel, which ranks with
// rank_dealt.  List 0: the first-order newborns left to the grid; list 1:
// the collision newborns left by the event end. ----
struct RankList {
  const uint64_t *keys;
  uint32_t nb, shift, id_end, nbk;
};

__device__ __forceinline__ RankList make_rank_list(const uint64_t *keys, uint32_t nb,
                                                   uint32_t shift, uint32_t id_end) {
  RankList R{keys, nb, shift, max(id_end, 1u), 1u};
  while (R.nbk * 4u < nb && R.nbk < kRankBucketsMax) R.nbk <<= 1;
  return R;
}

template <int LIST>
__device__ __forceinline__ RankList rank_list(const LatDev &L) {
  if (LIST == 0)
    return make_rank_list(L.birth_key, min(*L.birth_count, (uint32_t)L.birth_cap), 31, *L.next_id);
  return make_rank_list(L.wb_key, min(*L.wb_count, (uint32_t)L.wb_cap), 32, *L.next_id);
}

__device__ __forceinline__ uint32_t rank_bucket(const RankList &R, uint64_t key) {
  const uint64_t id = key >> R.shift;  // < id_end: owners exist before the numbering
  return (uint32_t)min(id * R.nbk / R.id_end, (uint64_t)(R.nbk - 1u));
}

template <int LIST>
__global__ void __launch_bounds__(kStageThreads) k_rank_count(const LatDev *__restrict__ Lp) {
  __shared__ uint32_t s_sum[kStageThreads];
  __shared__ uint32_t s_hist[kRankBucketsMax];
  const LatDev &L = *Lp;
  const RankList R = rank_list<LIST>(L);
  if (R.nb == 0 || (LIST == 1 && R.nb <= kSortLds)) return;  // nothing left to the grid
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < R.nb; q += gridDim.x * blockDim.x)
    atomicAdd(&L.rank_hist[rank_bucket(R, R.keys[q])], 1u);
  if (!last_workgroup(L.end_done)) return;
  // the last workgroup: exclusive prefix sums of the counts.  They are read
  // through L2 (other workgroups' atomics), a coalesced row per pass, into
  // LDS; each thread then sums a run of per buckets.
  const uint32_t tid = threadIdx.x;
  for (uint32_t b = tid; b < R.nbk; b += blockDim.x)
    s_hist[b] = __hip_atomic_load(&L.rank_hist[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const uint32_t per = (R.nbk + blockDim.x - 1) / blockDim.x;
  const uint32_t b0 = min(tid * per, R.nbk), b1 = min(b0 + per, R.nbk);
  uint32_t sum = 0;
  for (uint32_t b = b0; b < b1; ++b) sum += s_hist[b];
  s_sum[tid] = sum;
  __syncthreads();
  for (uint32_t d = 1; d < blockDim.x; d <<= 1) {
    const uint32_t add = tid >= d ? s_sum[tid - d] : 0u;
    __syncthreads();
    s_sum[tid] += add;
    __syncthreads();
  }
  uint32_t run = s_sum[tid] - sum;
  for (uint32_t b = b0; b < b1; ++b) {
    const uint32_t n = s_hist[b];
    s_hist[b] = run;
    run += n;
  }
  __syncthreads();
  for (uint32_t b = tid; b < R.nbk; b += blockDim.x) L.rank_off[b] = s_hist[b];
  if (tid == 0) L.rank_off[R.nbk] = R.nb;
}

// deals the keys into bucket order; the counts return to zero
template <int LIST>
__global__ void __launch_bounds__(kStageThreads) k_rank_deal(const LatDev *__restrict__ Lp) {
  const LatDev &L = *Lp;
  const RankList R = rank_list<LIST>(L);
  if (R.nb == 0 || (LIST == 1 && R.nb <= kSortLds)) return;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < R.nb; q += gridDim.x * blockDim.x) {
    const uint64_t key = R.keys[q];
    const uint32_t b = rank_bucket(R, key);
    const uint32_t k = atomicSub(&L.rank_hist[b], 1u) - 1u;
    L.rank_keys[L.rank_off[b] + k] = key;
  }
}

// f(true, key, rank) for every dealt key; every thread of a workgroup calls
// f once per pass (f(false, ...) past the end)
template <class F>
__device__ __forceinline__ void rank_dealt(const LatDev &L, const RankList &R, F f) {
  for (uint32_t base = blockIdx.x * blockDim.x; base < R.nb; base += gridDim.x * blockDim.x) {
    const uint32_t p = base + threadIdx.x;
    const bool valid = p < R.nb;
    uint64_t key = 0;
    uint32_t rank = 0;
    if (valid) {
      key = L.rank_keys[p];
      const uint32_t b = rank_bucket(R, key);
      const uint32_t lo = L.rank_off[b], hi = L.rank_off[b + 1];
      rank = lo;
      for (uint32_t j = lo; j < hi; ++j) rank += L.rank_keys[j] < key ? 1u : 0u;
    }
    f(valid, key, rank);
  }
}

// The first-order reaction that the candidate at (colour c, position pos)
// with id `id` fires in event e, or -1: a candidate whose voxel holds a
// species with first-order reactions fires the reaction whose cumulative
// threshold its draw falls under.  Independent of order (a candidate's
// species cannot change before its own turn), so any number of threads and
// workgroups may share the decisions of an event.
// (v: the candidate's voxel)
template <class FoTab>
__device__ __forceinline__ int first_order_decision(const LatDev &L, const FoTab &ft, uint64_t e,
                                                    const Bins &in, uint32_t c, uint32_t pos,
                                                    uint32_t id, uint32_t &v) {
  v = in.vox[c * L.cap + pos];
  const uint32_t sp = L.occ[v] & kSpeciesBits;
  if (!(ft.flags(sp) & kSpFirstOrder)) return -1;
  const U4 r = philox((uint32_t)e, id, kPhaseFirst, 0, L.key0, L.key1);
  return first_order_choice(ft, sp, r.x);
}

// the decisions of event e for candidates [first, ...) with the given
// stride, by one workgroup: the fire list is counted in *nfire (LDS)
template <class FoTab>
__device__ __forceinline__ void decide_first_order(const LatDev &L, const FoTab &ft, uint64_t e,
                                                   uint32_t first, uint32_t stride,
                                                   uint32_t *nfire) {
  const uint32_t buf = (uint32_t)(e & 1);
  const Bins &in = L.bins[buf];
  const uint32_t ncand = L.n_fo ? min(L.cand_count[buf], (uint32_t)L.cand_cap) : 0u;
  for (uint32_t q = first; q < ncand; q += stride) {
    const uint32_t c = L.cand_col[buf][q], pos = L.cand_pos[buf][q], id = L.cand_id[buf][q];
    uint32_t v;
    const int rx = first_order_decision(L, ft, e, in, c, pos, id, v);
    if (rx < 0) continue;
    const uint32_t slot = atomicAdd(nfire, 1u);
    L.fire_pos[slot] = pos;
    L.fire_vox[slot] = v;
    L.fire_id[slot] = id;
    L.fire_col[slot] = (uint8_t)c;
    L.fire_rx[slot] = (uint8_t)rx;
  }
}

// the event's opening work for one lattice, by one workgroup; decided: the
// fire list was built by k_decide
// defer: newborns beyond what one workgroup numbers in LDS are left to
// k_births (their count in *birth_count), which then writes the stage
// descriptors; *deferred tells the caller
// apply: k_fo_stage launches, one per stage, and k_births follow; more
// firings than this workgroup has threads are left to them (this pass then
// ends after the decisions), fewer are applied here as without them
// NT: the workgroup's threads
template <int NT = kBeginThreads>
__device__ __forceinline__ void begin_work(const LatDev &L, bool decided, bool defer, bool apply,
                                           uint32_t *deferred, FirstOrderTally *T) {
  uint32_t *__restrict__ fire_pos = L.fire_pos;
  uint32_t *__restrict__ fire_id = L.fire_id;
  uint8_t *__restrict__ fire_col = L.fire_col;
  uint8_t *__restrict__ fire_rx = L.fire_rx;
  __shared__ uint32_t s_perm[kMaxColours], s_colcnt[kMaxColours];
  __shared__ uint32_t s_nfire, s_nb, s_next;
  __shared__ uint64_t s_keys[kSortLds];
  __shared__ FoTabLds s_fo;
  const uint64_t e = *L.ev;
  const int tid = threadIdx.x;
  if (e >= L.stop_event) return;  // an idle member of an ensemble
  if (e >= L.tape_horizon) {
    if (tid == 0) set_error(L, kErrTape);
    return;
  }
  if (!decided && L.n_fo) s_fo.fill(L, e);  // published by the barrier below
  const uint32_t buf = (uint32_t)(e & 1);
  const Bins &in = L.bins[buf];
  const Bins &out = L.bins[buf ^ 1];
  if (tid == 0) {
    stage_order(L, e, s_perm);
    s_nfire = 0;
    s_nb = 0;
    s_next = *L.next_id;
  }
  const uint32_t ncol = L.ncol;
  if (tid < kMaxColours) {
    out.count[tid] = 0;
    s_colcnt[tid] = 0;
  }
  if (tid == 32) L.cand_count[buf ^ 1] = 0;
  __syncthreads();
  if (tid < (int)ncol) L.perm[tid] = s_perm[tid];

  // ---- first-order decisions ----
  if (!decided)
    decide_first_order(L, s_fo, e, tid, blockDim.x, &s_nfire);
  else if (tid == 0)
    s_nfire = min(__hip_atomic_load(L.fire_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                  (uint32_t)L.cap);
  __syncthreads();
  const uint32_t nfire = s_nfire;
  if (tid == 0) L.recent[kRecentFire] = nfire;
  if (apply && nfire > blockDim.x) {
    if (tid == 0) {
      if (!decided) *L.fire_count = nfire;  // the list the stage launches apply
      *deferred = 1;
    }
    return;
  }
  // a short list is applied here whatever the launch shape: the stage
  // launches then find it empty
  if (apply && decided && tid == 0) *L.fire_count = 0;

  // ---- application.  A firing molecule reads and writes only its closed
  // neighbourhood N[v] (its voxel and the 12 neighbours).  Molecules whose
  // N[v] meets no other firing molecule's commute with everything and are
  // applied at once; the others (rare) are applied stage by stage in the
  // event's order.  A few firings compare their neighbourhoods voxel by
  // voxel in LDS; more are tested by counting, per hashed voxel, the
  // neighbourhoods that contain it (a hash collision only sends a molecule
  // to the staged path, which is always correct). ----
  __shared__ uint32_t s_nbv[kFewFirings][13];
  if (nfire > 0 && nfire <= kFewFirings) {
    const bool mine = (uint32_t)tid < nfire;
    uint32_t c = 0, pos = 0, id = 0, rx = 0, v = 0;
    if (mine) {
      c = fire_col[tid];
      pos = fire_pos[tid];
      id = fire_id[tid];
      rx = fire_rx[tid];
      v = L.fire_vox[tid];
      const Coord cv = coord_of(L.geo, v);
      s_nbv[tid][0] = v;
#pragma unroll
      for (uint32_t n = 0; n < 12; ++n) s_nbv[tid][n + 1] = index_of(L.geo, step_coord(L.geo, cv, n));
    }
    __syncthreads();
    bool overlap = false;
    if (mine)
      for (uint32_t j = 0; j < nfire && !overlap; ++j) {
        if (j == (uint32_t)tid) continue;
        for (int a = 0; a < 13 && !overlap; ++a)
          for (int b = 0; b < 13; ++b) overlap |= s_nbv[tid][a] == s_nbv[j][b];
      }
    if (mine && !overlap) apply_first_order(L, e, in, c, pos, id, rx, v, &s_nb, T);
    if (mine && overlap) atomicAdd(&s_colcnt[c], 1u);
    __syncthreads();
    for (uint32_t g = 0; g < ncol; ++g) {
      const uint32_t cg = s_perm[g];
      if (s_colcnt[cg] == 0) continue;
      if (mine && overlap && c == cg) apply_first_order(L, e, in, c, pos, id, rx, v, &s_nb, T);
      __syncthreads();
    }
  } else if (nfire > 0 && nfire <= blockDim.x) {
    // one firing per thread: its colour, position, draw owner, reaction and
    // the 13 hashed voxels of its neighbourhood stay in registers through
    // the count, the test, the application and the cleanup
    const uint32_t nb_bits = L.nbr_bits;
    const bool mine = (uint32_t)tid < nfire;
    uint32_t c = 0, pos = 0, id = 0, rx = 0, v = 0, h[13];
    bool deferred = false;
    if (mine) {
      c = fire_col[tid];
      pos = fire_pos[tid];
      id = fire_id[tid];
      rx = fire_rx[tid];
      v = L.fire_vox[tid];
      const Coord cv = coord_of(L.geo, v);
      h[0] = hot_hash(v, nb_bits);
#pragma unroll
      for (uint32_t n = 0; n < 12; ++n)
        h[n + 1] = hot_hash(index_of(L.geo, step_coord(L.geo, cv, n)), nb_bits);
#pragma unroll
      for (int a = 0; a < 13; ++a) atomicAdd(&L.nbr_cnt[h[a]], 1u);
    }
    __syncthreads();
    if (mine) {
      uint32_t other = 0;
#pragma unroll
      for (int a = 0; a < 13; ++a)
        other |= __hip_atomic_load(&L.nbr_cnt[h[a]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ^ 1u;
      if (other == 0u) {
        apply_first_order(L, e, in, c, pos, id, rx, v, &s_nb, T);
      } else {
        deferred = true;  // to the staged pass
        atomicAdd(&s_colcnt[c], 1u);
      }
    }
    __syncthreads();
    for (uint32_t g = 0; g < ncol; ++g) {
      const uint32_t cg = s_perm[g];
      if (s_colcnt[cg] == 0) continue;
      if (deferred && c == cg) apply_first_order(L, e, in, c, pos, id, rx, v, &s_nb, T);
      __syncthreads();
    }
    // leave the counts at zero for the next event
    if (mine) {
#pragma unroll
      for (int a = 0; a < 13; ++a) atomicSub(&L.nbr_cnt[h[a]], 1u);
    }
    __syncthreads();
  } else if (nfire > 0) {
    // more firings than threads: every firing is applied in the event's
    // stage order, all those of one colour at once (their closed
    // neighbourhoods are disjoint, so they commute).  Counting overlaps as
    // above would cost 39 global atomics per firing, all issued from this
    // one workgroup's compute unit.
    for (uint32_t g = 0; g < ncol; ++g) {
      const uint32_t cg = s_perm[g];
      for (uint32_t q = tid; q < nfire; q += blockDim.x)
        if (fire_col[q] == cg)
          apply_first_order(L, e, in, cg, fire_pos[q], fire_id[q], fire_rx[q], L.fire_vox[q],
                            &s_nb, T);
      __syncthreads();
    }
  }

  // ---- newborn ids: ascending parent id, then product index.  The keys are
  // distinct (they end in the birth's slot), so a newborn's id is next_id
  // plus the number of smaller keys: counted in LDS up to kSortLds newborns,
  // else read off a bitonic sort in global memory ----
  const uint32_t nb = min(s_nb, (uint32_t)L.birth_cap);
  if (tid == 0) L.recent[kRecentFoBirths] = nb;
  if (nb == 0) return;
  const uint32_t base_id = s_next;
  if ((uint64_t)base_id + nb >= 0xFFFFFFFFull) {
    if (tid == 0) set_error(L, kErrIds);
    return;
  }
  __shared__ WgBins s_wb;
  auto bin_birth = [&](bool valid, uint64_t key, uint32_t id) {
    bin_first_order_births(L, in, valid, key, id, s_wb);
  };
  if (nb > kSortLds && defer) {
    if (tid == 0) {
      *L.birth_count = nb;  // k_births numbers them and writes the stage descriptors
      *deferred = 1;
    }
    return;
  }
  if (nb <= kSortLds) {
    for (uint32_t q = tid; q < nb; q += blockDim.x) s_keys[q] = L.birth_key[q];
    __syncthreads();
    for_each_ranked<kSortLds / NT>(
        s_keys, nb, tid, NT,
        [&](bool valid, uint64_t k, uint32_t r) { bin_birth(valid, k, base_id + r); });
  } else {
    uint32_t n2 = 1;
    while (n2 < nb) n2 <<= 1;
    for (uint32_t q = nb + tid; q < n2; q += blockDim.x) L.birth_key[q] = ~0ull;
    __syncthreads();
    bitonic_sort_keys(L.birth_key, n2, tid, blockDim.x);
    for (uint32_t q0 = 0; q0 < nb; q0 += blockDim.x) {
      const uint32_t q = q0 + tid;
      bin_birth(q < nb, q < nb ? L.birth_key[q] : 0ull, base_id + q);
    }
  }
  if (tid == 0) *L.next_id = base_id + nb;
}

// The first-order pass, then each stage's descriptor for the walk: its colour,
// its molecule count (final now: the walk appends only to the next event's
// bins) and the event, so that a stage launch starts with one load instead of
// a chain of three.  A lattice that does not run this event (idle or out of
// tape) gets empty stages, and so do the stages past its colour count.
// threads tid < kMaxColours of one workgroup: each stage's descriptor
__device__ __forceinline__ void write_stage_descriptors(const LatDev &L, uint32_t tid) {
  if (tid < kMaxColours) {
    const uint64_t e = *L.ev;
    const bool run = e < L.tape_horizon && e < L.stop_event && tid < L.ncol;
    const uint32_t c = run ? L.perm[tid] : 0u;
    // births were counted with atomics by other threads: read through L2
    const uint32_t n = run ? min(atomicOr(&L.bins[e & 1].count[c], 0u), (uint32_t)L.cap) : 0u;
    L.sdesc[tid] = make_uint4(c, n, (uint32_t)e, (uint32_t)(e >> 32));
  }
}

// desc: write the stage descriptors (for stage launches that read them);
// NT: the workgroup's threads
template <int NT = kBeginThreads>
__device__ __forceinline__ void begin_body(const LatDev &L, bool decided, bool defer, bool apply,
                                          bool desc = true) {
  __shared__ uint32_t s_deferred;
  __shared__ FirstOrderTally T;
  const uint32_t tid = threadIdx.x;
  if (tid == 0) {
    s_deferred = 0;
    T.fail = 0;
  }
  if (tid < 64) T.dsp[tid] = 0;
  if (tid < (uint32_t)kMaxReactions) T.fired[tid] = 0;
  __syncthreads();
  begin_work<NT>(L, decided, defer, apply, &s_deferred, &T);
  __syncthreads();  // every return of begin_work is taken by the whole block
  if (tid < 64 && T.dsp[tid]) atomicAdd(&stat_sp(L)[tid], (unsigned long long)(long long)T.dsp[tid]);
  if (tid < L.n_rx && T.fired[tid]) atomicAdd(&stat_fired(L)[tid], (unsigned long long)T.fired[tid]);
  if (tid == 0 && T.fail) atomicAdd(&stat_cnt(L)[3], (unsigned long long)T.fail);
  if (s_deferred) return;  // k_births finishes the pass
  if (tid == 0 && decided) *L.fire_count = 0;  // k_decide's list has been applied
  if (desc) write_stage_descriptors(L, tid);
}

// defer: k_births follows (newborns beyond the LDS ranking are left to it);
// apply: k_fo_stage launches apply the firings, then k_births
__global__ void __launch_bounds__(kBeginThreads) k_begin(const LatDev *__restrict__ Lp,
                                                         int decided, int defer, int apply,
                                                         int desc) {
  begin_body(*Lp, decided != 0, defer != 0, apply != 0, desc != 0);
}

// one workgroup per member lattice of an ensemble.  Half of k_begin's
// threads: a member's lists are short, and three such workgroups fit on a
// compute unit where one of k_begin's does, so that all members of a
// 512-member ensemble open their event at once.
constexpr int kBeginMultiThreads = 512;
__global__ void __launch_bounds__(kBeginMultiThreads) k_begin_multi(const LatDev *__restrict__ lats) {
  begin_body<kBeginMultiThreads>(lats[blockIdx.x], false, false, false);
}

// Stage g of the first-order application over many workgroups (events with
// many firings): every firing of the stage's colour cg, at once -- their
// closed neighbourhoods are disjoint.  A workgroup takes kFoTile entries of
// the fire list per pass and gathers those of the stage's colour in LDS, so
// its lanes work on firings, not on skipped entries; newborns take slots
// from *birth_count, one reservation per workgroup and pass.  The first
// tile's colours and the reaction tables are read alongside the list's
// length (lanes past it are dropped once it arrives).
__device__ __forceinline__ void fo_stage_body(const LatDev &L, uint64_t e, uint32_t cg) {
  constexpr int PER = kFoTile / kStageThreads;
  __shared__ FirstOrderTally T;
  __shared__ uint32_t s_idx[kFoTile];
  __shared__ uint32_t s_n;
  __shared__ WgSlots s_slots;
  __shared__ uint32_t s_tab[kStageTabWordsMax];
  const uint32_t tid = threadIdx.x;
  const Bins &in = L.bins[e & 1];
  const uint64_t cap = L.cap;
  const uint32_t nraw = *L.fire_count;
  const uint32_t t0 = blockIdx.x * kFoTile;
  uint32_t col0[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k)
    col0[k] = L.fire_col[min((uint64_t)t0 + k * kStageThreads + tid, cap - 1)];
  const uint32_t tw = L.stage_tab_words;
  uint32_t tw0 = 0, tw1 = 0;
  if (tid < tw) tw0 = L.stage_tab[tid];
  if (tid + kStageThreads < tw) tw1 = L.stage_tab[tid + kStageThreads];
  if (tid == 0) T.fail = 0;
  if (tid < 64) T.dsp[tid] = 0;
  for (uint32_t r = tid; r < (uint32_t)kMaxReactions; r += blockDim.x) T.fired[r] = 0;
  if (tid < tw) s_tab[tid] = tw0;
  if (tid + kStageThreads < tw) s_tab[tid + kStageThreads] = tw1;
  for (uint32_t i = tid + 2 * kStageThreads; i < tw; i += kStageThreads) s_tab[i] = L.stage_tab[i];
  const uint32_t nfire = (uint32_t)min((uint64_t)nraw, cap);
  __syncthreads();
  const RxTabLds tab{s_tab, stage_tab_layout(L.n_species, L.n_rx)};
  for (uint32_t t = t0; t < nfire; t += gridDim.x * kFoTile) {
    const uint32_t t1 = min(t + kFoTile, nfire);
    if (tid == 0) s_n = 0;
    __syncthreads();
    if (t == t0) {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const uint32_t q = t + k * kStageThreads + tid;
        if (q < t1 && col0[k] == cg) s_idx[atomicAdd(&s_n, 1u)] = q;
      }
    } else {
      for (uint32_t q = t + tid; q < t1; q += blockDim.x)
        if (L.fire_col[q] == cg) s_idx[atomicAdd(&s_n, 1u)] = q;
    }
    __syncthreads();
    const uint32_t n = s_n;
    for (uint32_t k0 = 0; k0 < n; k0 += blockDim.x) {
      const uint32_t k = k0 + tid;
      FoPlan p;
      uint32_t nb = 0;
      if (k < n) {
        const uint32_t q = s_idx[k];
        nb = plan_first_order(L, tab, e, cg, L.fire_pos[q], L.fire_id[q], L.fire_rx[q],
                              L.fire_vox[q], p);
      }
      const uint32_t b0 = wg_reserve(L.birth_count, nb, s_slots);
      if (k < n) commit_first_order(L, tab, in, p, b0, &T);
    }
    __syncthreads();  // s_idx and s_n serve the next pass
  }
  if (tid < 64 && T.dsp[tid]) atomicAdd(&stat_sp(L)[tid], (unsigned long long)(long long)T.dsp[tid]);
  for (uint32_t r = tid; r < L.n_rx; r += blockDim.x)
    if (T.fired[r]) atomicAdd(&stat_fired(L)[r], (unsigned long long)T.fired[r]);
  if (tid == 0 && T.fail) atomicAdd(&stat_cnt(L)[3], (unsigned long long)T.fail);
}

// the stage's colour from the event's stage order on the device
__global__ void __launch_bounds__(kStageThreads) k_fo_stage(const LatDev *__restrict__ Lp,
                                                            uint32_t g) {
  const LatDev &L = *Lp;
  const uint64_t e = *L.ev;
  if (e >= L.stop_event || e >= L.tape_horizon) return;
  fo_stage_body(L, e, L.perm[g]);
}

// the record, the stage's colour and the event from the host (a lattice
// stepped one event at a time from the host, within its tape)
__global__ void __launch_bounds__(kStageThreads) k_fo_stage_direct(const LatDev L, uint32_t cg,
                                                                   uint64_t e) {
  fo_stage_body(L, e, cg);
}

// The first-order newborns left to it (more than k_begin ranks in LDS, or
// all of them after k_fo_stage applied the firings): ids next_id + rank over
// the whole grid, binned for the running event; the last workgroup advances
// next_id, clears the fire list and writes the stage descriptors.  finish:
// the pass was handed over whatever the newborns (after k_fo_stage).
__global__ void __launch_bounds__(kStageThreads) k_births(const LatDev *__restrict__ Lp,
                                                          int finish) {
  const LatDev &L = *Lp;
  RankList R = rank_list<0>(L);
  if (R.nb == 0 && !finish) return;  // k_begin numbered this event's newborns (or had none)
  const uint64_t e = *L.ev;
  const Bins &in = L.bins[e & 1];
  const uint32_t base_id = *L.next_id;
  if ((uint64_t)base_id + R.nb >= 0xFFFFFFFFull) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_error(L, kErrIds);
    R.nb = 0;
  }
  const uint32_t nb = R.nb;
  if (blockIdx.x == 0 && threadIdx.x == 0) L.recent[kRecentFoBirths] = nb;
  __shared__ WgBins s_wb;
  if (nb)
    rank_dealt(L, R, [&](bool valid, uint64_t k, uint32_t r) {
      bin_first_order_births(L, in, valid, k, base_id + r, s_wb);
    });
  if (!last_workgroup(L.end_done)) return;
  if (threadIdx.x == 0) {
    *L.next_id = base_id + nb;
    *L.birth_count = 0;
    *L.fire_count = 0;  // the fire list has been applied
  }
  write_stage_descriptors(L, threadIdx.x);
}

// the first-order decisions of the coming event over many workgroups, for
// events with many candidates (k_begin then only applies the fire list)
// (the fire list grows by one reservation per workgroup and pass)
__global__ void __launch_bounds__(kStageThreads) k_decide(const LatDev *__restrict__ Lp) {
  __shared__ WgSlots s_slots;
  __shared__ FoTabLds s_fo;
  const LatDev &L = *Lp;
  const uint64_t e = *L.ev;
  if (e >= L.stop_event || e >= L.tape_horizon) return;
  s_fo.fill(L, e);
  __syncthreads();
  const uint32_t buf = (uint32_t)(e & 1);
  const Bins &in = L.bins[buf];
  const uint32_t ncand = L.n_fo ? min(L.cand_count[buf], (uint32_t)L.cand_cap) : 0u;
  for (uint32_t base = blockIdx.x * blockDim.x; base < ncand; base += gridDim.x * blockDim.x) {
    const uint32_t q = base + threadIdx.x;
    uint32_t c = 0, pos = 0, id = 0, v = 0;
    int rx = -1;
    if (q < ncand) {
      c = L.cand_col[buf][q];
      pos = L.cand_pos[buf][q];
      id = L.cand_id[buf][q];
      rx = first_order_decision(L, s_fo, e, in, c, pos, id, v);
    }
    const uint32_t slot = wg_reserve(L.fire_count, rx >= 0 ? 1u : 0u, s_slots);
    if (rx >= 0 && slot < L.cap) {
      L.fire_pos[slot] = pos;
      L.fire_vox[slot] = v;
      L.fire_id[slot] = id;
      L.fire_col[slot] = (uint8_t)c;
      L.fire_rx[slot] = (uint8_t)rx;
    }
  }
}

// =============================================================================
// k_end: clear reacted flags and the previous event's hot bitmap, advance the
// event counter (the last workgroup to finish does the bookkeeping)
// =============================================================================
constexpr int kEndThreads = kStageThreads;
constexpr int kEndBlocks = 32;
// one workgroup per member of an ensemble: a member's lists are short, and
// one workgroup needs no completion count
constexpr int kEndBlocksMulti = 1;

// workgroup bid of nblk: sweep flags and the previous hot bitmap; the last
// workgroup to finish advances the lattice's event counter
// Newborns of this walk's many-product collisions get ids next_id, ... in
// ascending (mover id, product index) order and join the next event's bins
// with their current species (one may have changed as a later partner);
// they are also tested as first-order candidates of the next event, which a
// walk does for every other molecule.  Run by one whole workgroup.
// a newborn of event e's many-product collisions (key = mover id << 32 |
// product index << 28 | slot) with id `id` joins the next event's bins and
// is tested as a first-order candidate of that event
// (called by the whole workgroup; threads without `valid` only help with
// the reservations)
struct WgBirthBins {
  WgBins bins;
  WgSlots cand;
};
__device__ __forceinline__ void bin_collision_birth(const LatDev &L, uint64_t e, const Bins &out,
                                                    uint32_t cnext, uint32_t cmax_next,
                                                    bool valid, uint64_t key, uint32_t id,
                                                    WgBirthBins &wb) {
  const uint32_t u = valid ? L.wb_vox[key & ((1u << 28) - 1u)] : 0u;
  const uint32_t c = valid ? colour_of_voxel(L.geo, u) : 0u;
  const uint32_t pos = wg_reserve_bins(out.count, valid, c, wb.bins);
  const bool binned = valid && pos < L.cap;
  if (valid && !binned) set_error(L, kErrBinOverflow);
  if (binned) {
    const uint64_t at = c * L.cap + pos;
    out.vox[at] = u;
    out.id[at] = id;
    out.sp[at] = (uint16_t)(L.occ[u] & kWordMask);
    if (out.disp) {
      out.disp[(0 * L.ncol + c) * L.cap + pos] = 0;
      out.disp[(1 * L.ncol + c) * L.cap + pos] = 0;
      out.disp[(2 * L.ncol + c) * L.cap + pos] = 0;
    }
  }
  if (!cmax_next) return;  // uniform: no first-order reactions next event
  bool cand = false;
  if (binned) {
    const U4 r = philox((uint32_t)(e + 1), id, kPhaseFirst, 0, L.key0, L.key1);
    cand = r.x < cmax_next;
  }
  const uint32_t k = wg_reserve(&L.cand_count[cnext], cand ? 1u : 0u, wb.cand);
  if (!cand) return;
  if (k < L.cand_cap) {
    L.cand_pos[cnext][k] = pos;
    L.cand_id[cnext][k] = id;
    L.cand_col[cnext][k] = (uint8_t)c;
  } else {
    set_error(L, kErrCandOverflow);
  }
}

__device__ __forceinline__ void number_births(const LatDev &L, uint64_t e) {
  __shared__ uint64_t s_wkeys[kSortLds];
  const uint32_t tid = threadIdx.x;
  const uint32_t nb = min(*L.wb_count, (uint32_t)L.wb_cap);
  if (nb == 0) return;
  const uint32_t base_id = *L.next_id;
  if ((uint64_t)base_id + nb >= 0xFFFFFFFFull) {
    if (tid == 0) set_error(L, kErrIds);
    return;
  }
  const Bins &out = L.bins[(e + 1) & 1];
  const uint32_t cnext = (uint32_t)((e + 1) & 1);
  const uint32_t cmax_next = (L.n_fo && e + 1 < L.tape_horizon) ? L.tape_cmax[e + 1] : 0u;
  // the newborn of key `key` gets id `id` (keys are distinct: they end in the
  // slot; its id is next_id plus the number of smaller keys)
  __shared__ WgBirthBins s_wb;
  auto bin_newborn = [&](bool valid, uint64_t key, uint32_t id) {
    bin_collision_birth(L, e, out, cnext, cmax_next, valid, key, id, s_wb);
  };
  if (nb <= kSortLds) {
    for (uint32_t q = tid; q < nb; q += blockDim.x) s_wkeys[q] = L.wb_key[q];
    __syncthreads();
    for_each_ranked<kSortLds / kEndThreads>(
        s_wkeys, nb, tid, kEndThreads,
        [&](bool valid, uint64_t k, uint32_t r) { bin_newborn(valid, k, base_id + r); });
  } else {
    uint32_t n2 = 1;
    while (n2 < nb) n2 <<= 1;  // <= wb_cap, a power of two
    for (uint32_t q = nb + tid; q < n2; q += blockDim.x) L.wb_key[q] = ~0ull;
    __syncthreads();
    bitonic_sort_keys(L.wb_key, n2, tid, blockDim.x);
    for (uint32_t q0 = 0; q0 < nb; q0 += blockDim.x) {
      const uint32_t q = q0 + tid;
      bin_newborn(q < nb, q < nb ? L.wb_key[q] : 0ull, base_id + q);
    }
  }
  __syncthreads();
  if (tid == 0) {
    *L.next_id = base_id + nb;
    *L.wb_count = 0;
  }
}

// BIRTHS: the lattice may have newborns of many-product collisions to number
// (the numbering's registers and LDS would otherwise limit every end kernel)
// defer: newborns beyond what one workgroup ranks in LDS are left to
// k_end_births, which follows
// SB: list entries a thread sweeps at a time (more for fewer threads)
template <bool BIRTHS, int SB = 1>
__device__ __forceinline__ void end_body(const LatDev &L, uint32_t bid, uint32_t nblk,
                                         bool defer) {
  const uint64_t e = *L.ev;
  if (e >= L.tape_horizon || e >= L.stop_event) return;
  const uint32_t cur = (uint32_t)(e & 1), prv = cur ^ 1u;
  const uint32_t stride = nblk * blockDim.x;
  const uint32_t me = bid * blockDim.x + threadIdx.x;
  // this walk's partners may walk again from the next event on
  const uint32_t nf = min(L.flag_count[cur], (uint32_t)L.flag_cap);
  if (bid == 0 && threadIdx.x == 0) L.recent[kRecentFlags] = nf;
  // Both sweeps take SB entries per thread at a time, each step's loads
  // issued for all of them before the next step uses any, so that one
  // workgroup sweeps long lists with the loads overlapped.  A slot past the
  // list repeats entry q0 and stores nothing.  A voxel listed twice (a
  // product that reacted again as a partner) gets the same word from every
  // thread that clears it.
  constexpr int kSweepBatch = SB;
  const uint64_t step = (uint64_t)kSweepBatch * stride;
  for (uint64_t q0 = me; q0 < nf; q0 += step) {
    uint32_t v[kSweepBatch];
    uint16_t w[kSweepBatch];
#pragma unroll
    for (int b = 0; b < kSweepBatch; ++b) {
      const uint64_t q = q0 + (uint64_t)b * stride;
      v[b] = L.flag_vox[cur][q < nf ? q : q0];
    }
#pragma unroll
    for (int b = 0; b < kSweepBatch; ++b) w[b] = L.occ[v[b]];
#pragma unroll
    for (int b = 0; b < kSweepBatch; ++b)
      if (q0 + (uint64_t)b * stride < nf) L.occ[v[b]] = (uint16_t)(w[b] & kWordMask);
  }
  // the previous walk's hot marks have served both of their events
  const uint32_t np = min(L.flag_count[prv], (uint32_t)L.flag_cap);
  for (uint64_t q0 = me; q0 < np; q0 += step) {
    uint32_t v[kSweepBatch];
#pragma unroll
    for (int b = 0; b < kSweepBatch; ++b) {
      const uint64_t q = q0 + (uint64_t)b * stride;
      v[b] = L.flag_vox[prv][q < np ? q : q0];
    }
#pragma unroll
    for (int b = 0; b < kSweepBatch; ++b) {
      if (q0 + (uint64_t)b * stride >= np) continue;
      const uint32_t h = hot_hash(v[b], L.hot_bits);
      atomicAnd(&L.hot[h >> 4], ~(1u << (((h & 15u) << 1) | prv)));
    }
  }
  // No release fence before counting in (on this part it writes back the
  // L2 of the workgroup's XCD, and a batched launch has thousands of
  // workgroups): the last workgroup reads nothing the others write in this
  // kernel (it masks the flag bit off every lattice word it reads and never
  // reads the hot bitmap), and each workgroup has used the event counter
  // before it counts itself in, so the last may advance it.  The kernel
  // boundary publishes all of it to the next launch.
  if (nblk > 1) {
    __shared__ uint32_t s_last;
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(L.end_done, 1u) == nblk - 1;
    __syncthreads();
    if (!s_last) return;
    // the last workgroup: every other one has finished its sweeps
    __threadfence();
  }
  if (BIRTHS && L.wb_count) {
    const uint32_t nwb = *L.wb_count;
    if (threadIdx.x == 0) L.recent[kRecentColBirths] = nwb;
    if (!(defer && nwb > kSortLds)) number_births(L, e);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    L.flag_count[prv] = 0;  // the next walk fills this list
    if (nblk > 1) *L.end_done = 0;
    *L.ev = e + 1;
  }
}

template <bool BIRTHS>
__global__ void __launch_bounds__(kEndThreads) k_end(const LatDev *__restrict__ Lp, int defer) {
  end_body<BIRTHS>(*Lp, blockIdx.x, gridDim.x, defer != 0);
}

template <bool BIRTHS>
__global__ void __launch_bounds__(kEndThreads) k_end_multi(const LatDev *__restrict__ lats) {
  end_body<BIRTHS>(lats[blockIdx.y], blockIdx.x, gridDim.x, false);
}

// The end of the previous event and the opening of the next in one
// workgroup, one launch instead of two, for a lattice without collision
// newborns to number and an opening that k_begin does alone (no decision,
// application or ranking launches): the end's sweeps take the whole
// workgroup, and the barrier between the two parts orders its stores (the
// cleared flags, the advanced event counter) before the opening's loads,
// every wave of the workgroup running on one compute unit.
// desc: as k_begin
__global__ void __launch_bounds__(kBeginThreads) k_end_begin(const LatDev *__restrict__ Lp,
                                                             int desc) {
  end_body<false, 4>(*Lp, 0, 1, false);
  __syncthreads();
  begin_body(*Lp, false, false, false, desc != 0);
}

// The collision newborns k_end left (more than one workgroup ranks in LDS):
// ids next_id + rank over the whole grid, binned for the next event.  k_end
// has advanced the event counter: the walk was event *ev - 1.
__global__ void __launch_bounds__(kStageThreads) k_end_births(const LatDev *__restrict__ Lp) {
  const LatDev &L = *Lp;
  const RankList R = rank_list<1>(L);
  const uint32_t nb = R.nb;
  if (nb == 0) return;  // numbered by k_end, or none
  const uint64_t e = *L.ev - 1;
  const uint32_t base_id = *L.next_id;
  if ((uint64_t)base_id + nb >= 0xFFFFFFFFull) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_error(L, kErrIds);
    return;
  }
  const Bins &out = L.bins[(e + 1) & 1];
  const uint32_t cnext = (uint32_t)((e + 1) & 1);
  const uint32_t cmax_next = (L.n_fo && e + 1 < L.tape_horizon) ? L.tape_cmax[e + 1] : 0u;
  __shared__ WgBirthBins s_wb;
  rank_dealt(L, R, [&](bool valid, uint64_t k, uint32_t r) {
    bin_collision_birth(L, e, out, cnext, cmax_next, valid, k, base_id + r, s_wb);
  });
  if (!last_workgroup(L.end_done)) return;
  if (threadIdx.x == 0) {
    *L.next_id = base_id + nb;
    *L.wb_count = 0;
  }
}

// =============================================================================
// k_msd: sum over the walkers of 3 X^2 + Y^2 + 8 Z^2 (= 3 |displacement|^2 / r^2)
// =============================================================================
__global__ void __launch_bounds__(kStageThreads) k_msd(const LatDev *__restrict__ Lp,
                                                       unsigned long long *out) {
  __shared__ unsigned long long s_red[kStageThreads / 64];
  const LatDev &L = *Lp;
  const Bins &in = L.bins[*L.ev & 1];
  unsigned long long acc = 0, n = 0;
  if (in.disp) {
    const uint32_t nc = L.ncol;
    for (uint32_t c = 0; c < nc; ++c) {
      const uint32_t cnt = min(in.count[c], (uint32_t)L.cap);
      for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cnt;
           i += (uint64_t)gridDim.x * blockDim.x) {
        if (in.id[c * L.cap + i] == kDeadId) continue;
        const long long X = in.disp[(0 * nc + c) * L.cap + i];
        const long long Y = in.disp[(1 * nc + c) * L.cap + i];
        const long long Z = in.disp[(2 * nc + c) * L.cap + i];
        acc += (unsigned long long)(3 * X * X + Y * Y + 8 * Z * Z);
        ++n;
      }
    }
  }
  acc = block_sum_u64(acc, s_red);
  n = block_sum_u64(n, s_red);
  if (threadIdx.x == 0) {
    atomicAdd(&out[0], acc);
    atomicAdd(&out[1], n);
  }
}

// dst[u] = src[linear(u)] (linear -> layout) or dst[linear(u)] = src[u]
__global__ void __launch_bounds__(kStageThreads) k_relayout(Geo g, uint64_t nv,
                                                            const uint16_t *__restrict__ src,
                                                            uint16_t *__restrict__ dst,
                                                            int to_layout_order) {
  for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < nv;
       u += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t lin = linear_of(g, coord_of(g, (uint32_t)u));
    if (to_layout_order) dst[u] = src[lin];
    else dst[lin] = src[u];
  }
}

hipError_t launch_relayout(const Geo &g, uint64_t nv, const uint16_t *src, uint16_t *dst,
                           bool to_layout_order, hipStream_t s) {
  hipLaunchKernelGGL(k_relayout, dim3(8192), dim3(kStageThreads), 0, s, g, nv, src, dst,
                     to_layout_order ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_msd(const LatDev *dL, unsigned long long *out, hipStream_t s) {
  hipLaunchKernelGGL(k_msd, dim3(256), dim3(kStageThreads), 0, s, dL, out);
  return hipGetLastError();
}

// =============================================================================
// host-side launchers
// =============================================================================
hipError_t launch_scan(const LatDev *dL, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_candidates, dim3(grid), dim3(kStageThreads), 0, s, dL);
  return hipGetLastError();
}

// workgroups of the count and deal launches of the newborn ranking (a
// grid-stride pass each; the count's last workgroup waits on all of them)
constexpr int kRankGrid = 256;

hipError_t launch_begin(const LatDev *dL, const BeginShape &b, uint32_t stages, hipStream_t s,
                        bool desc, const LatDev *Lh, const uint32_t *perm, uint64_t e) {
  if (b.decide > 0) hipLaunchKernelGGL(k_decide, dim3(b.decide), dim3(kStageThreads), 0, s, dL);
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(kBeginThreads), 0, s, dL, b.decide > 0 ? 1 : 0,
                     b.births > 0 ? 1 : 0, b.apply > 0 ? 1 : 0, desc ? 1 : 0);
  if (b.apply > 0)
    for (uint32_t g = 0; g < stages; ++g) {
      if (Lh)
        hipLaunchKernelGGL(k_fo_stage_direct, dim3(b.apply), dim3(kStageThreads), 0, s, *Lh,
                           perm[g], e);
      else hipLaunchKernelGGL(k_fo_stage, dim3(b.apply), dim3(kStageThreads), 0, s, dL, g);
    }
  if (b.births > 0 || b.apply > 0) {
    const int grid = b.births > 0 ? b.births : 1;
    const int rank_grid = std::min(grid, kRankGrid);
    hipLaunchKernelGGL(k_rank_count<0>, dim3(rank_grid), dim3(kStageThreads), 0, s, dL);
    hipLaunchKernelGGL(k_rank_deal<0>, dim3(rank_grid), dim3(kStageThreads), 0, s, dL);
    hipLaunchKernelGGL(k_births, dim3(grid), dim3(kStageThreads), 0, s, dL, b.apply > 0 ? 1 : 0);
  }
  return hipGetLastError();
}

hipError_t launch_stage(const LatDev *dL, uint32_t g, int grid, int items, bool disp, bool fcc,
                        hipStream_t s) {
  return fcc ? launch_stage_lat<1>(dL, g, grid, items, disp, s)
             : launch_stage_lat<0>(dL, g, grid, items, disp, s);
}

hipError_t launch_stage_direct(const LatDev &L, uint32_t c, uint64_t e, uint64_t due,
                               uint32_t cmax_next, int grid, int items, bool disp, bool fcc,
                               hipStream_t s) {
  return fcc ? launch_stage_direct_lat<1>(L, c, e, due, cmax_next, grid, items, disp, s)
             : launch_stage_direct_lat<0>(L, c, e, due, cmax_next, grid, items, disp, s);
}

// grid of the numbering of many collision newborns (a pass ranks this many
// times 256 keys; further ones take more passes)
constexpr int kEndBirthsGrid = 512;

hipError_t launch_end(const LatDev *dL, bool births, hipStream_t s, bool defer) {
  if (births && defer) {
    hipLaunchKernelGGL(k_end<true>, dim3(kEndBlocks), dim3(kEndThreads), 0, s, dL, 1);
    hipLaunchKernelGGL(k_rank_count<1>, dim3(kRankGrid), dim3(kStageThreads), 0, s, dL);
    hipLaunchKernelGGL(k_rank_deal<1>, dim3(kRankGrid), dim3(kStageThreads), 0, s, dL);
    hipLaunchKernelGGL(k_end_births, dim3(kEndBirthsGrid), dim3(kStageThreads), 0, s, dL);
  } else if (births) {
    hipLaunchKernelGGL(k_end<true>, dim3(kEndBlocks), dim3(kEndThreads), 0, s, dL, 0);
  } else {
    hipLaunchKernelGGL(k_end<false>, dim3(kEndBlocks), dim3(kEndThreads), 0, s, dL, 0);
  }
  return hipGetLastError();
}

hipError_t launch_event(const LatDev *dL, int grid, int items, bool disp, bool fcc,
                        const BeginShape &b, bool births, hipStream_t s) {
  const uint32_t stages = fcc ? kColoursFcc : kColoursHcp;
  hipError_t err = launch_begin(dL, b, stages, s);
  for (uint32_t g = 0; g < stages && err == hipSuccess; ++g)
    err = launch_stage(dL, g, grid, items, disp, fcc, s);
  if (err == hipSuccess) err = launch_end(dL, births, s);
  return err;
}

hipError_t launch_event_direct(const LatDev *dL, const LatDev &L, uint64_t e, uint64_t due,
                               uint32_t cmax_next, int grid, int items, bool disp, bool fcc,
                               const BeginShape &b, bool births, bool births_defer,
                               hipStream_t s, bool open_with_end, bool close) {
  const uint32_t stages = fcc ? kColoursFcc : kColoursHcp;
  const bool plain = b.decide == 0 && b.births == 0 && b.apply == 0;
  if (open_with_end && (births || !plain)) return hipErrorInvalidValue;
  uint32_t perm[kMaxColours];
  stage_order_of(L.key0, L.key1, e, stages, perm);
  // the direct stage kernels take their colour and count without the
  // descriptors; larger chunks take the descriptor form
  hipError_t err;
  if (open_with_end) {
    hipLaunchKernelGGL(k_end_begin, dim3(1), dim3(kBeginThreads), 0, s, dL, items > 4 ? 1 : 0);
    err = hipGetLastError();
  } else {
    err = launch_begin(dL, b, stages, s, items > 4, &L, perm, e);
  }
  for (uint32_t g = 0; g < stages && err == hipSuccess; ++g)
    err = items <= 4 ? launch_stage_direct(L, perm[g], e, due, cmax_next, grid, items, disp, fcc, s)
                     : launch_stage(dL, g, grid, items, disp, fcc, s);
  if (err == hipSuccess && close) err = launch_end(dL, births, s, births_defer);
  return err;
}

hipError_t launch_event_multi(const LatDev *lats, uint32_t R, uint32_t stages, int grid,
                              int items, bool births, hipStream_t s) {
  if (R == 0 || R > max_members() || stages > (uint32_t)kMaxColours) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_begin_multi, dim3(R), dim3(kBeginMultiThreads), 0, s, lats);
  hipError_t err = hipGetLastError();
  if (err == hipSuccess) err = launch_multi_prefix(lats, R, stages, items, s);
  for (uint32_t g = 0; g < stages && err == hipSuccess; ++g)
    err = launch_stage_multi(lats, R, g, grid, items, s);
  if (err != hipSuccess) return err;
  if (births)
    hipLaunchKernelGGL(k_end_multi<true>, dim3(kEndBlocksMulti, R), dim3(kEndThreads), 0, s, lats);
  else
    hipLaunchKernelGGL(k_end_multi<false>, dim3(kEndBlocksMulti, R), dim3(kEndThreads), 0, s, lats);
  return hipGetLastError();
}

int stage_items() { return 4; }
int stage_threads() { return kStageThreads; }

}  // namespace psc
