// psc_device.h -- device-side building blocks of the walk kernels shared by
// the translation units of libpsc's gfx950 code: block sizes, the per-event
// stage order, first-order helpers, and one chunk of a walk stage
// (stage_chunk), which both the single-lattice and the batched stage kernels
// run.
#pragma once

#include "psc_core.h"

namespace psc {

namespace {

constexpr int kStageThreads = 256;
constexpr int kBeginThreads = 1024;

__device__ __forceinline__ uint32_t colour_of_voxel(const Geo &g, uint32_t v) {
  return colour_of(g, coord_of(g, v));
}

__device__ __forceinline__ void set_error(const LatDev &L, uint32_t bit) { atomicOr(L.error, bit); }

// ---- stage order (stage_order_of) ------------------------------------------------
__device__ __forceinline__ void stage_order(const LatDev &L, uint64_t e, uint32_t *perm) {
  stage_order_of(L.key0, L.key1, e, L.ncol, perm);
}

// The first-order tables of event e as a decision reads them: per species
// its flags, first slot and slot count; per slot its cumulative threshold
// (this event's tape row) and reaction.  From the lattice record, or from a
// workgroup's copy in LDS (FoTabLds::fill), which turns a decision's chain
// of global lookups into LDS reads.
struct FoTabGlobal {
  const LatDev &L;
  uint64_t e;
  __device__ uint32_t flags(uint32_t sp) const { return L.sp_flags[sp]; }
  __device__ uint32_t first(uint32_t sp) const { return L.fo_first[sp]; }
  __device__ uint32_t count(uint32_t sp) const { return L.fo_n[sp]; }
  __device__ uint32_t thr(uint32_t slot) const { return L.tape_thr[e * (uint64_t)L.n_fo + slot]; }
  __device__ uint32_t rx(uint32_t slot) const { return L.fo_rx[slot]; }
};
struct FoTabLds {
  uint8_t flags_[64], count_[64];
  uint16_t first_[64], rx_[kMaxReactions];
  uint32_t thr_[kMaxReactions];
  __device__ uint32_t flags(uint32_t sp) const { return flags_[sp]; }
  __device__ uint32_t first(uint32_t sp) const { return first_[sp]; }
  __device__ uint32_t count(uint32_t sp) const { return count_[sp]; }
  __device__ uint32_t thr(uint32_t slot) const { return thr_[slot]; }
  __device__ uint32_t rx(uint32_t slot) const { return rx_[slot]; }
  // by the whole workgroup; the caller's barrier publishes it
  __device__ void fill(const LatDev &L, uint64_t e) {
    for (uint32_t i = threadIdx.x; i < 64; i += blockDim.x) {
      flags_[i] = L.sp_flags[i];
      count_[i] = L.fo_n[i];
      first_[i] = L.fo_first[i];
    }
    for (uint32_t i = threadIdx.x; i < L.n_fo; i += blockDim.x) {
      rx_[i] = L.fo_rx[i];
      thr_[i] = L.tape_thr[e * (uint64_t)L.n_fo + i];
    }
  }
};

// first-order reaction fired by a molecule of species sp with first draw r0,
// or -1: the slot whose cumulative threshold first exceeds r0
template <class FoTab>
__device__ __forceinline__ int first_order_choice(const FoTab &ft, uint32_t sp, uint32_t r0) {
  const uint32_t first = ft.first(sp), n = ft.count(sp);
  for (uint32_t a = 0; a < n; ++a)
    if (r0 < ft.thr(first + a)) return (int)ft.rx(first + a);
  return -1;
}

// the words used to place extra first-order products: r.y, r.z, r.w of block
// 0, then the four words of blocks 1, 2, 3
__device__ __forceinline__ uint32_t placement_word(const LatDev &L, uint64_t e, uint32_t id, const U4 &r0,
                                          int q) {
  if (q == 0) return r0.y;
  if (q == 1) return r0.z;
  if (q == 2) return r0.w;
  const int b = 1 + (q - 3) / 4, w = (q - 3) % 4;
  const U4 r = philox((uint32_t)e, id, kPhaseFirst, (uint32_t)b, L.key0, L.key1);
  return w == 0 ? r.x : (w == 1 ? r.y : (w == 2 ? r.z : r.w));
}

// ---- block-wide helpers ----------------------------------------------------------
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long x,
                                                   unsigned long long *s_tmp) {
  // wavefront reduction, then one value per wave through LDS
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) s_tmp[wave] = x;
  __syncthreads();
  unsigned long long total = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) total += s_tmp[w];
  __syncthreads();
  return total;
}

// statistics replica of the calling workgroup: counters that many
// workgroups add to are spread over kStatRep copies (summed on the host), so
// that their atomics do not queue on one cache line
__device__ __forceinline__ uint32_t stat_rep() { return (blockIdx.x + blockIdx.y) & (kStatRep - 1u); }
__device__ __forceinline__ unsigned long long *stat_cnt(const LatDev &L) {
  return L.cnt + kCntStride * stat_rep();
}
__device__ __forceinline__ unsigned long long *stat_sp(const LatDev &L) {
  return L.sp_count + kSpStride * stat_rep();
}
__device__ __forceinline__ unsigned long long *stat_fired(const LatDev &L) {
  return L.fired + (uint64_t)L.fired_stride * stat_rep();
}

}  // namespace

// =============================================================================
// k_stage: one colour stage of the walk
// =============================================================================
// shared scratch of one walk-stage workgroup
struct StageShared {
  uint32_t cnt[kMaxColours], base[kMaxColours], loff[kMaxColours];
  uint32_t ncand, cand_base, nflag, flag_base, total;
  unsigned long long att, hop, col;
  int32_t dsp[64];   // species count changes of this chunk
  uint32_t any_rx;
};

// a chunk's surviving entries in LDS, colour-major, so that they leave for
// the bins in contiguous runs (coalesced stores)
template <int ITEMS>
struct StageStaging {
  uint32_t vox[kStageThreads * ITEMS];
  uint32_t id[kStageThreads * ITEMS];
  uint32_t spc[kStageThreads * ITEMS];  // species | colour << 16
};

// Molecules [base, base + kStageThreads * ITEMS) of colour bin c of lattice L
// in event e: each attempts one hop; collisions with a registered partner
// fire the second-order reaction; survivors are appended to the next event's
// bins through block-local slots (LDS) and one global reservation per colour.
// The kernels' buffers all live in device memory: a view in the global
// address space makes loads and stores through it global instructions
// instead of flat ones.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> global(T *p) {
  return (gptr<T>)p;
}

// The walk's reaction tables as a stage reads them: from the lattice record
// (global memory; the batched kernel) or from the workgroup's packed copy in
// LDS (stage_tab_layout).  A collision looks up the pair's reaction, its
// threshold and products one after the other: from LDS that chain costs
// tens of cycles instead of three global round trips behind the stage's
// random reads.
struct RxTabGlobal {
  const LatDev &L;
  __device__ int pair(uint32_t a, uint32_t b) const { return L.pair_rx[a * 64 + b]; }
  __device__ uint32_t thr(int rx) const { return L.rx_thr[rx]; }
  __device__ bool always(int rx) const { return L.rx_always[rx] != 0; }
  __device__ uint32_t nprod(int rx) const { return L.rx_nprod[rx]; }
  __device__ uint32_t prod(int rx, uint32_t k) const { return L.rx_prod[rx * 12 + k]; }
};
struct RxTabLds {
  const uint32_t *w;  // the workgroup's copy (LDS)
  StageTabLayout t;
  __device__ int pair(uint32_t a, uint32_t b) const {
    return ((const int16_t *)(w + t.pair))[a * 64 + b];
  }
  __device__ uint32_t thr(int rx) const { return w[t.thr + rx]; }
  __device__ bool always(int rx) const { return ((const uint8_t *)(w + t.always))[rx] != 0; }
  __device__ uint32_t nprod(int rx) const { return ((const uint8_t *)(w + t.nprod))[rx]; }
  __device__ uint32_t prod(int rx, uint32_t k) const {
    return ((const uint16_t *)(w + t.prod))[rx * 12 + k];
  }
};

// DM: displacement planes never (0), always (1), or as the lattice says (2)
// A collision of the mover (id, species sp, voxel v) with the partner at t
// (species psp) fires reaction rx (2.4.2).  The first product takes the
// partner's voxel and identity: the partner's entry (wherever it is) stays
// valid, flagged so that it does not walk again in this event, its voxel
// marked hot so that its cached species is refreshed.  The second takes the
// mover's voxel and identity; with one product the mover's identity ends.
// Further products need as many distinct vacant neighbours of v, else
// nothing happens (a placement failure): each takes entry floor(w k / 2^32)
// of the k vacant neighbours left in stencil order, w = r2, r3 of the walk
// draw, then further blocks; they are numbered at the end of the event.
// EXTRA: the reaction may have more than two products; LAT: 0 HCP, 1 FCC
template <bool EXTRA, int LAT, class OccP, class HotP, class Tab>
__device__ __forceinline__ void fire_collision(const LatDev &L, const Tab &tab, StageShared &sh, uint64_t e,
                                               uint32_t buf, uint32_t hbits, OccP occ, HotP hot,
                                               int rx, uint32_t v, uint32_t t, uint32_t sp,
                                               uint32_t psp, uint32_t id, uint32_t &osp,
                                               uint32_t &ocol, bool &flag, uint32_t &ftgt) {
  const uint32_t m = EXTRA ? tab.nprod(rx) : min(tab.nprod(rx), 2u);
  // the mover's compartment, which the partner shares: every product stays in it
  const uint32_t comp = osp & kCompBits;
  uint32_t vmask = 0;
  Coord cv;
  if (EXTRA && m > 2) {
    cv = coord_of(L.geo, v);
    for (uint32_t n = 0; n < 12; ++n) {
      Coord cn;
      if (step_target_t<LAT>(L.geo, cv, n, cn) && occ[index_of(L.geo, cn)] == comp)
        vmask |= 1u << n;
    }
    if (__popc(vmask) < (int)(m - 2)) {
      atomicAdd(&stat_cnt(L)[3], 1ull);
      return;
    }
  }
  const uint32_t prod0 = tab.prod(rx, 0);
  occ[t] = (uint16_t)(prod0 | comp | kReactedFlag);
  const uint32_t ht = hot_hash(t, hbits);
  atomicOr((uint32_t *)&hot[ht >> 4], 1u << (((ht & 15u) << 1) | buf));
  flag = true;
  ftgt = t;
  atomicSub(&sh.dsp[sp], 1);
  atomicSub(&sh.dsp[psp], 1);
  atomicAdd(&sh.dsp[prod0 & 63u], 1);
  sh.any_rx = 1;
  if (m >= 2) {
    const uint32_t prod1 = tab.prod(rx, 1);
    occ[v] = (uint16_t)(prod1 | comp);
    osp = prod1 | comp;
    atomicAdd(&sh.dsp[prod1 & 63u], 1);
  } else {
    occ[v] = (uint16_t)comp;
    ocol = 0xFFu;
  }
  for (uint32_t q = 0; EXTRA && q + 2 < m; ++q) {
    uint32_t w;
    if (q < 2) {
      const U4 r0 = philox((uint32_t)e, id, kPhaseWalk, 0, L.key0, L.key1);
      w = q == 0 ? r0.z : r0.w;
    } else {
      const U4 rb = philox((uint32_t)e, id, kPhaseWalk, 1 + (q - 2) / 4, L.key0, L.key1);
      const uint32_t k = (q - 2) & 3u;
      w = k == 0 ? rb.x : (k == 1 ? rb.y : (k == 2 ? rb.z : rb.w));
    }
    uint32_t x = scale32(w, (uint32_t)__popc(vmask)), n = 0;
    for (;; ++n) {
      if (!((vmask >> n) & 1u)) continue;
      if (x == 0) break;
      --x;
    }
    vmask &= ~(1u << n);
    Coord cn;
    step_target_t<LAT>(L.geo, cv, n, cn);
    const uint32_t u = index_of(L.geo, cn);
    const uint16_t ps = (uint16_t)tab.prod(rx, 2 + q);
    occ[u] = (uint16_t)(ps | comp);
    atomicAdd(&sh.dsp[ps & 63u], 1);
    const uint32_t slot = atomicAdd(L.wb_count, 1u);
    if (slot < L.wb_cap) {
      L.wb_vox[slot] = u;
      L.wb_key[slot] = ((uint64_t)id << 32) | ((uint64_t)(2 + q) << 28) | slot;
    } else {
      set_error(L, kErrBirthOverflow);
    }
  }
  atomicAdd(&stat_fired(L)[rx], 1ull);
}

// the event's tape words the walk reads: the species due in event e, and
// the largest first-order threshold of event e + 1 (0: no candidates to
// collect)
__device__ __forceinline__ uint64_t due_of(const LatDev &L, uint64_t e) { return L.tape_due[e]; }
__device__ __forceinline__ uint32_t cmax_after(const LatDev &L, uint64_t e) {
  return (L.n_fo && e + 1 < L.tape_horizon) ? L.tape_cmax[e + 1] : 0u;
}

// SPEC: the chunk's entries are read before the bin's count arrives (n is
// then ignored and read here): lanes clamp to the bin's capacity and are
// marked dead once the count is known, one dependent read shorter.
// due, cmax_next: due_of(L, e) and cmax_after(L, e); tab: the reaction
// tables; tab_fill: the workgroup's LDS copy that this chunk fills from the
// record's packed tables (the workgroup's first chunk), else null
template <int ITEMS, int DM, int LAT, bool SPEC = false, class Tab>
__device__ __forceinline__ void stage_chunk(const LatDev &L, uint64_t e, uint32_t c, uint64_t base, uint32_t n,
                            uint64_t due, uint32_t cmax_next, const Tab &tab, uint32_t *tab_fill,
                            StageShared &S, StageStaging<ITEMS> &stg) {
  constexpr uint32_t NC = LAT ? kColoursFcc : kColoursHcp;
  static_assert(64 * ITEMS < (1 << 21), "a wave's counts fill 21-bit fields");
  StageShared *sh = &S;
  const int tid = threadIdx.x;
  const uint32_t buf = (uint32_t)(e & 1);
  const Bins &in = L.bins[buf];
  const Bins &out = L.bins[buf ^ 1];
  const uint32_t cnext = (uint32_t)((e + 1) & 1);
  const uint64_t cap = L.cap;
  if (SPEC) n = in.count[c];  // issued with the entries below, used after them
  const uint64_t last = SPEC ? cap - 1 : (uint64_t)n - 1;
  const bool disp = DM == 2 ? in.disp != nullptr : DM == 1;
  const auto hot = global(L.hot);
  const auto occ = global(L.occ);
  const auto ivox = global(in.vox), iid = global(in.id), ovox = global(out.vox), oid = global(out.id);
  const auto isp = global(in.sp), osp_ = global(out.sp);
  const auto idsp = global(in.disp), odsp = global(out.disp);
  const uint32_t hbits = L.hot_bits;
  unsigned long long n_att = 0, n_hop = 0, n_col = 0;
  uint32_t *s_cnt = sh->cnt, *s_base = sh->base;
  uint32_t &s_ncand = sh->ncand, &s_cand_base = sh->cand_base;
  uint32_t &s_nflag = sh->nflag, &s_flag_base = sh->flag_base;

  uint32_t vox[ITEMS], id[ITEMS], ocol[ITEMS], lpos[ITEMS], osp[ITEMS];
  int32_t d0[ITEMS], d1[ITEMS], d2[ITEMS];
  bool cand[ITEMS], flag[ITEMS];
  uint32_t ftgt[ITEMS];

  // bin entries: lanes past the end read the last entry (base < n, or the
  // bin's last slot) and are then marked dead, so no load sits behind a
  // branch
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t idx = min(base + (uint64_t)it * kStageThreads + tid, last);
    vox[it] = ivox[c * cap + idx];
    id[it] = iid[c * cap + idx];
    osp[it] = isp[c * cap + idx];
    d0[it] = d1[it] = d2[it] = 0;
  }
  if (disp) {
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const uint64_t idx = min(base + (uint64_t)it * kStageThreads + tid, last);
      d0[it] = idsp[(0 * NC + c) * cap + idx];
      d1[it] = idsp[(1 * NC + c) * cap + idx];
      d2[it] = idsp[(2 * NC + c) * cap + idx];
    }
  }
  // the packed tables when this chunk fills the LDS copy: up to two words
  // per thread read now, behind the entries, and stored before the barrier
  // that precedes their first use
  const uint32_t tw = tab_fill ? L.stage_tab_words : 0u;
  uint32_t tw0 = 0, tw1 = 0;
  if ((uint32_t)tid < tw) tw0 = L.stage_tab[tid];
  if ((uint32_t)tid + kStageThreads < tw) tw1 = L.stage_tab[tid + kStageThreads];
  if (SPEC) {
    n = (uint32_t)min((uint64_t)n, cap);
    // a workgroup past the count leaves once it is known; the empty asm
    // keeps the entry reads above that test, where they overlap the count's
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) asm volatile("" ::"v"(vox[it]), "v"(id[it]), "v"(osp[it]));
    if (base >= n) return;
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    ocol[it] = 0xFFu;
    cand[it] = false;
    flag[it] = false;
    if (base + (uint64_t)it * kStageThreads + tid >= n) {
      id[it] = kDeadId;
      if (SPEC) {  // a slot past the count may hold anything: voxel 0, vacant
        vox[it] = 0;
        osp[it] = 0;
      }
    }
  }

  constexpr uint32_t kWallBit = 1u << 16;  // in mv: the target lies beyond a wall
  // Load phase: every item's draw, target and target word before any store.
  // Same-stage molecules have disjoint closed neighbourhoods, so no store of
  // this stage changes a word loaded here; issuing all loads first keeps
  // 2 x ITEMS reads in flight per thread.  The phase has no branch: dead
  // entries and tail lanes hold valid voxels (their results are dropped
  // below), and a molecule whose cached species is not due reads voxel 0
  // instead of its target.
  uint32_t tgt[ITEMS], wt[ITEMS], hw[ITEMS], hs[ITEMS], ry[ITEMS], mv[ITEMS];
  bool loaded[ITEMS];
  int drx[ITEMS];  // reaction | partner species << 8 of a deferred collision, or -1
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    drx[it] = -1;
    const uint32_t v = vox[it];
    const U4 r = philox((uint32_t)e, id[it], kPhaseWalk, 0, L.key0, L.key1);
    const uint32_t dir = scale32(r.x, 12);
    const Coord cv = coord_of(L.geo, v);
    Coord ct;
    const bool open = step_target_t<LAT>(L.geo, cv, dir, ct);
    tgt[it] = index_of(L.geo, ct);
    ry[it] = r.y;
    mv[it] = dir | (LAT ? 0u : (cv.k & 1u) << 4) | (colour_t<LAT>(ct) << 8) |
             (open ? 0u : kWallBit);
    const uint32_t h = hot_hash(v, hbits);
    hw[it] = hot[h >> 4];
    hs[it] = (h & 15u) << 1;
    loaded[it] = ((due >> (osp[it] & 63u)) & 1ull) != 0;
    wt[it] = occ[loaded[it] ? tgt[it] : 0u];
  }

  // The chunk's LDS counters, cleared only now: the barrier waits for every
  // scalar read in flight, and the reads above (entries, targets) are then
  // already under way.  The previous chunk's copy-out reads none of them.
  if (tid < (int)NC) s_cnt[tid] = 0;
  if (tid == 32) s_ncand = 0;
  if (tid == 33) s_nflag = 0;
  if (tid == 34) {
    sh->att = 0;
    sh->hop = 0;
    sh->col = 0;
    sh->any_rx = 0;
  }
  if (tid < 64) sh->dsp[tid] = 0;
  if (tw) {
    if ((uint32_t)tid < tw) tab_fill[tid] = tw0;
    if ((uint32_t)tid + kStageThreads < tw) tab_fill[tid + kStageThreads] = tw1;
    for (uint32_t i = tid + 2 * kStageThreads; i < tw; i += kStageThreads) tab_fill[i] = L.stage_tab[i];
  }
  __syncthreads();

  // Commit phase.
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    if (id[it] == kDeadId) continue;
    const uint32_t v = vox[it];
    const uint32_t t = tgt[it];
    uint32_t sp = osp[it] & kSpeciesBits;
    ocol[it] = c;  // stays in place unless it hops or is consumed
    if ((hw[it] >> hs[it]) & 3u) {
      // the cached species may be stale, or the molecule may have reacted
      // as a partner earlier in this walk: consult the lattice word
      const uint16_t w = occ[v];
      sp = w & kSpeciesBits;
      osp[it] = w & kWordMask;
      if (w & kReactedFlag) continue;
    }
    if (!((due >> sp) & 1ull)) continue;
    ++n_att;
    if (mv[it] & kWallBit) continue;  // a wall: the molecule stays, no collision
    const uint32_t w_t = loaded[it] ? wt[it] : (uint32_t)occ[t];
    const uint32_t comp = osp[it] & kCompBits;
    // a voxel of another compartment: the molecule stays, no collision (2.3)
    if ((w_t & kCompBits) != comp) continue;
    if ((w_t & kSpeciesBits) == 0) {
      occ[t] = (uint16_t)osp[it];
      occ[v] = (uint16_t)comp;
      vox[it] = t;
      ocol[it] = (mv[it] >> 8) & (LAT ? 31u : 15u);
      int32_t X, Y, Z;
      hop_vector_t<LAT>(mv[it] & 15u, (mv[it] >> 4) & 1u, X, Y, Z);
      d0[it] += X;
      d1[it] += Y;
      d2[it] += Z;
      ++n_hop;
      continue;
    }
    ++n_col;
    const uint32_t psp = w_t & kSpeciesBits;
    const int rx = tab.pair(sp, psp);
    if (rx < 0) continue;
    if (!tab.always(rx) && !(ry[it] < tab.thr(rx))) continue;
    if (tab.nprod(rx) > 2) {
      // more than two products: applied after this loop (rare), where fewer
      // of the items' values are live
      drx[it] = rx | (int)(psp << 8);
      continue;
    }
    fire_collision<false, LAT>(L, tab, *sh, e, buf, hbits, occ, hot, rx, v, t, sp, psp, id[it],
                               osp[it], ocol[it], flag[it], ftgt[it]);
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it)
    if (drx[it] >= 0)
      fire_collision<true, LAT>(L, tab, *sh, e, buf, hbits, occ, hot, drx[it] & 0xFF, vox[it],
                                tgt[it], osp[it] & 63u, (uint32_t)drx[it] >> 8, id[it], osp[it],
                                ocol[it], flag[it], ftgt[it]);

  // ---- survivors: block-local slots per colour (LDS atomics), one global
  // reservation per colour per chunk, entries staged colour-major in LDS and
  // written out in contiguous runs.  Flags and first-order candidates of the
  // next event are reserved in the same round. ----
  uint32_t fslot[ITEMS], cslot[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    if (ocol[it] != 0xFFu) {
      lpos[it] = atomicAdd(&s_cnt[ocol[it]], 1u);
      // can this molecule fire a first-order reaction in the next event?
      if (cmax_next) {
        const U4 r = philox((uint32_t)(e + 1), id[it], kPhaseFirst, 0, L.key0, L.key1);
        cand[it] = r.x < cmax_next;
      }
      if (cand[it]) cslot[it] = atomicAdd(&s_ncand, 1u);
    }
    if (flag[it]) fslot[it] = atomicAdd(&s_nflag, 1u);
  }
  // the chunk's counters: summed over the wave first, then one LDS atomic
  // per wave and counter (64-bit LDS atomics from every lane to one address
  // take microseconds).  Per thread each count is at most ITEMS, per wave at
  // most 64 ITEMS < 2^21: three fields of one 64-bit word.
  {
    constexpr unsigned long long kField = (1ull << 21) - 1;
    unsigned long long pk = n_att | (n_hop << 21) | (n_col << 42);
    for (int off = 32; off > 0; off >>= 1) pk += __shfl_xor(pk, off, 64);
    if ((tid & 63) == 0) {
      if (pk & kField) atomicAdd(&sh->att, pk & kField);
      if ((pk >> 21) & kField) atomicAdd(&sh->hop, (pk >> 21) & kField);
      if (pk >> 42) atomicAdd(&sh->col, pk >> 42);
    }
  }
  __syncthreads();
  // one wave per job: bin reservations; flag and candidate reservations;
  // local colour offsets and the chunk's counters; species count changes
  if (tid < (int)NC) {
    s_base[tid] = s_cnt[tid] ? atomicAdd(&out.count[tid], s_cnt[tid]) : 0u;
  } else if (tid == 64) {
    if (s_ncand) s_cand_base = atomicAdd(&L.cand_count[cnext], s_ncand);
  } else if (tid == 65) {
    if (s_nflag) s_flag_base = atomicAdd(&L.flag_count[buf], s_nflag);
  } else if (tid == 128) {
    uint32_t acc = 0;
    for (uint32_t k = 0; k < NC; ++k) {
      sh->loff[k] = acc;
      acc += s_cnt[k];
    }
    sh->total = acc;
  } else if (tid == 129) {
    unsigned long long *cnt = stat_cnt(L);
    if (sh->att) atomicAdd(&cnt[0], sh->att);
    if (sh->hop) atomicAdd(&cnt[1], sh->hop);
    if (sh->col) atomicAdd(&cnt[2], sh->col);
  } else if (tid >= 192) {
    const int k = tid - 192;
    if (sh->any_rx && sh->dsp[k])
      atomicAdd(&stat_sp(L)[k], (unsigned long long)(long long)sh->dsp[k]);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    if (flag[it]) {
      const uint64_t f = (uint64_t)s_flag_base + fslot[it];
      if (f < L.flag_cap) L.flag_vox[buf][f] = ftgt[it];
      else set_error(L, kErrFlagOverflow);
    }
    if (ocol[it] == 0xFFu) continue;
    const uint32_t oc = ocol[it];
    const uint32_t q = sh->loff[oc] + lpos[it];
    stg.vox[q] = vox[it];
    stg.id[q] = id[it];
    stg.spc[q] = osp[it] | (oc << 16);
    const uint64_t pos = (uint64_t)s_base[oc] + lpos[it];
    if (pos >= cap) continue;  // reported by the copy below
    if (disp) {
      odsp[(0 * NC + oc) * cap + pos] = d0[it];
      odsp[(1 * NC + oc) * cap + pos] = d1[it];
      odsp[(2 * NC + oc) * cap + pos] = d2[it];
    }
    if (cand[it]) {
      const uint64_t r = (uint64_t)s_cand_base + cslot[it];
      if (r < L.cand_cap) {
        L.cand_pos[cnext][r] = (uint32_t)pos;
        L.cand_id[cnext][r] = id[it];
        L.cand_col[cnext][r] = (uint8_t)oc;
      } else {
        set_error(L, kErrCandOverflow);
      }
    }
  }
  __syncthreads();
  // The next chunk rewrites this LDS only after two more barriers, which
  // every thread reaches after finishing this copy.
  const uint32_t total = sh->total;
  for (uint32_t q = tid; q < total; q += kStageThreads) {
    const uint32_t w = stg.spc[q];
    const uint32_t oc = w >> 16;
    const uint64_t pos = (uint64_t)s_base[oc] + (q - sh->loff[oc]);
    if (pos >= cap) {
      set_error(L, kErrBinOverflow);
      continue;
    }
    ovox[oc * cap + pos] = stg.vox[q];
    oid[oc * cap + pos] = stg.id[q];
    osp_[oc * cap + pos] = (uint16_t)(w & 0xFFFFu);
  }
}

}  // namespace psc
