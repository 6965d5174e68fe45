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
#include "psc_core.h"

namespace psc {

namespace {

constexpr int kStageThreads = 256;
constexpr int kBeginThreads = 1024;

__device__ __forceinline__ uint32_t colour_of_voxel(const Geo &g, uint32_t v) {
  return colour_of(g, coord_of(g, v));
}

__device__ __forceinline__ void set_error(const LatDev &L, uint32_t bit) { atomicOr(L.error, bit); }

// ---- stage order ---------------------------------------------------------------
// Fisher-Yates over the n colours, slot i = n-1..1 swapping with
// floor(r (i+1) / 2^32), r in sequence from the words of
// Philox(seed; e, 0xFFFFFFFF, phase 2, block 0, 1, ...).
__device__ __forceinline__ void stage_order(const LatDev &L, uint64_t e, uint32_t *perm) {
  const uint32_t n = L.ncol;
  uint32_t w[kMaxColours];
  for (uint32_t b = 0; 4 * b < n; ++b) {
    const U4 r = philox((uint32_t)e, 0xFFFFFFFFu, kPhaseStage, b, L.key0, L.key1);
    w[4 * b + 0] = r.x;
    w[4 * b + 1] = r.y;
    w[4 * b + 2] = r.z;
    w[4 * b + 3] = r.w;
  }
  for (uint32_t c = 0; c < n; ++c) perm[c] = c;
  int idx = 0;
  for (int i = (int)n - 1; i >= 1; --i) {
    const uint32_t j = scale32(w[idx++], (uint32_t)(i + 1));
    const uint32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
}

// first-order reaction fired by a molecule of species sp with first draw r0,
// or -1: the slot whose cumulative threshold first exceeds r0
__device__ __forceinline__ int first_order_choice(const LatDev &L, uint64_t e, uint32_t sp, uint32_t r0) {
  const uint32_t first = L.fo_first[sp], n = L.fo_n[sp];
  const uint32_t *C = L.tape_thr + e * (uint64_t)L.n_fo + first;
  for (uint32_t a = 0; a < n; ++a)
    if (r0 < C[a]) return (int)L.fo_rx[first + a];
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

}  // namespace

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

// For each of the nb distinct keys in LDS, f(key, rank) with rank = the
// number of smaller keys.  Each thread holds up to PER keys (PER * nthreads
// >= nb) and reads the list once.
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
  for (int a = 0; a < PER; ++a)
    if (tid + a * nthreads < nb) f(mine[a], rank[a]);
}

// one first-order firing of the molecule at (colour c, position pos): the
// first product stays in place, the others go to distinct vacant neighbours
// chosen by the placement words; too few vacant neighbours: no change
__device__ __forceinline__ void apply_first_order(const LatDev &L, uint64_t e, const Bins &in, uint32_t c,
                                  uint32_t pos, uint32_t id, uint32_t rx, uint32_t *s_nb) {
  const uint64_t at = c * L.cap + pos;
  const uint32_t v = in.vox[at];
  const uint32_t m = L.rx_nprod[rx];
  const uint16_t *prod = L.rx_prod + rx * 12;
  const uint32_t sp0 = L.occ[v] & 63u;
  if (m == 0) {
    L.occ[v] = 0;
    in.id[at] = kDeadId;
    atomicAdd(&L.sp_count[sp0], ~0ull);  // -1
    atomicAdd(&L.fired[rx], 1ull);
    return;
  }
  uint32_t dest[kMaxProducts];
  if (m > 1) {
    uint32_t vac[12];
    int nv = 0;
    const Coord cv = coord_of(L.geo, v);
    for (uint32_t n = 0; n < 12; ++n) {
      Coord ct;
      if (!step_target(L.geo, cv, n, ct)) continue;  // beyond a wall
      const uint32_t t = index_of(L.geo, ct);
      if (L.occ[t] == 0) vac[nv++] = t;
    }
    if (nv < (int)(m - 1)) {
      atomicAdd(&L.cnt[3], 1ull);
      return;
    }
    const U4 r = philox((uint32_t)e, id, kPhaseFirst, 0, L.key0, L.key1);
    for (uint32_t a = 0; a + 1 < m; ++a) {
      const uint32_t x = scale32(placement_word(L, e, id, r, (int)a), (uint32_t)nv);
      dest[a] = vac[x];
      for (int y = (int)x; y + 1 < nv; ++y) vac[y] = vac[y + 1];
      --nv;
    }
  }
  L.occ[v] = prod[0];
  in.sp[at] = prod[0];  // the entry stays; its cached species follows
  atomicAdd(&L.sp_count[sp0], ~0ull);
  atomicAdd(&L.sp_count[prod[0] & 63u], 1ull);
  for (uint32_t a = 0; a + 1 < m; ++a) {
    L.occ[dest[a]] = prod[a + 1];
    atomicAdd(&L.sp_count[prod[a + 1] & 63u], 1ull);
    const uint32_t b = atomicAdd(s_nb, 1u);
    if (b < L.birth_cap) {
      L.birth_key[b] = ((uint64_t)id << 31) | ((uint64_t)(a + 1) << 27) | b;
      L.birth_vox[b] = dest[a];
      L.birth_sp[b] = prod[a + 1];
    } else {
      atomicOr(L.error, kErrBirthOverflow);
    }
  }
  atomicAdd(&L.fired[rx], 1ull);
}

// First-order decisions of event e for candidates [first, ...) with the
// given stride: a candidate whose voxel holds a species with first-order
// reactions and whose draw falls under a cumulative threshold joins the fire
// list, counted in *nfire (LDS inside one workgroup, else global memory).
// Independent of order (a candidate's species cannot change before its own
// turn), so any number of threads and workgroups may share the list.
__device__ __forceinline__ void decide_first_order(const LatDev &L, uint64_t e, uint32_t first,
                                                   uint32_t stride, uint32_t *nfire) {
  const uint32_t buf = (uint32_t)(e & 1);
  const Bins &in = L.bins[buf];
  const uint32_t ncand = L.n_fo ? min(L.cand_count[buf], (uint32_t)L.cand_cap) : 0u;
  for (uint32_t q = first; q < ncand; q += stride) {
    const uint32_t c = L.cand_col[buf][q], pos = L.cand_pos[buf][q], id = L.cand_id[buf][q];
    const uint32_t v = in.vox[c * L.cap + pos];
    const uint32_t sp = L.occ[v] & 63u;
    if (!(L.sp_flags[sp] & kSpFirstOrder)) continue;
    const U4 r = philox((uint32_t)e, id, kPhaseFirst, 0, L.key0, L.key1);
    const int rx = first_order_choice(L, e, sp, r.x);
    if (rx < 0) continue;
    const uint32_t slot = atomicAdd(nfire, 1u);
    L.fire_pos[slot] = pos;
    L.fire_id[slot] = id;
    L.fire_col[slot] = (uint8_t)c;
    L.fire_rx[slot] = (uint8_t)rx;
  }
}

// the event's opening work for one lattice, by one workgroup; decided: the
// fire list was built by k_decide
__device__ __forceinline__ void begin_work(const LatDev &L, bool decided) {
  uint32_t *__restrict__ fire_pos = L.fire_pos;
  uint32_t *__restrict__ fire_id = L.fire_id;
  uint8_t *__restrict__ fire_col = L.fire_col;
  uint8_t *__restrict__ fire_rx = L.fire_rx;
  __shared__ uint32_t s_perm[kMaxColours], s_colcnt[kMaxColours];
  __shared__ uint32_t s_nfire, s_nb, s_next;
  __shared__ uint64_t s_keys[kSortLds];
  const uint64_t e = *L.ev;
  const int tid = threadIdx.x;
  if (e >= L.stop_event) return;  // an idle member of an ensemble
  if (e >= L.tape_horizon) {
    if (tid == 0) set_error(L, kErrTape);
    return;
  }
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
    decide_first_order(L, e, tid, blockDim.x, &s_nfire);
  else if (tid == 0)
    s_nfire = min(__hip_atomic_load(L.fire_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                  (uint32_t)L.cap);
  __syncthreads();
  const uint32_t nfire = s_nfire;

  // ---- application.  A firing molecule reads and writes only its closed
  // neighbourhood N[v] (its voxel and the 12 neighbours).  Molecules whose
  // N[v] meets no other firing molecule's commute with everything and are
  // applied at once; the others (rare) are applied stage by stage in the
  // event's order.  Overlaps are found by counting, per hashed voxel, the
  // neighbourhoods that contain it (a hash collision only sends a molecule
  // to the staged path, which is always correct). ----
  if (nfire > 0 && nfire <= blockDim.x) {
    // one firing per thread: its colour, position, draw owner, reaction and
    // the 13 hashed voxels of its neighbourhood stay in registers through
    // the count, the test, the application and the cleanup
    const uint32_t nb_bits = L.nbr_bits;
    const bool mine = (uint32_t)tid < nfire;
    uint32_t c = 0, pos = 0, id = 0, rx = 0, h[13];
    bool deferred = false;
    if (mine) {
      c = fire_col[tid];
      pos = fire_pos[tid];
      id = fire_id[tid];
      rx = fire_rx[tid];
      const uint32_t v = in.vox[c * L.cap + pos];
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
        apply_first_order(L, e, in, c, pos, id, rx, &s_nb);
      } else {
        deferred = true;  // to the staged pass
        atomicAdd(&s_colcnt[c], 1u);
      }
    }
    __syncthreads();
    for (uint32_t g = 0; g < ncol; ++g) {
      const uint32_t cg = s_perm[g];
      if (s_colcnt[cg] == 0) continue;
      if (deferred && c == cg) apply_first_order(L, e, in, c, pos, id, rx, &s_nb);
      __syncthreads();
    }
    // leave the counts at zero for the next event
    if (mine) {
#pragma unroll
      for (int a = 0; a < 13; ++a) atomicSub(&L.nbr_cnt[h[a]], 1u);
    }
    __syncthreads();
  } else if (nfire > 0) {
    const uint32_t nb_bits = L.nbr_bits;
    for (uint32_t q = tid; q < nfire; q += blockDim.x) {
      const uint32_t c = fire_col[q];
      const uint32_t v = in.vox[c * L.cap + fire_pos[q]];
      const Coord cv = coord_of(L.geo, v);
      atomicAdd(&L.nbr_cnt[hot_hash(v, nb_bits)], 1u);
      for (uint32_t n = 0; n < 12; ++n)
        atomicAdd(&L.nbr_cnt[hot_hash(index_of(L.geo, step_coord(L.geo, cv, n)), nb_bits)], 1u);
    }
    __syncthreads();
    for (uint32_t q = tid; q < nfire; q += blockDim.x) {
      const uint32_t c = fire_col[q];
      const uint32_t v = in.vox[c * L.cap + fire_pos[q]];
      const Coord cv = coord_of(L.geo, v);
      // the 13 counts (each at least 1: the molecule's own) are read at once
      // through L2, then tested together
      uint32_t other = __hip_atomic_load(&L.nbr_cnt[hot_hash(v, nb_bits)], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) ^ 1u;
#pragma unroll
      for (uint32_t n = 0; n < 12; ++n)
        other |= __hip_atomic_load(
                     &L.nbr_cnt[hot_hash(index_of(L.geo, step_coord(L.geo, cv, n)), nb_bits)],
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ^ 1u;
      const bool alone = other == 0u;
      if (alone) {
        apply_first_order(L, e, in, c, fire_pos[q], fire_id[q], fire_rx[q], &s_nb);
      } else {
        fire_col[q] = (uint8_t)(c | 0x80u);  // deferred to the staged pass
        atomicAdd(&s_colcnt[c], 1u);
      }
    }
    __syncthreads();
    for (uint32_t g = 0; g < ncol; ++g) {
      const uint32_t c = s_perm[g];
      if (s_colcnt[c] == 0) continue;
      for (uint32_t q = tid; q < nfire; q += blockDim.x)
        if (fire_col[q] == (c | 0x80u))
          apply_first_order(L, e, in, c, fire_pos[q], fire_id[q], fire_rx[q], &s_nb);
      __syncthreads();
    }
    // leave the counts at zero for the next event
    for (uint32_t q = tid; q < nfire; q += blockDim.x) {
      const uint32_t c = fire_col[q] & 0x7Fu;
      const uint32_t v = in.vox[c * L.cap + fire_pos[q]];
      const Coord cv = coord_of(L.geo, v);
      atomicSub(&L.nbr_cnt[hot_hash(v, nb_bits)], 1u);
      for (uint32_t n = 0; n < 12; ++n)
        atomicSub(&L.nbr_cnt[hot_hash(index_of(L.geo, step_coord(L.geo, cv, n)), nb_bits)], 1u);
    }
    __syncthreads();
  }

  // ---- newborn ids: ascending parent id, then product index.  The keys are
  // distinct (they end in the birth's slot), so a newborn's id is next_id
  // plus the number of smaller keys: counted in LDS up to kSortLds newborns,
  // else read off a bitonic sort in global memory ----
  const uint32_t nb = min(s_nb, (uint32_t)L.birth_cap);
  if (nb == 0) return;
  const uint32_t base_id = s_next;
  if ((uint64_t)base_id + nb >= 0xFFFFFFFFull) {
    if (tid == 0) set_error(L, kErrIds);
    return;
  }
  auto bin_birth = [&](uint64_t key, uint32_t id) {
    const uint32_t src = (uint32_t)(key & ((1u << 27) - 1u));
    const uint32_t v = L.birth_vox[src];
    const uint32_t c = colour_of_voxel(L.geo, v);
    const uint32_t pos = atomicAdd(&in.count[c], 1u);
    if (pos < L.cap) {
      const uint64_t at = c * L.cap + pos;
      in.vox[at] = v;
      in.id[at] = id;
      in.sp[at] = L.birth_sp[src];
      if (in.disp) {
        in.disp[(0 * ncol + c) * L.cap + pos] = 0;
        in.disp[(1 * ncol + c) * L.cap + pos] = 0;
        in.disp[(2 * ncol + c) * L.cap + pos] = 0;
      }
    } else {
      set_error(L, kErrBinOverflow);
    }
  };
  if (nb <= kSortLds) {
    for (uint32_t q = tid; q < nb; q += blockDim.x) s_keys[q] = L.birth_key[q];
    __syncthreads();
    for_each_ranked<kSortLds / kBeginThreads>(
        s_keys, nb, tid, kBeginThreads, [&](uint64_t k, uint32_t r) { bin_birth(k, base_id + r); });
  } else {
    uint32_t n2 = 1;
    while (n2 < nb) n2 <<= 1;
    for (uint32_t q = nb + tid; q < n2; q += blockDim.x) L.birth_key[q] = ~0ull;
    __syncthreads();
    bitonic_sort_keys(L.birth_key, n2, tid, blockDim.x);
    for (uint32_t q = tid; q < nb; q += blockDim.x) bin_birth(L.birth_key[q], base_id + q);
  }
  if (tid == 0) *L.next_id = base_id + nb;
}

// The first-order pass, then each stage's descriptor for the walk: its colour,
// its molecule count (final now: the walk appends only to the next event's
// bins) and the event, so that a stage launch starts with one load instead of
// a chain of three.  A lattice that does not run this event (idle or out of
// tape) gets empty stages, and so do the stages past its colour count.
__device__ __forceinline__ void begin_body(const LatDev &L, bool decided) {
  begin_work(L, decided);
  __syncthreads();  // every return of begin_work is taken by the whole block
  const uint32_t tid = threadIdx.x;
  if (tid == 0 && decided) *L.fire_count = 0;  // k_decide's list has been applied
  if (tid < kMaxColours) {
    const uint64_t e = *L.ev;
    const bool run = e < L.tape_horizon && e < L.stop_event && tid < L.ncol;
    const uint32_t c = run ? L.perm[tid] : 0u;
    // births were counted with atomics by other threads: read through L2
    const uint32_t n = run ? min(atomicOr(&L.bins[e & 1].count[c], 0u), (uint32_t)L.cap) : 0u;
    L.sdesc[tid] = make_uint4(c, n, (uint32_t)e, (uint32_t)(e >> 32));
  }
}

__global__ void __launch_bounds__(kBeginThreads) k_begin(const LatDev *__restrict__ Lp,
                                                         int decided) {
  begin_body(*Lp, decided != 0);
}

// one workgroup per member lattice of an ensemble
__global__ void __launch_bounds__(kBeginThreads) k_begin_multi(const LatDev *__restrict__ lats) {
  begin_body(lats[blockIdx.x], false);
}

// the first-order decisions of the coming event over many workgroups, for
// events with many candidates (k_begin then only applies the fire list)
__global__ void __launch_bounds__(kStageThreads) k_decide(const LatDev *__restrict__ Lp) {
  const LatDev &L = *Lp;
  const uint64_t e = *L.ev;
  if (e >= L.stop_event || e >= L.tape_horizon) return;
  decide_first_order(L, e, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x,
                     L.fire_count);
}

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
template <bool EXTRA, int LAT, class OccP, class HotP>
__device__ __forceinline__ void fire_collision(const LatDev &L, StageShared &sh, uint64_t e,
                                               uint32_t buf, uint32_t hbits, OccP occ, HotP hot,
                                               int rx, uint32_t v, uint32_t t, uint32_t sp,
                                               uint32_t psp, uint32_t id, uint32_t &osp,
                                               uint32_t &ocol, bool &flag, uint32_t &ftgt) {
  const uint32_t m = EXTRA ? L.rx_nprod[rx] : min(L.rx_nprod[rx], 2u);
  uint32_t vmask = 0;
  Coord cv;
  if (EXTRA && m > 2) {
    cv = coord_of(L.geo, v);
    for (uint32_t n = 0; n < 12; ++n) {
      Coord cn;
      if (step_target_t<LAT>(L.geo, cv, n, cn) && occ[index_of(L.geo, cn)] == 0) vmask |= 1u << n;
    }
    if (__popc(vmask) < (int)(m - 2)) {
      atomicAdd(&L.cnt[3], 1ull);
      return;
    }
  }
  const uint16_t *prod = L.rx_prod + rx * 12;
  occ[t] = (uint16_t)(prod[0] | kReactedFlag);
  const uint32_t ht = hot_hash(t, hbits);
  atomicOr((uint32_t *)&hot[ht >> 4], 1u << (((ht & 15u) << 1) | buf));
  flag = true;
  ftgt = t;
  atomicSub(&sh.dsp[sp], 1);
  atomicSub(&sh.dsp[psp], 1);
  atomicAdd(&sh.dsp[prod[0] & 63u], 1);
  sh.any_rx = 1;
  if (m >= 2) {
    occ[v] = prod[1];
    osp = prod[1];
    atomicAdd(&sh.dsp[prod[1] & 63u], 1);
  } else {
    occ[v] = 0;
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
    const uint16_t ps = prod[2 + q];
    occ[u] = ps;
    atomicAdd(&sh.dsp[ps & 63u], 1);
    const uint32_t slot = atomicAdd(L.wb_count, 1u);
    if (slot < L.wb_cap) {
      L.wb_vox[slot] = u;
      L.wb_key[slot] = ((uint64_t)id << 32) | ((uint64_t)(2 + q) << 28) | slot;
    } else {
      set_error(L, kErrBirthOverflow);
    }
  }
  atomicAdd(&L.fired[rx], 1ull);
}

template <int ITEMS, int DM, int LAT>
__device__ __forceinline__ void stage_chunk(const LatDev &L, uint64_t e, uint32_t c, uint64_t base, uint32_t n,
                            StageShared &S, StageStaging<ITEMS> &stg) {
  constexpr uint32_t NC = LAT ? kColoursFcc : kColoursHcp;
  StageShared *sh = &S;
  const int tid = threadIdx.x;
  const uint32_t buf = (uint32_t)(e & 1);
  const Bins &in = L.bins[buf];
  const Bins &out = L.bins[buf ^ 1];
  const uint64_t due = L.tape_due[e];
  const uint32_t cmax_next = (L.n_fo && e + 1 < L.tape_horizon) ? L.tape_cmax[e + 1] : 0u;
  const uint32_t cnext = (uint32_t)((e + 1) & 1);
  const uint64_t cap = L.cap;
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
  __syncthreads();

  uint32_t vox[ITEMS], id[ITEMS], ocol[ITEMS], lpos[ITEMS], osp[ITEMS];
  int32_t d0[ITEMS], d1[ITEMS], d2[ITEMS];
  bool cand[ITEMS], flag[ITEMS];
  uint32_t ftgt[ITEMS];

  // bin entries: lanes past the end read the last entry (base < n) and are
  // then marked dead, so no load sits behind a branch
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t idx = min(base + (uint64_t)it * kStageThreads + tid, (uint64_t)n - 1);
    vox[it] = ivox[c * cap + idx];
    id[it] = iid[c * cap + idx];
    osp[it] = isp[c * cap + idx];
    d0[it] = d1[it] = d2[it] = 0;
  }
  if (disp) {
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const uint64_t idx = min(base + (uint64_t)it * kStageThreads + tid, (uint64_t)n - 1);
      d0[it] = idsp[(0 * NC + c) * cap + idx];
      d1[it] = idsp[(1 * NC + c) * cap + idx];
      d2[it] = idsp[(2 * NC + c) * cap + idx];
    }
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    ocol[it] = 0xFFu;
    cand[it] = false;
    flag[it] = false;
    if (base + (uint64_t)it * kStageThreads + tid >= n) id[it] = kDeadId;
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

  // Commit phase.
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    if (id[it] == kDeadId) continue;
    const uint32_t v = vox[it];
    const uint32_t t = tgt[it];
    uint32_t sp = osp[it] & 63u;
    ocol[it] = c;  // stays in place unless it hops or is consumed
    if ((hw[it] >> hs[it]) & 3u) {
      // the cached species may be stale, or the molecule may have reacted
      // as a partner earlier in this walk: consult the lattice word
      const uint16_t w = occ[v];
      sp = w & 63u;
      osp[it] = sp;
      if (w & kReactedFlag) continue;
    }
    if (!((due >> sp) & 1ull)) continue;
    ++n_att;
    if (mv[it] & kWallBit) continue;  // a wall: the molecule stays, no collision
    const uint32_t w_t = loaded[it] ? wt[it] : (uint32_t)occ[t];
    if (w_t == 0) {
      occ[t] = (uint16_t)sp;
      occ[v] = 0;
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
    const uint32_t psp = w_t & 63u;
    const int rx = L.pair_rx[sp * 64 + psp];
    if (rx < 0) continue;
    if (!L.rx_always[rx] && !(ry[it] < L.rx_thr[rx])) continue;
    if (L.rx_nprod[rx] > 2) {
      // more than two products: applied after this loop (rare), where fewer
      // of the items' values are live
      drx[it] = rx | (int)(psp << 8);
      continue;
    }
    fire_collision<false, LAT>(L, *sh, e, buf, hbits, occ, hot, rx, v, t, sp, psp, id[it],
                               osp[it], ocol[it], flag[it], ftgt[it]);
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it)
    if (drx[it] >= 0)
      fire_collision<true, LAT>(L, *sh, e, buf, hbits, occ, hot, drx[it] & 0xFF, vox[it],
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
  if (n_att) atomicAdd(&sh->att, n_att);
  if (n_hop) atomicAdd(&sh->hop, n_hop);
  if (n_col) atomicAdd(&sh->col, n_col);
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
    if (sh->att) atomicAdd(&L.cnt[0], sh->att);
    if (sh->hop) atomicAdd(&L.cnt[1], sh->hop);
    if (sh->col) atomicAdd(&L.cnt[2], sh->col);
  } else if (tid >= 192) {
    const int k = tid - 192;
    if (sh->any_rx && sh->dsp[k])
      atomicAdd(&L.sp_count[k], (unsigned long long)(long long)sh->dsp[k]);
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
    if (L.geo.fcc) stage_chunk<ITEMS, 2, 1>(L, e, d.x, (uint64_t)(q - s_pre[a]) * chunk, d.y, S, T);
    else stage_chunk<ITEMS, 2, 0>(L, e, d.x, (uint64_t)(q - s_pre[a]) * chunk, d.y, S, T);
  }
}

// =============================================================================
// k_end: clear reacted flags and the previous event's hot bitmap, advance the
// event counter (the last workgroup to finish does the bookkeeping)
// =============================================================================
constexpr int kEndThreads = kStageThreads;
constexpr int kEndBlocks = 32;
constexpr int kEndBlocksMulti = 4;

// workgroup bid of nblk: sweep flags and the previous hot bitmap; the last
// workgroup to finish advances the lattice's event counter
// Newborns of this walk's many-product collisions get ids next_id, ... in
// ascending (mover id, product index) order and join the next event's bins
// with their current species (one may have changed as a later partner);
// they are also tested as first-order candidates of the next event, which a
// walk does for every other molecule.  Run by one whole workgroup.
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
  auto bin_newborn = [&](uint64_t key, uint32_t id) {
    const uint32_t u = L.wb_vox[key & ((1u << 28) - 1u)];
    const uint32_t c = colour_of_voxel(L.geo, u);
    const uint32_t pos = atomicAdd(&out.count[c], 1u);
    if (pos >= L.cap) {
      set_error(L, kErrBinOverflow);
      return;
    }
    const uint64_t at = c * L.cap + pos;
    out.vox[at] = u;
    out.id[at] = id;
    out.sp[at] = (uint16_t)(L.occ[u] & kSpeciesMask);
    if (out.disp) {
      out.disp[(0 * L.ncol + c) * L.cap + pos] = 0;
      out.disp[(1 * L.ncol + c) * L.cap + pos] = 0;
      out.disp[(2 * L.ncol + c) * L.cap + pos] = 0;
    }
    if (cmax_next) {
      const U4 r = philox((uint32_t)(e + 1), id, kPhaseFirst, 0, L.key0, L.key1);
      if (r.x < cmax_next) {
        const uint32_t k = atomicAdd(&L.cand_count[cnext], 1u);
        if (k < L.cand_cap) {
          L.cand_pos[cnext][k] = pos;
          L.cand_id[cnext][k] = id;
          L.cand_col[cnext][k] = (uint8_t)c;
        } else {
          set_error(L, kErrCandOverflow);
        }
      }
    }
  };
  if (nb <= kSortLds) {
    for (uint32_t q = tid; q < nb; q += blockDim.x) s_wkeys[q] = L.wb_key[q];
    __syncthreads();
    for_each_ranked<kSortLds / kEndThreads>(
        s_wkeys, nb, tid, kEndThreads, [&](uint64_t k, uint32_t r) { bin_newborn(k, base_id + r); });
  } else {
    uint32_t n2 = 1;
    while (n2 < nb) n2 <<= 1;  // <= wb_cap, a power of two
    for (uint32_t q = nb + tid; q < n2; q += blockDim.x) L.wb_key[q] = ~0ull;
    __syncthreads();
    bitonic_sort_keys(L.wb_key, n2, tid, blockDim.x);
    for (uint32_t q = tid; q < nb; q += blockDim.x) bin_newborn(L.wb_key[q], base_id + q);
  }
  __syncthreads();
  if (tid == 0) {
    *L.next_id = base_id + nb;
    *L.wb_count = 0;
  }
}

__device__ __forceinline__ void end_body(const LatDev &L, uint32_t bid, uint32_t nblk) {
  const uint64_t e = *L.ev;
  if (e >= L.tape_horizon || e >= L.stop_event) return;
  const uint32_t cur = (uint32_t)(e & 1), prv = cur ^ 1u;
  const uint32_t stride = nblk * blockDim.x;
  const uint32_t me = bid * blockDim.x + threadIdx.x;
  // this walk's partners may walk again from the next event on
  const uint32_t nf = min(L.flag_count[cur], (uint32_t)L.flag_cap);
  for (uint32_t q = me; q < nf; q += stride) {
    const uint32_t v = L.flag_vox[cur][q];
    L.occ[v] = (uint16_t)(L.occ[v] & kSpeciesMask);
  }
  // the previous walk's hot marks have served both of their events
  const uint32_t np = min(L.flag_count[prv], (uint32_t)L.flag_cap);
  for (uint32_t q = me; q < np; q += stride) {
    const uint32_t h = hot_hash(L.flag_vox[prv][q], L.hot_bits);
    atomicAnd(&L.hot[h >> 4], ~(1u << (((h & 15u) << 1) | prv)));
  }
  // No release fence before counting in (on this part it writes back the
  // L2 of the workgroup's XCD, and a batched launch has thousands of
  // workgroups): the last workgroup reads nothing the others write in this
  // kernel (it masks the flag bit off every lattice word it reads and never
  // reads the hot bitmap), and each workgroup has used the event counter
  // before it counts itself in, so the last may advance it.  The kernel
  // boundary publishes all of it to the next launch.
  __shared__ uint32_t s_last;
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(L.end_done, 1u) == nblk - 1;
  __syncthreads();
  if (!s_last) return;
  // the last workgroup: every other one has finished its sweeps
  __threadfence();
  if (L.wb_count) number_births(L, e);
  __syncthreads();
  if (threadIdx.x == 0) {
    L.flag_count[prv] = 0;  // the next walk fills this list
    *L.end_done = 0;
    *L.ev = e + 1;
  }
}

__global__ void __launch_bounds__(kEndThreads) k_end(const LatDev *__restrict__ Lp) {
  end_body(*Lp, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kEndThreads) k_end_multi(const LatDev *__restrict__ lats) {
  end_body(lats[blockIdx.y], blockIdx.x, gridDim.x);
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

hipError_t launch_begin(const LatDev *dL, int decide_grid, hipStream_t s) {
  if (decide_grid > 0)
    hipLaunchKernelGGL(k_decide, dim3(decide_grid), dim3(kStageThreads), 0, s, dL);
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(kBeginThreads), 0, s, dL, decide_grid > 0 ? 1 : 0);
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

hipError_t launch_stage(const LatDev *dL, uint32_t g, int grid, int items, bool disp, bool fcc,
                        hipStream_t s) {
  if (fcc) {
    if (disp) launch_stage_dm<1, 1>(dL, g, grid, items, s);
    else launch_stage_dm<0, 1>(dL, g, grid, items, s);
  } else {
    if (disp) launch_stage_dm<1, 0>(dL, g, grid, items, s);
    else launch_stage_dm<0, 0>(dL, g, grid, items, s);
  }
  return hipGetLastError();
}

hipError_t launch_end(const LatDev *dL, hipStream_t s) {
  hipLaunchKernelGGL(k_end, dim3(kEndBlocks), dim3(kEndThreads), 0, s, dL);
  return hipGetLastError();
}

hipError_t launch_event(const LatDev *dL, int grid, int items, bool disp, bool fcc,
                        int decide_grid, hipStream_t s) {
  hipError_t err = launch_begin(dL, decide_grid, s);
  const uint32_t stages = fcc ? kColoursFcc : kColoursHcp;
  for (uint32_t g = 0; g < stages && err == hipSuccess; ++g)
    err = launch_stage(dL, g, grid, items, disp, fcc, s);
  if (err == hipSuccess) err = launch_end(dL, s);
  return err;
}

hipError_t launch_event_multi(const LatDev *lats, uint32_t R, uint32_t stages, int grid,
                              int items, hipStream_t s) {
  if (R == 0 || R > kMaxMembers || stages > (uint32_t)kMaxColours) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_begin_multi, dim3(R), dim3(kBeginThreads), 0, s, lats);
  for (uint32_t g = 0; g < stages; ++g) {
    switch (items) {
    case 1: hipLaunchKernelGGL(k_stage_multi<1>, dim3(grid), dim3(kStageThreads), 0, s, lats, R, g); break;
    case 2: hipLaunchKernelGGL(k_stage_multi<2>, dim3(grid), dim3(kStageThreads), 0, s, lats, R, g); break;
    case 8: hipLaunchKernelGGL(k_stage_multi<8>, dim3(grid), dim3(kStageThreads), 0, s, lats, R, g); break;
    default: hipLaunchKernelGGL(k_stage_multi<4>, dim3(grid), dim3(kStageThreads), 0, s, lats, R, g); break;
    }
  }
  hipLaunchKernelGGL(k_end_multi, dim3(kEndBlocksMulti, R), dim3(kEndThreads), 0, s, lats);
  return hipGetLastError();
}

uint32_t max_members() { return kMaxMembers; }

int stage_items() { return 4; }
int stage_threads() { return kStageThreads; }

}  // namespace psc
