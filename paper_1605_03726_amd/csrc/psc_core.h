// psc_core.h -- definitions shared by the host core and the gfx950 kernels of
// libpsc: the device-side lattice record, the counter-based generator, the
// stencils of the two close packings (HCP, FCC) in twisted Cartesian
// coordinates and division by invariant integers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psc {

// ---- occupancy words -------------------------------------------------------
// uint16 per voxel: species id (0 = vacant) in bits 0-5, the voxel's
// compartment (a group of voxels, 2) in bits 6-13.  Bit 15 marks a voxel
// whose molecule took part, as the partner, in a collision reaction during
// the current walk: that molecule does not walk again in this event.  The
// flag is cleared before the walk ends.  A vacant voxel's word is its
// compartment bits alone; a molecule never changes compartment (a hop into
// another compartment fails, 2.3), so a bin entry caches its molecule's word.
constexpr uint16_t kSpeciesBits = 0x003F;
constexpr uint16_t kCompBits = 0x3FC0;
constexpr uint32_t kCompShift = 6;
constexpr uint16_t kWordMask = 0x7FFF;  // species and compartment, flag off
constexpr uint16_t kReactedFlag = 0x8000;
constexpr int kMaxCompartments = 256;

constexpr uint32_t kDeadId = 0xFFFFFFFFu;   // entry of a molecule that died
// stage colours: 16 on both lattices
constexpr int kColoursHcp = 16, kColoursFcc = 16, kMaxColours = 16;
constexpr int kMaxSpecies = 63;
constexpr int kMaxProducts = 11;
constexpr int kMaxReactions = 255;

// Philox counter phase word
constexpr uint32_t kPhaseWalk = 0, kPhaseFirst = 1, kPhaseStage = 2, kPhasePlace = 3;

// device error bits
constexpr uint32_t kErrBinOverflow = 1u, kErrCandOverflow = 2u, kErrFlagOverflow = 4u,
                   kErrBirthOverflow = 8u, kErrTape = 16u, kErrIds = 32u,
                   kErrCapacity = 64u;

// species flags
constexpr uint8_t kSpMobile = 1, kSpFirstOrder = 2;

// Statistics counters (attempts, hops, collisions, placement failures; live
// molecules per species; firings per reaction) are kept in kStatRep
// replicas, one per group of workgroups, each starting on its own 128-byte
// line; the host sums them.  A counter that every workgroup of a stage adds
// to would otherwise queue those 64-bit atomics on one line.
constexpr uint32_t kStatRep = 16;
constexpr uint32_t kCntStride = 16;  // words per replica of the four counters
constexpr uint32_t kSpStride = 64;   // words per replica of the species counts

// ---- Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ---------------------
// Counter (c0, c1, c2, c3) = (event, molecule id, phase, block), key = seed.
struct U4 {
  uint32_t x, y, z, w;
};

__host__ __device__ inline uint32_t mulhi32(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umulhi(a, b);
#else
  return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
#endif
}

__host__ __device__ inline U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = mulhi32(M0, c0), lo0 = M0 * c0;
    const uint32_t hi1 = mulhi32(M1, c2), lo1 = M1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return U4{c0, c1, c2, c3};
}

// floor(r * m / 2^32): a uniform integer in [0, m) from one 32-bit word
__host__ __device__ inline uint32_t scale32(uint32_t r, uint32_t m) {
  return (uint32_t)(((uint64_t)r * (uint64_t)m) >> 32);
}

// ---- the walk's reaction tables packed into 32-bit words, as the stage
// kernels copy them into LDS: offsets in words of the pair table's rows 0..ns
// (64 int16 each), the thresholds (n_rx words), the products (12 uint16 per
// reaction), the product counts and the always-fire flags (a byte per
// reaction each) ----
struct StageTabLayout {
  uint32_t pair, thr, prod, nprod, always, words;
};
__host__ __device__ constexpr StageTabLayout stage_tab_layout(uint32_t n_species, uint32_t n_rx) {
  return StageTabLayout{0,
                        (n_species + 1) * 32,
                        (n_species + 1) * 32 + n_rx,
                        (n_species + 1) * 32 + n_rx * 7,
                        (n_species + 1) * 32 + n_rx * 7 + (n_rx + 3) / 4,
                        (n_species + 1) * 32 + n_rx * 7 + 2 * ((n_rx + 3) / 4)};
}
// the largest packing: 63 species, 255 reactions
constexpr uint32_t kStageTabWordsMax = stage_tab_layout(kMaxSpecies, kMaxReactions).words;

// ---- stage order of event e: Fisher-Yates over the n <= 16 colours, slot
// i = n-1..1 swapping with floor(r (i+1) / 2^32), r in sequence from the
// words of Philox(key; e, 0xFFFFFFFF, phase 2, block 0, 1, ...).  The
// device draws it at the start of each event; the host draws the same to
// hand each stage launch its colour. ----
static_assert(kMaxColours <= 16, "the stage order draws one Philox block per 4 colours");
__host__ __device__ inline void stage_order_of(uint32_t key0, uint32_t key1, uint64_t e,
                                               uint32_t n, uint32_t *perm) {
  uint32_t w[16];
  for (uint32_t b = 0; 4 * b < n; ++b) {
    const U4 r = philox((uint32_t)e, 0xFFFFFFFFu, kPhaseStage, b, key0, key1);
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

// ---- division by an invariant 32-bit divisor ------------------------------
// Granlund & Montgomery, "Division by invariant integers using
// multiplication" (PLDI 1994), unsigned case: with l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1, q = (t + ((n - t) >> s1)) >> s2 where
// t = mulhi(m, n), s1 = min(l, 1), s2 = max(l - 1, 0); exact for all n < 2^32.
struct DivU32 {
  uint32_t d, m, s1, s2;
};

inline DivU32 make_div(uint32_t d) {
  uint32_t l = 0;
  while (l < 32 && (1ull << l) < d) ++l;
  DivU32 q;
  q.d = d;
  q.m = (uint32_t)((((1ull << l) - d) << 32) / d + 1ull);
  q.s1 = l < 1 ? l : 1;
  q.s2 = l > 0 ? l - 1 : 0;
  return q;
}

__host__ __device__ inline uint32_t divu(uint32_t n, const DivU32 &q) {
  const uint32_t t = mulhi32(q.m, n);
  return (t + ((n - t) >> q.s1)) >> q.s2;
}

// ---- geometry -----------------------------------------------------------------
// Voxel (i, j, k), v = i + ni (j + nj k).  Rows of close-packed voxels along
// i, rows of a layer shifted by half a voxel in turn along j, layers along k
// (2.1): the voxel centre is x = r (2i + s), y = (r / sqrt3)(3j + p),
// z = 2 sqrt(2/3) r k with the layer phase p = k & 1 (HCP, ABAB stacking) or
// p = k mod 3 (FCC, ABC stacking) and s = (j + p) & 1.  The stencils and hop
// vectors below follow from these positions; tables are bit-packed so that
// lanes taking different directions do not diverge.
// Memory layout of the occupancy words.  Linear: v = i + ni (j + nj k).
// Brick: the lattice is cut into 4 x 4 x 4 bricks of 64 words (one 128-byte
// cache line each), bricks in linear order, voxels inside a brick in linear
// order: u = 64 ((kb nbj + jb) nbi + ib) + 16 (k & 3) + 4 (j & 3) + (i & 3)
// with ib = i / 4 etc.  Two thirds of the hops then stay inside the mover's
// line (one sixth in the linear layout).  The layout changes addresses only;
// the ABI always speaks linear indices.
struct Geo {
  uint32_t ni, nj, nk;
  DivU32 dni, dnj;
  uint32_t brick;       // 1: brick layout
  uint32_t walls;       // 1: the box is closed by walls (no periodic wrap)
  uint32_t fcc;         // 1: face-centred cubic lattice (ABC stacking), 0: HCP
  uint32_t nbi, nbj;    // bricks along i and j
  DivU32 dnbi, dnbj;
};

struct Coord {
  int32_t i, j, k;
};

__host__ __device__ inline Coord coord_of(const Geo &g, uint32_t v) {
  Coord c;
  if (g.brick) {
    const uint32_t b = v >> 6;
    const uint32_t a = divu(b, g.dnbi);
    const uint32_t kb = divu(a, g.dnbj);
    c.i = (int32_t)(((b - a * g.nbi) << 2) | (v & 3u));
    c.j = (int32_t)(((a - kb * g.nbj) << 2) | ((v >> 2) & 3u));
    c.k = (int32_t)((kb << 2) | ((v >> 4) & 3u));
    return c;
  }
  const uint32_t a = divu(v, g.dni);
  const uint32_t k = divu(a, g.dnj);
  c.i = (int32_t)(v - a * g.ni);
  c.j = (int32_t)(a - k * g.nj);
  c.k = (int32_t)k;
  return c;
}

// linear index of a coordinate (the ABI's voxel index)
__host__ __device__ inline uint32_t linear_of(const Geo &g, const Coord &c) {
  return (uint32_t)c.i + g.ni * ((uint32_t)c.j + g.nj * (uint32_t)c.k);
}

__host__ __device__ inline uint32_t index_of(const Geo &g, const Coord &c) {
  if (g.brick) {
    const uint32_t ib = (uint32_t)c.i >> 2, jb = (uint32_t)c.j >> 2, kb = (uint32_t)c.k >> 2;
    return (((kb * g.nbj + jb) * g.nbi + ib) << 6) | (((uint32_t)c.k & 3u) << 4) |
           (((uint32_t)c.j & 3u) << 2) | ((uint32_t)c.i & 3u);
  }
  return (uint32_t)c.i + g.ni * ((uint32_t)c.j + g.nj * (uint32_t)c.k);
}

// layout index <-> linear index
__host__ __device__ inline uint32_t to_layout(const Geo &g, uint32_t lin) {
  if (!g.brick) return lin;
  const uint32_t a = divu(lin, g.dni);
  const uint32_t k = divu(a, g.dnj);
  Coord c;
  c.i = (int32_t)(lin - a * g.ni);
  c.j = (int32_t)(a - k * g.nj);
  c.k = (int32_t)k;
  return index_of(g, c);
}

__host__ __device__ inline uint32_t to_linear(const Geo &g, uint32_t u) {
  return g.brick ? linear_of(g, coord_of(g, u)) : u;
}

// Stage colour of a voxel: voxels of one colour are >= 3 hops apart.
//   HCP: 8 (k & 1) + 4 (j & 1) + ((i - j + k) mod 4)
//   FCC: (2a + 3b + 7k) mod 16 on the lattice's Bravais coordinates
//   a = i - floor((j + q) / 2) - floor(k / 3), b = j - floor(k / 3),
//   q = k mod 3 (periodic when the i and j edges are multiples of 8);
//   unsigned wrap-around keeps the residue, 16 dividing 2^32
// LAT: 0 HCP, 1 FCC
template <int LAT>
__host__ __device__ inline uint32_t colour_t(const Coord &c) {
  if (LAT) {
    const uint32_t i = (uint32_t)c.i, j = (uint32_t)c.j, k = (uint32_t)c.k;
    const uint32_t k3 = k / 3u, q = k - 3u * k3;
    return (2u * i + 3u * j + 7u * k - 2u * ((j + q) >> 1) - 5u * k3) & 15u;
  }
  return 8u * (uint32_t)(c.k & 1) + 4u * (uint32_t)(c.j & 1) +
         (uint32_t)((c.i + 3 * c.j + c.k) & 3);
}

__host__ __device__ inline uint32_t colour_of(const Geo &g, const Coord &c) {
  return g.fcc ? colour_t<1>(c) : colour_t<0>(c);
}

__host__ __device__ inline uint32_t n_colours(const Geo &g) {
  return g.fcc ? (uint32_t)kColoursFcc : (uint32_t)kColoursHcp;  // 16 on both
}

// Target coordinate of hop n from c (periodic).  Rows 0..7, 9, 10 are shared
// by both lattices with the in-row offset s: 0:(+1,0,0) 1:(-1,0,0) 2:(s,+1,0)
// 3:(s-1,+1,0) 4:(s,-1,0) 5:(s-1,-1,0) 6:(s,a,+1) 7:(s-1,a,+1) 9:(s,b,-1)
// 10:(s-1,b,-1), and rows 8:(0,c,+1), 11:(0,d,-1).
//   HCP (ABAB, p = k & 1): s = (j + k) & 1, a = b = 0, c = d = 2p - 1.
//   FCC (ABC, q = k mod 3): s = (j + q) & 1; a = 0, c = -1 for q < 2 and
//   a = 1, c = 0 for q = 2; b = 0, d = 1 for q > 0 and b = -1, d = 0 for
//   q = 0 (the layer above is shifted by (r, r/sqrt3) in the plane, the one
//   below by the opposite).
template <int LAT>
__host__ __device__ inline Coord step_coord_t(const Geo &g, const Coord &c, uint32_t n) {
  int32_t s, a = 0, b = 0, cu, dd;
  if (LAT) {
    const int32_t q = (int32_t)((uint32_t)c.k % 3u);
    s = (c.j + q) & 1;
    a = q == 2 ? 1 : 0;
    cu = q == 2 ? 0 : -1;
    b = q == 0 ? -1 : 0;
    dd = q == 0 ? 0 : 1;
  } else {
    s = (c.j + c.k) & 1;
    cu = dd = 2 * (c.k & 1) - 1;
  }
  // rows 2..7, 9, 10 have di = s (even rows of each pair) or s - 1 (rows
  // 3, 5, 7, 10); rows 0, 1 have di = +1, -1; rows 8, 11 have di = 0
  constexpr uint32_t kUsesS = 0x6FCu, kMinusOne = 0x4A8u;
  int32_t di;
  if ((kUsesS >> n) & 1u)
    di = s - (int32_t)((kMinusOne >> n) & 1u);
  else
    di = (n == 0) ? 1 : (n == 1 ? -1 : 0);
  int32_t dj = 0;
  if (n == 2 || n == 3) dj = 1;
  else if (n == 4 || n == 5) dj = -1;
  else if (n == 8) dj = cu;
  else if (n == 11) dj = dd;
  else if (LAT && (n == 6 || n == 7)) dj = a;
  else if (LAT && (n == 9 || n == 10)) dj = b;
  const int32_t dk = (n >= 6 && n <= 8) ? 1 : (n >= 9 ? -1 : 0);
  Coord t;
  t.i = c.i + di;
  t.j = c.j + dj;
  t.k = c.k + dk;
  if (t.i < 0) t.i += (int32_t)g.ni;
  else if (t.i >= (int32_t)g.ni) t.i -= (int32_t)g.ni;
  if (t.j < 0) t.j += (int32_t)g.nj;
  else if (t.j >= (int32_t)g.nj) t.j -= (int32_t)g.nj;
  if (t.k < 0) t.k += (int32_t)g.nk;
  else if (t.k >= (int32_t)g.nk) t.k -= (int32_t)g.nk;
  return t;
}

__host__ __device__ inline Coord step_coord(const Geo &g, const Coord &c, uint32_t n) {
  return g.fcc ? step_coord_t<1>(g, c, n) : step_coord_t<0>(g, c, n);
}

// target of hop n from c in the lattice's box: false if a wall closes the box
// there (t is then the periodic image, a valid voxel that must not be used)
template <int LAT>
__host__ __device__ inline bool step_target_t(const Geo &g, const Coord &c, uint32_t n, Coord &t) {
  t = step_coord_t<LAT>(g, c, n);
  if (!g.walls) return true;
  // every hop moves each coordinate by at most 1, and the edges are >= 4:
  // wrapping moved exactly the coordinates that left the box
  const int32_t di = t.i - c.i, dj = t.j - c.j, dk = t.k - c.k;
  return di >= -1 && di <= 1 && dj >= -1 && dj <= 1 && dk >= -1 && dk <= 1;
}

__host__ __device__ inline bool step_target(const Geo &g, const Coord &c, uint32_t n, Coord &t) {
  return g.fcc ? step_target_t<1>(g, c, n, t) : step_target_t<0>(g, c, n, t);
}

// Hop vector of row n (X in r, Y in r/sqrt3, Z in 2 sqrt(2/3) r):
//   X = 2,-2,1,-1,1,-1,1,-1,0,1,-1,0   Z = 0,0,0,0,0,0,1,1,1,-1,-1,-1
//   HCP: Y = 0,0,3,3,-3,-3,c,c,d,c,c,d  with c = 1-2p, d = 4p-2 (p = k & 1)
//   FCC: Y = 0,0,3,3,-3,-3,1,1,-2,-1,-1,2 (a Bravais lattice: no phase)
template <int LAT>
__host__ __device__ inline void hop_vector_t(uint32_t n, int32_t p, int32_t &X, int32_t &Y,
                                             int32_t &Z) {
  // X + 2 packed 4 bits per row: 4,0,3,1,3,1,3,1,2,3,1,2
  constexpr uint64_t kX = 0x213213131304ull;
  X = (int32_t)((kX >> (4 * n)) & 0xFu) - 2;
  if (LAT) {
    // Y + 3 packed 4 bits per row: 3,3,6,6,0,0,4,4,1,2,2,5
    constexpr uint64_t kY = 0x522144006633ull;
    Y = (int32_t)((kY >> (4 * n)) & 0xFu) - 3;
  } else {
    const int32_t c = 1 - 2 * p, d = 4 * p - 2;
    if (n < 2) Y = 0;
    else if (n < 4) Y = 3;
    else if (n < 6) Y = -3;
    else if (n == 8 || n == 11) Y = d;
    else Y = c;
  }
  Z = (n >= 6 && n <= 8) ? 1 : (n >= 9 ? -1 : 0);
}

// ---- device-side lattice record ----------------------------------------------
// Molecules live in per-colour bins (the colour of their voxel), double
// buffered by event parity: the walk of event e reads bins[e & 1] and appends
// every surviving molecule to bins[(e + 1) & 1] under its new colour.  The
// order inside a bin carries no meaning: same-colour updates commute.
struct Bins {
  uint32_t *vox;    // [ncol * cap]
  uint32_t *id;     // [ncol * cap]
  uint16_t *sp;     // [ncol * cap] species when the entry was last written
  int32_t *disp;    // [3 * ncol * cap] (dx | dy | dz planes) or nullptr
  uint32_t *count;  // [kMaxColours] (entries past ncol stay zero)
};

// Voxels where a collision put a product on the partner's voxel are marked
// in a hash bitmap.  Only there can a bin entry's cached species be stale
// (the partner keeps its entry and its id but changes species), or the
// molecule be one that must not walk again in this event; everywhere else the
// walk trusts the cached species and never reads the lattice word at the
// mover's voxel.  Each 32-bit word holds 16 hash slots with one bit per event
// parity (bit 2 slot + parity), so one load answers "marked in this or the
// previous event"; event e sets parity e & 1 and the end of event e clears
// parity (e + 1) & 1 for reuse by event e + 1.
__host__ __device__ inline uint32_t hot_hash(uint32_t v, uint32_t bits) {
  return (v * 0x9E3779B1u) >> (32u - bits);
}

struct LatDev {
  Geo geo;
  uint64_t nv;
  uint32_t key0, key1;
  uint16_t *occ;
  uint64_t cap;        // per colour bin
  Bins bins[2];

  // first-order candidates for the next event: (colour, position, id) of
  // molecules whose first draw can fire some first-order reaction
  uint32_t *cand_pos[2];
  uint32_t *cand_id[2];
  uint8_t *cand_col[2];
  uint32_t *cand_count;   // [2]
  uint64_t cand_cap;

  // voxels where a collision put a product on the partner's voxel, by event
  // parity: the walk of event e appends to list e & 1; its end clears their
  // reacted flags and the hot marks of the previous event's list
  uint32_t *flag_vox[2];
  uint32_t *flag_count;   // [2]
  uint64_t flag_cap;

  // first-order newborns of one event: key = parent id << 31 | product
  // index << 27 | slot
  uint64_t *birth_key;
  uint32_t *birth_vox;
  uint16_t *birth_sp;
  uint32_t *birth_count;
  uint64_t birth_cap;

  // newborns of collision reactions with more than two products in the
  // running walk (null when no such reaction is registered): voxel, and key
  // (mover id << 32 | product index << 28 | slot); numbered and binned by
  // the end of the event in key order
  uint32_t *wb_vox;
  uint64_t *wb_key;
  uint32_t *wb_count;
  uint64_t wb_cap;

  // ranking of many newborns over the grid (null when no reaction has
  // newborns): bucket counts (zero between uses), their exclusive prefix
  // sums, and the keys dealt into bucket order
  uint32_t *rank_hist;    // [kRankBucketsMax]
  uint32_t *rank_off;     // [kRankBucketsMax + 1]
  uint64_t *rank_keys;    // [birth_cap]

  // stale-entry filter (see hot_hash)
  uint32_t *hot;          // [2^hot_bits / 16] words
  uint32_t hot_bits;      // log2 of the number of hash slots
  uint32_t *end_done;     // completion counter of the multi-block k_end

  // scratch of the first-order pass: molecules firing this event, and their
  // count (zero between events)
  uint32_t *fire_pos, *fire_id, *fire_vox;  // fire_vox: the firing molecule's voxel
  uint8_t *fire_col, *fire_rx;
  uint32_t *fire_count;

  // the last event's first-order fire list length, first-order newborn
  // count and collision newborn count: the host sizes later events'
  // launches from them
  uint32_t *recent;  // [kRecentN]

  // first-order conflict test: per hashed voxel, how many firing molecules
  // have it in their closed neighbourhood (zero between events)
  uint32_t *nbr_cnt;
  uint32_t nbr_bits;

  // model
  uint32_t n_species, n_rx, n_fo;  // n_fo: first-order slots (see fo_rx)
  const uint8_t *sp_flags;         // [64]
  const int16_t *pair_rx;          // [64 * 64] second-order reaction or -1
  const uint32_t *rx_thr;          // [n_rx] fire iff r1 < thr, unless always
  const uint8_t *rx_always;        // [n_rx]
  const uint8_t *rx_nprod;         // [n_rx]
  const uint16_t *rx_prod;         // [n_rx * 12]
  // the four tables above packed for the stage kernels' copies in LDS
  // (stage_tab_layout): rows 0..n_species of pair_rx, then rx_thr, rx_prod,
  // rx_nprod and rx_always
  const uint32_t *stage_tab;
  uint32_t stage_tab_words;
  const uint16_t *fo_first;        // [64] first slot of the species
  const uint8_t *fo_n;             // [64] slots of the species
  const uint16_t *fo_rx;           // [n_fo] reaction of each slot

  // event tape (host-computed): due species mask, cumulative first-order
  // thresholds per slot, and their maximum, for each event
  const uint64_t *tape_due;
  const uint32_t *tape_thr;        // [horizon * n_fo]
  const uint32_t *tape_cmax;
  uint64_t tape_horizon;

  // event state
  uint64_t stop_event;             // the lattice idles once ev reaches it
  uint64_t *ev;                    // events completed
  uint32_t ncol;                   // stage colours of the lattice (16)
  uint32_t *perm;                  // [kMaxColours] stage order of the running event
  uint4 *sdesc;                    // [kMaxColours] per stage: colour, count, event
                                   // (lo, hi); stages past ncol are empty
  uint32_t *next_id;
  // statistics, kStatRep replicas each (see kStatRep)
  unsigned long long *cnt;         // [kStatRep * kCntStride] attempts, hops, collisions,
                                   // placement failures
  unsigned long long *sp_count;    // [kStatRep * kSpStride] live molecules per species
                                   // (two's complement deltas)
  unsigned long long *fired;       // [kStatRep * fired_stride] firings per reaction
  uint32_t fired_stride;           // n_rx rounded up to a 128-byte line
  uint32_t *error;
};

hipError_t launch_scan(const LatDev *dL, int grid, hipStream_t s);
// disp: the lattice tracks displacements (its bins carry the planes)
// fcc: the lattice is face-centred cubic, else HCP;
// Launch shape of an event's first-order pass (workgroups; 0: none):
//   decide  the decisions in a launch of their own (events with many
//           candidates), else inside k_begin;
//   births  first-order newborns beyond what one workgroup ranks in LDS are
//           numbered by a launch of that many workgroups (events expecting
//           many), else by k_begin alone;
//   apply   more firings than k_begin has threads are applied by one
//           launch per stage of that many workgroups (events with a decision
//           launch), then numbered by the births launch (at least one
//           workgroup); fewer are applied inside k_begin.
struct BeginShape {
  int decide = 0, births = 0, apply = 0;
};
// fire-list entries an application workgroup scans per pass
constexpr uint32_t kFoTile = 2048;
// the last event's counts (LatDev::recent)
enum { kRecentFire = 0, kRecentFoBirths = 1, kRecentColBirths = 2, kRecentFlags = 3, kRecentN = 4 };
// most buckets of the grid-wide newborn ranking (their counts fit in LDS)
constexpr uint32_t kRankBucketsMax = 8192;
// births: the lattice (any member) has collision reactions with more than
// two products, whose newborns the event end numbers
hipError_t launch_event(const LatDev *dL, int grid, int items, bool disp, bool fcc,
                        const BeginShape &b, bool births, hipStream_t s);
// event e of a lattice launched from the host, which holds its record L
// (equal to *dL) and its tape: the stages take the record, their colour, the
// event, the species due in it (tape_due[e]) and the next event's largest
// first-order threshold (0 when none or past the tape) as arguments
// (k_stage_direct)
// open_with_end: the previous event's end was left to this launch, which runs
// it with this event's opening in one kernel (k_end_begin; only without
// collision births and for an opening with no launches of its own, else
// hipErrorInvalidValue); close: launch this event's end (else the next
// event's opening runs it)
hipError_t launch_event_direct(const LatDev *dL, const LatDev &L, uint64_t e, uint64_t due,
                               uint32_t cmax_next, int grid, int items, bool disp, bool fcc,
                               const BeginShape &b, bool births, bool births_defer,
                               hipStream_t s, bool open_with_end = false, bool close = true);
hipError_t launch_stage_direct(const LatDev &L, uint32_t c, uint64_t e, uint64_t due,
                               uint32_t cmax_next, int grid, int items, bool disp, bool fcc,
                               hipStream_t s);
// device bytes of an ensemble's member records: n records, then room for
// each stage's chunk prefix over the members (launch_event_multi writes it
// after R <= n records)
inline size_t member_records_bytes(uint32_t n) {
  return (size_t)n * sizeof(LatDev) + (size_t)kMaxColours * (n + 1) * sizeof(uint32_t);
}
// stages: the most stages of any member (16); lats: member_records_bytes(R)
// bytes or more
hipError_t launch_event_multi(const LatDev *lats, uint32_t R, uint32_t stages, int grid,
                              int items, bool births, hipStream_t s);
// desc: write the stage descriptors that the descriptor-form stage kernels
// read (the direct form does not need them); Lh, perm, e: the host's copy of
// the record, the event's stage order and the event, for the first-order
// stage launches to take as arguments (null: they read the device's)
hipError_t launch_begin(const LatDev *dL, const BeginShape &b, uint32_t stages, hipStream_t s,
                        bool desc = true, const LatDev *Lh = nullptr,
                        const uint32_t *perm = nullptr, uint64_t e = 0);
hipError_t launch_stage(const LatDev *dL, uint32_t g, int grid, int items, bool disp, bool fcc,
                        hipStream_t s);
// the stage kernels of one lattice kind (LAT: 0 HCP, 1 FCC) and the batched
// stage kernel of an ensemble, each in a translation unit of its own
template <int LAT>
hipError_t launch_stage_lat(const LatDev *dL, uint32_t g, int grid, int items, bool disp,
                            hipStream_t s);
template <int LAT>
hipError_t launch_stage_direct_lat(const LatDev &L, uint32_t c, uint64_t e, uint64_t due,
                                   uint32_t cmax_next, int grid, int items, bool disp,
                                   hipStream_t s);
hipError_t launch_stage_multi(const LatDev *lats, uint32_t R, uint32_t g, int grid, int items,
                              hipStream_t s);
// each stage's chunk prefix over the members, for the batched stage launches
// of the same chunk size
hipError_t launch_multi_prefix(const LatDev *lats, uint32_t R, uint32_t stages, int items,
                               hipStream_t s);
uint32_t max_members();
hipError_t launch_msd(const LatDev *dL, unsigned long long *out, hipStream_t s);
// occupancy between the linear (ABI) order and the lattice's layout
hipError_t launch_relayout(const Geo &g, uint64_t nv, const uint16_t *src, uint16_t *dst,
                           bool to_layout_order, hipStream_t s);
// births: the lattice has collision newborns to number; defer: more than
// one workgroup ranks in LDS go to a grid-wide numbering that follows
// (else the end's own workgroup numbers them all)
hipError_t launch_end(const LatDev *dL, bool births, hipStream_t s, bool defer = true);
int stage_items();
int stage_threads();

}  // namespace psc
