/*
 * psc_oracle.c -- plain CPU reference of the pSpatiocyte lattice walk.
 *
 * TEST INFRASTRUCTURE ONLY: linked by nothing in the product library.  See
 * psc_oracle.h for what it computes and which paper passages it follows.
 * Built with -ffp-contract=off so that its few FP64 expressions round the
 * same way as the product's host code.
 */
#include "psc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAX_SPECIES 64
#define MAX_RX 256
#define MAX_PROD 11
#define NO_SLOT 0xFFFFFFFFu

/* ========================================================================== */
/* Philox-4xW-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  One round maps the counter (x0,x1,x2,x3) with   */
/* key (k0,k1) to (hi(M1*x2)^x1^k0, lo(M1*x2), hi(M0*x0)^x3^k1, lo(M0*x0));   */
/* the key is bumped by the Weyl constants between rounds.                    */
/* ========================================================================== */
static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(M0, x0, &hi0, &lo0);
    mulhilo32(M1, x2, &hi1, &lo1);
    uint32_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, x0, &hi0, &lo0);
    mulhilo64(M1, x2, &hi1, &lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* the simulation's draws: key = seed, counter = (event, id, phase, block) */
static void draw4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t phase,
                  uint32_t block, uint32_t out[4]) {
  uint32_t ctr[4] = {c0, c1, phase, block};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32(ctr, key, out);
}

/* uniform integer in [0, m) from one 32-bit word: floor(r * m / 2^32) */
static uint32_t scale32(uint32_t r, uint32_t m) {
  return (uint32_t)(((uint64_t)r * (uint64_t)m) >> 32);
}

/* ========================================================================== */
/* Geometry (2.1, Fig. 3).  Voxel (i,j,k), v = i + ni*(j + nj*k).  With       */
/* s = (j+k)&1 and p = k&1 the voxel centre is                                */
/*   x = r (2i + s),  y = (r/sqrt3)(3j + p),  z = 2 sqrt(2/3) r k,            */
/* i.e. rows along i, rows shifted by half a voxel on alternate j (one zigzag */
/* axis) and layers shifted on alternate k (the other), stacked ABAB (HCP).   */
/* ========================================================================== */
static void ijk_of(uint32_t ni, uint32_t nj, uint32_t v, uint32_t *i, uint32_t *j,
                   uint32_t *k) {
  *i = v % ni;
  *j = (v / ni) % nj;
  *k = (v / ni) / nj;
}

static uint32_t v_of(uint32_t ni, uint32_t nj, uint32_t i, uint32_t j, uint32_t k) {
  return (uint32_t)((uint64_t)i + (uint64_t)ni * ((uint64_t)j + (uint64_t)nj * k));
}

/* The 12 neighbours, written as (di, dj, dk) in index space for parities s, p.
 * Row n of the table; derived from the voxel centres above so that every
 * neighbour lies at distance exactly 2r. */
/* FCC (ABC stacking, layer phase q = k mod 3, in-row offset s = (j+q)&1):
 * rows 0..5 as HCP; above: (s, a, +1), (s-1, a, +1), (0, c, +1) with
 * a = 0, c = -1 for q < 2 and a = +1, c = 0 for q = 2; below:
 * (s, b, -1), (s-1, b, -1), (0, d, -1) with b = 0, d = +1 for q > 0 and
 * b = -1, d = 0 for q = 0.  Derived from the positions below (the layer
 * above is shifted by t = (r, r/sqrt3) in the plane, the one below by -t). */
static void stencil_fcc(int n, uint32_t j, uint32_t k, int *di, int *dj, int *dk) {
  int q = (int)(k % 3u), s = (int)((j + (uint32_t)q) & 1u);
  int a = q < 2 ? 0 : 1, c = q < 2 ? -1 : 0;
  int b = q > 0 ? 0 : -1, d = q > 0 ? 1 : 0;
  switch (n) {
  case 0: *di = 1;     *dj = 0;  *dk = 0;  break;
  case 1: *di = -1;    *dj = 0;  *dk = 0;  break;
  case 2: *di = s;     *dj = 1;  *dk = 0;  break;
  case 3: *di = s - 1; *dj = 1;  *dk = 0;  break;
  case 4: *di = s;     *dj = -1; *dk = 0;  break;
  case 5: *di = s - 1; *dj = -1; *dk = 0;  break;
  case 6: *di = s;     *dj = a;  *dk = 1;  break;
  case 7: *di = s - 1; *dj = a;  *dk = 1;  break;
  case 8: *di = 0;     *dj = c;  *dk = 1;  break;
  case 9: *di = s;     *dj = b;  *dk = -1; break;
  case 10: *di = s - 1; *dj = b; *dk = -1; break;
  default: *di = 0;    *dj = d;  *dk = -1; break;
  }
}

static void stencil(int n, int s, int p, int *di, int *dj, int *dk) {
  switch (n) {
  case 0: *di = 1;     *dj = 0;         *dk = 0;  break;
  case 1: *di = -1;    *dj = 0;         *dk = 0;  break;
  case 2: *di = s;     *dj = 1;         *dk = 0;  break;
  case 3: *di = s - 1; *dj = 1;         *dk = 0;  break;
  case 4: *di = s;     *dj = -1;        *dk = 0;  break;
  case 5: *di = s - 1; *dj = -1;        *dk = 0;  break;
  case 6: *di = s;     *dj = 0;         *dk = 1;  break;
  case 7: *di = s - 1; *dj = 0;         *dk = 1;  break;
  case 8: *di = 0;     *dj = 2 * p - 1; *dk = 1;  break;
  case 9: *di = s;     *dj = 0;         *dk = -1; break;
  case 10: *di = s - 1; *dj = 0;        *dk = -1; break;
  default: *di = 0;    *dj = 2 * p - 1; *dk = -1; break;
  }
}

/* Displacement of hop n in integer units: X in r, Y in r/sqrt3, Z in
 * 2 sqrt(2/3) r.  |hop|^2 = r^2 (X^2 + Y^2/3 + 8 Z^2/3) = 4 r^2. */
static void hopvec(int n, int p, int32_t *X, int32_t *Y, int32_t *Z) {
  static const int32_t tx[12] = {2, -2, 1, -1, 1, -1, 1, -1, 0, 1, -1, 0};
  static const int32_t tz[12] = {0, 0, 0, 0, 0, 0, 1, 1, 1, -1, -1, -1};
  int32_t ty;
  if (n == 0 || n == 1) ty = 0;
  else if (n == 2 || n == 3) ty = 3;
  else if (n == 4 || n == 5) ty = -3;
  else if (n == 8 || n == 11) ty = 4 * p - 2;
  else ty = 1 - 2 * p;
  *X = tx[n];
  *Y = ty;
  *Z = tz[n];
}

static uint32_t wrap(int64_t x, uint32_t n) {
  int64_t m = x % (int64_t)n;
  if (m < 0) m += n;
  return (uint32_t)m;
}

/* Neighbour n of v for either lattice and boundary: periodic boxes wrap, a
 * box closed by walls has no neighbour beyond a face (ORC_OUTSIDE) -- the
 * space there is another compartment. */
uint32_t orc_neighbour_l(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, int n,
                         int lattice, int boundary) {
  uint32_t i, j, k;
  int di, dj, dk;
  ijk_of(ni, nj, v, &i, &j, &k);
  if (lattice == ORC_LATTICE_FCC) stencil_fcc(n, j, k, &di, &dj, &dk);
  else stencil(n, (int)((j + k) & 1u), (int)(k & 1u), &di, &dj, &dk);
  int64_t a = (int64_t)i + di, b = (int64_t)j + dj, c = (int64_t)k + dk;
  if (boundary == ORC_BOUNDARY_REFLECT) {
    if (a < 0 || b < 0 || c < 0 || a >= ni || b >= nj || c >= nk) return ORC_OUTSIDE;
    return v_of(ni, nj, (uint32_t)a, (uint32_t)b, (uint32_t)c);
  }
  return v_of(ni, nj, wrap(a, ni), wrap(b, nj), wrap(c, nk));
}

uint32_t orc_neighbour(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, int n) {
  return orc_neighbour_l(ni, nj, nk, v, n, ORC_LATTICE_HCP, ORC_BOUNDARY_PERIODIC);
}

uint32_t orc_neighbour_b(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, int n,
                         int boundary) {
  return orc_neighbour_l(ni, nj, nk, v, n, ORC_LATTICE_HCP, boundary);
}

void orc_neighbour_table_l(uint32_t ni, uint32_t nj, uint32_t nk, int lattice, int boundary,
                           uint32_t *out) {
  uint64_t nv = (uint64_t)ni * nj * nk;
  for (uint64_t v = 0; v < nv; v++)
    for (int n = 0; n < 12; n++)
      out[12 * v + n] = orc_neighbour_l(ni, nj, nk, (uint32_t)v, n, lattice, boundary);
}

void orc_neighbour_table(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t *out) {
  uint64_t nv = (uint64_t)ni * nj * nk;
  for (uint64_t v = 0; v < nv; v++)
    for (int n = 0; n < 12; n++) out[12 * v + n] = orc_neighbour(ni, nj, nk, (uint32_t)v, n);
}

/* FCC hop n in the same units (r, r/sqrt3, 2 sqrt(2/3) r); the layer phase
 * does not enter: FCC is a Bravais lattice */
static void hopvec_fcc(int n, int32_t *X, int32_t *Y, int32_t *Z) {
  static const int32_t tx[12] = {2, -2, 1, -1, 1, -1, 1, -1, 0, 1, -1, 0};
  static const int32_t ty[12] = {0, 0, 3, 3, -3, -3, 1, 1, -2, -1, -1, 2};
  static const int32_t tz[12] = {0, 0, 0, 0, 0, 0, 1, 1, 1, -1, -1, -1};
  *X = tx[n];
  *Y = ty[n];
  *Z = tz[n];
}

void orc_hop_vector_l(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, int n, int lattice,
                      int32_t out[3]) {
  uint32_t i, j, k;
  (void)nk;
  ijk_of(ni, nj, v, &i, &j, &k);
  if (lattice == ORC_LATTICE_FCC) hopvec_fcc(n, &out[0], &out[1], &out[2]);
  else hopvec(n, (int)(k & 1u), &out[0], &out[1], &out[2]);
}

void orc_hop_vector(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, int n,
                    int32_t out[3]) {
  orc_hop_vector_l(ni, nj, nk, v, n, ORC_LATTICE_HCP, out);
}

/* HCP: x = r(2i + s), y = (r/sqrt3)(3j + p), z = 2 sqrt(2/3) r k with
 * s = (j+k)&1, p = k&1 (ABAB).  FCC: the same with p -> q = k mod 3 and
 * s = (j+q)&1 (ABC: layer q shifted by q (r, r/sqrt3), reduced into the box). */
void orc_position_l(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, double rv, int lattice,
                    double out[3]) {
  uint32_t i, j, k;
  (void)nk;
  ijk_of(ni, nj, v, &i, &j, &k);
  uint32_t p = lattice == ORC_LATTICE_FCC ? k % 3u : (k & 1u);
  double s = (double)((j + p) & 1u);
  out[0] = rv * (2.0 * i + s);
  out[1] = rv / sqrt(3.0) * (3.0 * j + (double)p);
  out[2] = 2.0 * sqrt(2.0 / 3.0) * rv * k;
}

void orc_position(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, double rv,
                  double out[3]) {
  orc_position_l(ni, nj, nk, v, rv, ORC_LATTICE_HCP, out);
}

/* stage colour: voxels of one colour are >= 3 hops apart.  HCP (16):
 * 8(k&1) + 4(j&1) + ((i - j + k) mod 4).  FCC (16): a linear form on the
 * lattice's own (Bravais) coordinates a = i - floor((j+q)/2) - floor(k/3),
 * b = j - floor(k/3), k with q = k mod 3: (2a + 3b + 7k) mod 16, periodic
 * when ni and nj are multiples of 8 (found by search, checked by the tests
 * on the neighbour graph). */
int orc_colour_l(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, int lattice) {
  uint32_t i, j, k;
  (void)nk;
  ijk_of(ni, nj, v, &i, &j, &k);
  if (lattice == ORC_LATTICE_FCC) {
    int64_t q = k % 3u, a = (int64_t)i - ((int64_t)j + q) / 2 - (int64_t)(k / 3u);
    int64_t b = (int64_t)j - (int64_t)(k / 3u);
    int64_t c = (2 * a + 3 * b + 7 * (int64_t)k) % 16;
    return (int)(c < 0 ? c + 16 : c);
  }
  int64_t m = ((int64_t)i - (int64_t)j + (int64_t)k) % 4;
  if (m < 0) m += 4;
  return (int)(8 * (k & 1u) + 4 * (j & 1u) + (uint32_t)m);
}

int orc_colour(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v) {
  return orc_colour_l(ni, nj, nk, v, ORC_LATTICE_HCP);
}

int orc_n_colours(int lattice) { (void)lattice; return 16; }

/* stage order of an event: Fisher-Yates over n colours, slot i = n-1..1
 * swapping with j = floor(w (i + 1) / 2^32), words from blocks 0, 1, ... of
 * Philox(seed; event, 0xFFFFFFFF, PHASE_STAGE) */
void orc_stage_order_n(uint64_t seed, uint64_t event, int n, uint8_t *out) {
  uint32_t words[ORC_MAX_COLOURS];
  for (int b = 0; 4 * b < n; b++)
    draw4(seed, (uint32_t)event, 0xFFFFFFFFu, ORC_PHASE_STAGE, (uint32_t)b, &words[4 * b]);
  for (int c = 0; c < n; c++) out[c] = (uint8_t)c;
  int w = 0;
  for (int i = n - 1; i >= 1; i--) {
    uint32_t j = scale32(words[w++], (uint32_t)(i + 1));
    uint8_t t = out[i];
    out[i] = out[j];
    out[j] = t;
  }
}

void orc_stage_order(uint64_t seed, uint64_t event, uint8_t out[16]) {
  orc_stage_order_n(seed, event, 16, out);
}

/* probability -> 32-bit threshold: an event of probability p happens iff a
 * uniform 32-bit word r satisfies r < floor(p 2^32) (capped at 2^32 - 1). */
uint32_t orc_prob_to_u32(double p) {
  if (!(p > 0.0)) return 0u;
  double x = p * 4294967296.0;
  if (x >= 4294967295.0) return 0xFFFFFFFFu;
  return (uint32_t)floor(x);
}

/* Second-order reaction probability on collision, eq. (6) of 2.4.2:
 * p = k / (6 sqrt2 (DA + DB) r).  Returned as a 33-bit threshold T:
 * the reaction fires iff r1 < T; p >= 1 gives T = 2^32 (always). */
uint64_t orc_second_order_threshold(double k, double DA, double DB, double rv) {
  double den = 6.0 * sqrt(2.0);
  den = den * (DA + DB);
  den = den * rv;
  double p = k / den;
  if (p >= 1.0) return 4294967296ull;
  if (!(p > 0.0)) return 0ull;
  return (uint64_t)floor(p * 4294967296.0);
}

/* interval between diffusion events, eq. (2) of 2.3: tau = 2 r^2 / (3 D) */
double orc_tau(double rv, double D) {
  double num = 2.0 * rv;
  num = num * rv;
  double den = 3.0 * D;
  return num / den;
}

/* ========================================================================== */
/* Simulation state                                                           */
/* ========================================================================== */
typedef struct {
  int n_reac, n_prod;
  uint16_t reac[2];
  uint16_t prod[MAX_PROD];
  double k;
  uint64_t thr2; /* second order: 33-bit threshold */
} orc_rx;

struct orc_sim {
  uint32_t ni, nj, nk;
  uint64_t nv;
  int boundary;       /* ORC_BOUNDARY_PERIODIC or ORC_BOUNDARY_REFLECT */
  int lattice;        /* ORC_LATTICE_HCP or ORC_LATTICE_FCC */
  int n_col;          /* stage colours: 16 (HCP) or 24 (FCC) */
  double rv;
  uint64_t seed;

  int n_species;                    /* ids 1..n_species */
  double D[MAX_SPECIES];
  double tau[MAX_SPECIES];
  uint64_t n_walks[MAX_SPECIES];    /* diffusion events done per species */

  int n_rx;
  orc_rx rx[MAX_RX];
  int pair_rx[MAX_SPECIES][MAX_SPECIES]; /* second-order reaction id or -1 */
  int n_first[MAX_SPECIES];              /* first-order reactions per species */
  int first_rx[MAX_SPECIES][MAX_RX];     /* their ids, in registration order */
  int frozen;

  uint16_t *occ;      /* nv: species id, 0 = vacant */
  uint8_t *comp;      /* nv: compartment of each voxel, or NULL (all 0) */
  uint32_t *slot_at;  /* nv: molecule slot at voxel (valid where occ != 0) */

  /* molecule table, one slot per molecule ever made, ascending id */
  uint64_t n_slots, cap;
  uint32_t *id, *vox;
  uint16_t *sp;
  uint8_t *alive;
  int64_t *dx, *dy, *dz;
  uint64_t n_alive;

  uint64_t count[MAX_SPECIES];   /* live molecules per species */

  uint32_t next_id;
  uint64_t event;
  double t;
  uint64_t place_calls;

  uint64_t cnt[ORC_CNT_N];
  uint64_t fired[MAX_RX];

  /* products beyond the second of collision reactions in the running walk:
   * their slots sit at the end of the table from walk_slot0 on, with ids
   * assigned when the walk ends; pend_key[q] orders slot walk_slot0 + q */
  uint64_t walk_slot0;
  uint64_t *pend_key;
  uint64_t pend_cap;
  int oom;            /* an allocation failed during a walk */
};

static int grow_slots(orc_sim *s, uint64_t need) {
  if (need <= s->cap) return 0;
  uint64_t c = s->cap ? s->cap : 1024;
  while (c < need) c *= 2;
  uint32_t *id = realloc(s->id, c * sizeof *id);
  if (!id) return -1;
  s->id = id;
  uint32_t *vox = realloc(s->vox, c * sizeof *vox);
  if (!vox) return -1;
  s->vox = vox;
  uint16_t *sp = realloc(s->sp, c * sizeof *sp);
  if (!sp) return -1;
  s->sp = sp;
  uint8_t *al = realloc(s->alive, c * sizeof *al);
  if (!al) return -1;
  s->alive = al;
  int64_t *a = realloc(s->dx, c * sizeof *a);
  if (!a) return -1;
  s->dx = a;
  a = realloc(s->dy, c * sizeof *a);
  if (!a) return -1;
  s->dy = a;
  a = realloc(s->dz, c * sizeof *a);
  if (!a) return -1;
  s->dz = a;
  s->cap = c;
  return 0;
}

/* new molecule at voxel v (occupancy written by the caller) */
static int mol_new(orc_sim *s, uint32_t id, uint32_t v, uint16_t species) {
  if (grow_slots(s, s->n_slots + 1)) return -1;
  uint32_t slot = (uint32_t)s->n_slots++;
  s->id[slot] = id;
  s->vox[slot] = v;
  s->sp[slot] = species;
  s->alive[slot] = 1;
  s->dx[slot] = s->dy[slot] = s->dz[slot] = 0;
  s->slot_at[v] = slot;
  s->n_alive++;
  s->count[species]++;
  return 0;
}

static void mol_set_species(orc_sim *s, uint32_t slot, uint16_t species) {
  s->count[s->sp[slot]]--;
  s->sp[slot] = species;
  s->count[species]++;
}

static void mol_kill(orc_sim *s, uint32_t slot) {
  s->count[s->sp[slot]]--;
  s->alive[slot] = 0;
  s->n_alive--;
}

/* drop dead slots once they dominate (keeps ascending-id order) */
static void compact(orc_sim *s) {
  if (s->n_slots - s->n_alive < s->n_slots / 2 + 1024) return;
  uint64_t w = 0;
  for (uint64_t r = 0; r < s->n_slots; r++) {
    if (!s->alive[r]) continue;
    s->id[w] = s->id[r];
    s->vox[w] = s->vox[r];
    s->sp[w] = s->sp[r];
    s->alive[w] = 1;
    s->dx[w] = s->dx[r];
    s->dy[w] = s->dy[r];
    s->dz[w] = s->dz[r];
    w++;
  }
  s->n_slots = w;
  for (uint64_t q = 0; q < w; q++) s->slot_at[s->vox[q]] = (uint32_t)q;
}

orc_sim *orc_create(uint32_t ni, uint32_t nj, uint32_t nk, double rv, uint64_t seed) {
  if (ni < 4 || nj < 4 || nk < 4 || ni % 4 || nj % 4 || nk % 4) return NULL;
  uint64_t nv = (uint64_t)ni * nj * nk;
  if (nv > 4294967296ull) return NULL;
  orc_sim *s = calloc(1, sizeof *s);
  if (!s) return NULL;
  s->ni = ni; s->nj = nj; s->nk = nk; s->nv = nv;
  s->rv = rv;
  s->seed = seed;
  s->occ = calloc(nv, sizeof *s->occ);
  s->slot_at = malloc(nv * sizeof *s->slot_at);
  if (!s->occ || !s->slot_at) {
    orc_destroy(s);
    return NULL;
  }
  for (int a = 0; a < MAX_SPECIES; a++)
    for (int b = 0; b < MAX_SPECIES; b++) s->pair_rx[a][b] = -1;
  s->n_col = 16;
  return s;
}

void orc_destroy(orc_sim *s) {
  if (!s) return;
  free(s->pend_key);
  free(s->occ); free(s->slot_at); free(s->comp);
  free(s->id); free(s->vox); free(s->sp); free(s->alive);
  free(s->dx); free(s->dy); free(s->dz);
  free(s);
}

int orc_set_lattice(orc_sim *s, int lattice) {
  if (lattice != ORC_LATTICE_HCP && lattice != ORC_LATTICE_FCC) return -1;
  /* stacking and colour periods */
  if (lattice == ORC_LATTICE_FCC && (s->nk % 12 || s->ni % 8 || s->nj % 8)) return -1;
  s->lattice = lattice;
  s->n_col = orc_n_colours(lattice);
  return 0;
}

/* Compartments (2): every voxel belongs to one group of voxels, given by the
 * caller; molecules never leave the compartment of their voxel (2.3) */
int orc_set_compartments(orc_sim *s, const uint8_t *comp) {
  if (!s->comp) s->comp = malloc(s->nv);
  if (!s->comp) return -1;
  memcpy(s->comp, comp, s->nv);
  return 0;
}

static uint8_t comp_at(const orc_sim *s, uint32_t v) { return s->comp ? s->comp[v] : 0; }

int orc_set_boundary(orc_sim *s, int boundary) {
  if (boundary != ORC_BOUNDARY_PERIODIC && boundary != ORC_BOUNDARY_REFLECT) return -1;
  s->boundary = boundary;
  return 0;
}

int orc_add_species(orc_sim *s, double D) {
  if (s->frozen || !(D >= 0.0) || s->n_species + 1 >= MAX_SPECIES) return -1;
  int id = ++s->n_species;
  s->D[id] = D;
  s->tau[id] = D > 0.0 ? orc_tau(s->rv, D) : 0.0;
  return id;
}

int orc_add_reaction(orc_sim *s, int n_reac, const uint16_t *reac, int n_prod,
                     const uint16_t *prod, double k) {
  if (s->frozen || s->n_rx >= MAX_RX || !(k >= 0.0)) return -1;
  if (n_reac < 1 || n_reac > 2) return -1;
  for (int a = 0; a < n_reac; a++)
    if (reac[a] < 1 || reac[a] > s->n_species) return -1;
  for (int a = 0; a < n_prod; a++)
    if (prod[a] < 1 || prod[a] > s->n_species) return -1;
  if (n_reac == 1 && (n_prod < 0 || n_prod > MAX_PROD)) return -1;
  if (n_reac == 2 && (n_prod < 1 || n_prod > MAX_PROD)) return -1;
  orc_rx *r = &s->rx[s->n_rx];
  r->n_reac = n_reac;
  r->n_prod = n_prod;
  for (int a = 0; a < n_reac; a++) r->reac[a] = reac[a];
  for (int a = 0; a < n_prod; a++) r->prod[a] = prod[a];
  r->k = k;
  if (n_reac == 2) {
    uint16_t A = reac[0], B = reac[1];
    if (s->pair_rx[A][B] >= 0) return -1;
    if (!(s->D[A] + s->D[B] > 0.0)) return -1;
    r->thr2 = orc_second_order_threshold(k, s->D[A], s->D[B], s->rv);
    s->pair_rx[A][B] = s->pair_rx[B][A] = s->n_rx;
  } else {
    s->first_rx[reac[0]][s->n_first[reac[0]]++] = s->n_rx;
  }
  return s->n_rx++;
}

/* Uniform initial placement (the homogeneous start of 3.4): attempt a of
 * the c-th placement call draws v = floor(r0 * nv / 2^32) from
 * Philox(seed; c, a, PHASE_PLACE, 0) and takes it if vacant. */
int orc_place_uniform(orc_sim *s, uint16_t species, uint64_t count) {
  if (species < 1 || species > s->n_species) return -1;
  uint64_t vacant = s->nv - s->n_alive;
  if (count > vacant) return -1;
  if ((uint64_t)s->next_id + count >= 0xFFFFFFFFull) return -1;
  uint32_t call = (uint32_t)s->place_calls;
  uint64_t attempt = 0;
  for (uint64_t q = 0; q < count; q++) {
    for (;;) {
      uint32_t r[4];
      draw4(s->seed, call, (uint32_t)attempt, ORC_PHASE_PLACE, 0, r);
      attempt++;
      uint32_t v = (uint32_t)(((uint64_t)r[0] * s->nv) >> 32);
      if (s->occ[v] == 0) {
        s->occ[v] = species;
        if (mol_new(s, s->next_id++, v, species)) return -1;
        break;
      }
    }
  }
  s->place_calls++;
  return 0;
}

/* The same placement restricted to compartment c: attempt a of the call is
 * taken if its voxel is vacant and belongs to c. */
int orc_place_uniform_in(orc_sim *s, uint16_t species, uint64_t count, int c) {
  if (species < 1 || species > s->n_species) return -1;
  uint64_t vacant = 0;
  for (uint64_t v = 0; v < s->nv; v++) vacant += s->occ[v] == 0 && comp_at(s, (uint32_t)v) == c;
  if (count > vacant) return -1;
  if ((uint64_t)s->next_id + count >= 0xFFFFFFFFull) return -1;
  uint32_t call = (uint32_t)s->place_calls;
  uint64_t attempt = 0;
  for (uint64_t q = 0; q < count; q++) {
    for (;;) {
      uint32_t r[4];
      draw4(s->seed, call, (uint32_t)attempt, ORC_PHASE_PLACE, 0, r);
      attempt++;
      uint32_t v = (uint32_t)(((uint64_t)r[0] * s->nv) >> 32);
      if (s->occ[v] == 0 && comp_at(s, v) == c) {
        s->occ[v] = species;
        if (mol_new(s, s->next_id++, v, species)) return -1;
        break;
      }
    }
  }
  s->place_calls++;
  return 0;
}

/* advances the diffusion-event clock: t_e = min over mobile species of
 * (n_s + 1) tau_s, due = the species attaining it (2.2, 2.3) */
static int next_event(orc_sim *s, double *t_e, uint8_t due[MAX_SPECIES]) {
  double tmin = INFINITY;
  for (int a = 1; a <= s->n_species; a++) {
    if (!(s->D[a] > 0.0)) continue;
    double ta = (double)(s->n_walks[a] + 1) * s->tau[a];
    if (ta < tmin) tmin = ta;
  }
  if (tmin == INFINITY) return -1;
  for (int a = 0; a < MAX_SPECIES; a++) due[a] = 0;
  for (int a = 1; a <= s->n_species; a++) {
    if (!(s->D[a] > 0.0)) continue;
    if ((double)(s->n_walks[a] + 1) * s->tau[a] == tmin) due[a] = 1;
  }
  *t_e = tmin;
  return 0;
}

int orc_load(orc_sim *s, const uint16_t *occ, uint64_t n_mol, const uint32_t *id,
             const uint32_t *vox, const int32_t *dx, const int32_t *dy,
             const int32_t *dz, uint64_t event, uint32_t next_id) {
  /* validate: ids strictly ascending and < next_id, occupancy consistent */
  uint64_t occupied = 0;
  for (uint64_t v = 0; v < s->nv; v++) {
    if (occ[v] > s->n_species) return -1;
    if (occ[v]) occupied++;
  }
  if (occupied != n_mol) return -1;
  for (uint64_t q = 0; q < n_mol; q++) {
    if (q && id[q] <= id[q - 1]) return -1;
    if (id[q] >= next_id || next_id == 0xFFFFFFFFu) return -1;
    if (vox[q] >= s->nv || occ[vox[q]] == 0) return -1;
  }
  memcpy(s->occ, occ, s->nv * sizeof *occ);
  s->n_slots = 0;
  s->n_alive = 0;
  for (int a = 0; a < MAX_SPECIES; a++) s->count[a] = 0;
  for (uint64_t v = 0; v < s->nv; v++) s->slot_at[v] = NO_SLOT;
  for (uint64_t q = 0; q < n_mol; q++) {
    if (s->slot_at[vox[q]] != NO_SLOT) return -1; /* two molecules, one voxel */
    if (mol_new(s, id[q], vox[q], occ[vox[q]])) return -1;
    s->dx[q] = dx ? dx[q] : 0;
    s->dy[q] = dy ? dy[q] : 0;
    s->dz[q] = dz ? dz[q] : 0;
  }
  s->next_id = next_id;
  /* replay the event clock up to `event` */
  for (int a = 0; a < MAX_SPECIES; a++) s->n_walks[a] = 0;
  s->t = 0.0;
  s->event = 0;
  for (uint64_t e = 0; e < event; e++) {
    double te;
    uint8_t due[MAX_SPECIES];
    if (next_event(s, &te, due)) return -1;
    for (int a = 1; a <= s->n_species; a++)
      if (due[a]) s->n_walks[a]++;
    s->t = te;
  }
  s->event = event;
  return 0;
}

/* ---- product placement shared by both first-order laws ------------------- */
/* Extra products (2nd, 3rd, ...) go to distinct vacant neighbours of v in
 * v's compartment; the
 * vacant neighbours are listed in stencil order and each product takes
 * entry floor(w * count / 2^32) of the remaining list, w taken in sequence
 * from `words` (2.4.1: extra products need vacant neighbours).  Returns -1
 * (and changes nothing) when too few are vacant. */
static int pick_vacant(const orc_sim *s, uint32_t v, int n_extra,
                       const uint32_t *words, uint32_t *out) {
  uint32_t cand[12];
  int nc = 0;
  for (int n = 0; n < 12; n++) {
    uint32_t t = orc_neighbour_l(s->ni, s->nj, s->nk, v, n, s->lattice, s->boundary);
    if (t != ORC_OUTSIDE && comp_at(s, t) == comp_at(s, v) && s->occ[t] == 0) cand[nc++] = t;
  }
  if (nc < n_extra) return -1;
  for (int q = 0; q < n_extra; q++) {
    uint32_t x = scale32(words[q], (uint32_t)nc);
    out[q] = cand[x];
    for (int y = (int)x; y + 1 < nc; y++) cand[y] = cand[y + 1];
    nc--;
  }
  return 0;
}

typedef struct {
  uint32_t parent;
  int order;
  uint32_t vox;
  uint16_t species;
} birth;

static int birth_cmp(const void *a, const void *b) {
  const birth *x = a, *y = b;
  if (x->parent != y->parent) return x->parent < y->parent ? -1 : 1;
  return x->order - y->order;
}

/* per-species cumulative first-order thresholds for interval dt (2.4.1):
 * q = 1 - exp(-K dt) is the chance that one molecule reacts at all
 * (K = sum of its first-order rate constants; eq. 4 with a0 = K for one
 * molecule), reaction j is chosen with weight k_j / K (eq. 5). */
static void first_thresholds(const orc_sim *s, int species, double dt, uint32_t *C) {
  double K = 0.0;
  for (int a = 0; a < s->n_first[species]; a++) K += s->rx[s->first_rx[species][a]].k;
  double q = -expm1(-K * dt);
  double acc = 0.0;
  for (int a = 0; a < s->n_first[species]; a++) {
    double kj = s->rx[s->first_rx[species][a]].k;
    acc = acc + q * kj / K;
    C[a] = orc_prob_to_u32(acc);
  }
}

/* fires first-order reaction `r` on molecule `slot`, drawing placement words
 * from `words`; newborns are recorded for id assignment (mode C) or given
 * ids at once (assign_now, mode S).  Returns 1 if fired, 0 if it failed. */
static int fire_first(orc_sim *s, uint32_t slot, int r, const uint32_t *words,
                      birth *births, uint64_t *n_births, int assign_now) {
  const orc_rx *x = &s->rx[r];
  uint32_t v = s->vox[slot];
  if (x->n_prod == 0) {
    s->occ[v] = 0;
    mol_kill(s, slot);
    s->fired[r]++;
    return 1;
  }
  uint32_t dest[MAX_PROD];
  if (x->n_prod > 1 && pick_vacant(s, v, x->n_prod - 1, words, dest)) {
    s->cnt[ORC_CNT_PLACE_FAIL]++;
    return 0;
  }
  s->occ[v] = x->prod[0];
  mol_set_species(s, slot, x->prod[0]);
  for (int q = 1; q < x->n_prod; q++) {
    s->occ[dest[q - 1]] = x->prod[q];
    if (assign_now) {
      mol_new(s, s->next_id++, dest[q - 1], x->prod[q]);
    } else {
      birth b = {s->id[slot], q, dest[q - 1], x->prod[q]};
      births[(*n_births)++] = b;
    }
  }
  s->fired[r]++;
  return 1;
}

/* placement words for a first-order firing: words 1..3 of block 0, then the
 * four words of blocks 1, 2, ... of the same counter */
static void placement_words(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t phase,
                            const uint32_t first[4], uint32_t *words) {
  words[0] = first[1];
  words[1] = first[2];
  words[2] = first[3];
  for (uint32_t b = 1; b <= 3; b++) draw4(seed, c0, c1, phase, b, &words[3 + 4 * (b - 1)]);
}

/* molecules bucketed by the colour of their voxel, ascending slot (= id)
 * inside each bucket; `want` selects species */
typedef struct {
  uint32_t *slots;
  uint64_t start[ORC_MAX_COLOURS + 1];
} buckets;

static int bucket_by_colour(const orc_sim *s, const uint8_t *want, buckets *b) {
  uint64_t count[ORC_MAX_COLOURS] = {0};
  const int nc = s->n_col;
  for (uint64_t q = 0; q < s->n_slots; q++)
    if (s->alive[q] && want[s->sp[q]])
      count[orc_colour_l(s->ni, s->nj, s->nk, s->vox[q], s->lattice)]++;
  b->start[0] = 0;
  for (int c = 0; c < nc; c++) b->start[c + 1] = b->start[c] + count[c];
  b->slots = malloc((b->start[nc] + 1) * sizeof *b->slots);
  if (!b->slots) return -1;
  uint64_t fill[ORC_MAX_COLOURS];
  for (int c = 0; c < nc; c++) fill[c] = b->start[c];
  for (uint64_t q = 0; q < s->n_slots; q++)
    if (s->alive[q] && want[s->sp[q]])
      b->slots[fill[orc_colour_l(s->ni, s->nj, s->nk, s->vox[q], s->lattice)]++] = (uint32_t)q;
  return 0;
}

/* ---- first-order pass, per-molecule law in stage order (mode C) ---------- */
static int first_order_coloured(orc_sim *s, double dt, const uint8_t *order,
                                int reverse) {
  uint8_t want[MAX_SPECIES] = {0};
  int any = 0;
  for (int a = 1; a <= s->n_species; a++)
    if (s->n_first[a]) want[a] = 1, any = 1;
  if (!any) return 0;
  uint32_t C[MAX_SPECIES][MAX_RX];
  for (int a = 1; a <= s->n_species; a++)
    if (s->n_first[a]) first_thresholds(s, a, dt, C[a]);
  buckets b;
  if (bucket_by_colour(s, want, &b)) return -1;
  uint64_t n_part = b.start[s->n_col];
  birth *births = malloc((n_part * MAX_PROD + 1) * sizeof *births);
  if (!births) { free(b.slots); return -1; }
  uint64_t n_births = 0;
  for (int g = 0; g < s->n_col; g++) {
    int c = order[g];
    uint64_t lo = b.start[c], hi = b.start[c + 1];
    for (uint64_t z = 0; z < hi - lo; z++) {
      uint32_t slot = b.slots[reverse ? hi - 1 - z : lo + z];
      uint16_t A = s->sp[slot];
      uint32_t r[4];
      draw4(s->seed, (uint32_t)s->event, s->id[slot], ORC_PHASE_FIRST, 0, r);
      int chosen = -1;
      for (int a = 0; a < s->n_first[A]; a++)
        if (r[0] < C[A][a]) { chosen = s->first_rx[A][a]; break; }
      if (chosen < 0) continue;
      uint32_t words[16];
      placement_words(s->seed, (uint32_t)s->event, s->id[slot], ORC_PHASE_FIRST, r, words);
      fire_first(s, slot, chosen, words, births, &n_births, 0);
    }
  }
  /* newborns take consecutive ids in ascending parent id, then product order */
  qsort(births, n_births, sizeof *births, birth_cmp);
  for (uint64_t q = 0; q < n_births; q++)
    if (mol_new(s, s->next_id++, births[q].vox, births[q].species)) {
      free(births); free(b.slots);
      return -1;
    }
  free(births);
  free(b.slots);
  return 0;
}

/* ---- first-order pass, Gillespie direct method over dt (mode S) ---------- */
static int first_order_ssa(orc_sim *s, double dt) {
  int any = 0;
  for (int a = 1; a <= s->n_species; a++)
    if (s->n_first[a]) any = 1;
  if (!any) return 0;
  double tl = 0.0;
  for (uint32_t d = 0;; d++) {
    /* propensities with molecule counts, a_j = k_j N_j (2.4.1, eq. 3) */
    double a0 = 0.0;
    double aj[MAX_RX];
    int ids[MAX_RX], m = 0;
    for (int r = 0; r < s->n_rx; r++) {
      if (s->rx[r].n_reac != 1) continue;
      aj[m] = s->rx[r].k * (double)s->count[s->rx[r].reac[0]];
      ids[m] = r;
      a0 += aj[m];
      m++;
    }
    if (!(a0 > 0.0)) break;
    uint32_t w[4];
    draw4(s->seed, (uint32_t)s->event, d, ORC_PHASE_SSA, 0, w);
    double u1 = ((double)w[0] + 1.0) / 4294967296.0;
    tl += -log(u1) / a0;
    if (tl > dt) break;
    /* reaction u with sum_{i<u} a_i < a0 R <= sum_{i<=u} a_i (eq. 5) */
    double target = a0 * (((double)w[1] + 1.0) / 4294967296.0);
    double cum = 0.0;
    int u = ids[m - 1];
    for (int z = 0; z < m; z++) {
      cum += aj[z];
      if (target <= cum) { u = ids[z]; break; }
    }
    /* the reactant: uniform among species A's molecules, counted in
     * ascending id */
    uint16_t A = s->rx[u].reac[0];
    if (s->count[A] == 0) continue;
    uint64_t pick = scale32(w[2], (uint32_t)s->count[A]);
    uint32_t slot = 0;
    for (uint64_t q = 0, seen = 0; q < s->n_slots; q++) {
      if (!s->alive[q] || s->sp[q] != A) continue;
      if (seen++ == pick) { slot = (uint32_t)q; break; }
    }
    /* placement words: w[3], then blocks 1, 2, 3 of this draw counter */
    uint32_t words[16];
    words[0] = w[3];
    for (uint32_t blk = 1; blk <= 3; blk++)
      draw4(s->seed, (uint32_t)s->event, d, ORC_PHASE_SSA, blk, &words[1 + 4 * (blk - 1)]);
    fire_first(s, slot, u, words, NULL, NULL, 1);
  }
  return 0;
}

/* words for placing collision products: r2, r3 of the walk draw of molecule
 * id, then blocks 1, 2, ... of the same counter */
static void walk_words(const orc_sim *s, uint32_t id, int n, uint32_t *out) {
  uint32_t r[4];
  draw4(s->seed, (uint32_t)s->event, id, ORC_PHASE_WALK, 0, r);
  int k = 0;
  out[k++] = r[2];
  if (k < n) out[k++] = r[3];
  for (uint32_t blk = 1; k < n; blk++) {
    draw4(s->seed, (uint32_t)s->event, id, ORC_PHASE_WALK, blk, r);
    for (int j = 0; j < 4 && k < n; j++) out[k++] = r[j];
  }
}

static int pend_push(orc_sim *s, uint64_t key) {
  uint64_t q = s->n_slots - s->walk_slot0;
  if (q + 1 > s->pend_cap) {
    uint64_t c = s->pend_cap ? 2 * s->pend_cap : 64;
    uint64_t *k = realloc(s->pend_key, c * sizeof *k);
    if (!k) return -1;
    s->pend_key = k;
    s->pend_cap = c;
  }
  s->pend_key[q] = key;
  return 0;
}

/* End of a walk: the newborns of collision reactions get their ids in
 * ascending (mover id, product index) order, the same whatever order the
 * walk took; their slots are put in that order so that the table stays in
 * ascending id. */
static void finish_births(orc_sim *s) {
  uint64_t n = s->n_slots - s->walk_slot0;
  for (uint64_t z = 1; z < n; z++) {  /* insertion sort: newborns are few */
    for (uint64_t y = z; y > 0 && s->pend_key[y - 1] > s->pend_key[y]; y--) {
      uint64_t a = s->walk_slot0 + y - 1, b = a + 1;
      uint64_t tk = s->pend_key[y - 1]; s->pend_key[y - 1] = s->pend_key[y]; s->pend_key[y] = tk;
      uint32_t tv = s->vox[a]; s->vox[a] = s->vox[b]; s->vox[b] = tv;
      uint16_t ts = s->sp[a]; s->sp[a] = s->sp[b]; s->sp[b] = ts;
      uint8_t ta = s->alive[a]; s->alive[a] = s->alive[b]; s->alive[b] = ta;
    }
  }
  for (uint64_t z = 0; z < n; z++) {
    uint64_t q = s->walk_slot0 + z;
    s->id[q] = s->next_id++;
    s->slot_at[s->vox[q]] = (uint32_t)q;
  }
}

/* ---- one molecule's diffusion attempt (2.3) with collision (2.4.2) ------- */
static void attempt(orc_sim *s, uint32_t slot, int dir, int fire_forced,
                    uint32_t r1, uint8_t *reacted) {
  uint32_t a = s->vox[slot];
  uint16_t A = s->sp[slot];
  s->cnt[ORC_CNT_ATTEMPTS]++;
  uint32_t t = orc_neighbour_l(s->ni, s->nj, s->nk, a, dir, s->lattice, s->boundary);
  /* a wall, or a voxel of another compartment: the molecule stays, no
   * collision (2.3) */
  if (t == ORC_OUTSIDE || comp_at(s, t) != comp_at(s, a)) return;
  if (s->occ[t] == 0) {
    /* vacant: the molecule hops and carries its unwrapped displacement */
    int32_t hv[3];
    orc_hop_vector_l(s->ni, s->nj, s->nk, a, dir, s->lattice, hv);
    s->occ[t] = A;
    s->occ[a] = 0;
    s->vox[slot] = t;
    s->slot_at[t] = slot;
    s->dx[slot] += hv[0];
    s->dy[slot] += hv[1];
    s->dz[slot] += hv[2];
    s->cnt[ORC_CNT_HOPS]++;
    return;
  }
  /* occupied: a collision; reacts only with a registered partner */
  s->cnt[ORC_CNT_COLLISIONS]++;
  uint16_t B = s->occ[t];
  int r = s->pair_rx[A][B];
  if (r < 0) return;
  int fires = fire_forced >= 0 ? fire_forced : ((uint64_t)r1 < s->rx[r].thr2);
  if (!fires) return;
  const orc_rx *x = &s->rx[r];
  /* products beyond the second go to distinct vacant neighbours of the
   * mover's voxel (chosen as first-order products are, from the walk draw's
   * words r2, r3 and further blocks); too few vacant: the reaction fails
   * with no change */
  const int n_extra = x->n_prod > 2 ? x->n_prod - 2 : 0;
  uint32_t extra_vox[MAX_PROD];
  if (n_extra > 0) {
    uint32_t words[MAX_PROD];
    walk_words(s, s->id[slot], n_extra, words);
    if (pick_vacant(s, a, n_extra, words, extra_vox)) {
      s->cnt[ORC_CNT_PLACE_FAIL]++;
      return;
    }
  }
  uint32_t q = s->slot_at[t];
  /* first product in the partner's voxel, keeping the partner's identity */
  s->occ[t] = x->prod[0];
  mol_set_species(s, q, x->prod[0]);
  if (reacted && q < s->walk_slot0) reacted[q] = 1;  /* newborns do not walk anyway */
  if (x->n_prod >= 2) {
    /* second product in the mover's voxel, keeping the mover's identity */
    s->occ[a] = x->prod[1];
    mol_set_species(s, slot, x->prod[1]);
  } else {
    s->occ[a] = 0;
    mol_kill(s, slot);
  }
  for (int e = 0; e < n_extra; e++) {
    uint32_t v = extra_vox[e];
    s->occ[v] = x->prod[2 + e];
    if (pend_push(s, ((uint64_t)s->id[slot] << 8) | (uint64_t)(2 + e)) ||
        mol_new(s, 0xFFFFFFFFu, v, x->prod[2 + e]))
      s->oom = 1;
  }
  s->fired[r]++;
}

/* ---- one walk ------------------------------------------------------------ */
static int walk(orc_sim *s, const uint8_t due[MAX_SPECIES], const uint8_t *order,
                int mode) {
  uint8_t *reacted = calloc(s->n_slots + 1, 1);
  if (!reacted) return -1;
  uint64_t n_slots0 = s->n_slots;
  s->walk_slot0 = n_slots0;
  if (mode == ORC_MODE_S) {
    /* the paper's order: species ascending, molecules in ascending id */
    uint32_t *list = malloc((n_slots0 + 1) * sizeof *list);
    if (!list) { free(reacted); return -1; }
    uint64_t n = 0;
    for (int a = 1; a <= s->n_species; a++) {
      if (!due[a]) continue;
      for (uint64_t q = 0; q < n_slots0; q++)
        if (s->alive[q] && s->sp[q] == a) list[n++] = (uint32_t)q;
    }
    for (uint64_t z = 0; z < n; z++) {
      uint32_t slot = list[z];
      if (!s->alive[slot] || reacted[slot]) continue;
      uint32_t r[4];
      draw4(s->seed, (uint32_t)s->event, s->id[slot], ORC_PHASE_WALK, 0, r);
      attempt(s, slot, (int)scale32(r[0], 12), -1, r[1], reacted);
    }
    free(list);
  } else {
    buckets b;
    if (bucket_by_colour(s, due, &b)) { free(reacted); return -1; }
    for (int g = 0; g < s->n_col; g++) {
      int c = order[g];
      uint64_t lo = b.start[c], hi = b.start[c + 1];
      for (uint64_t z = 0; z < hi - lo; z++) {
        uint32_t slot = b.slots[mode == ORC_MODE_C_REV ? hi - 1 - z : lo + z];
        if (!s->alive[slot] || reacted[slot]) continue;
        uint32_t r[4];
        draw4(s->seed, (uint32_t)s->event, s->id[slot], ORC_PHASE_WALK, 0, r);
        attempt(s, slot, (int)scale32(r[0], 12), -1, r[1], reacted);
      }
    }
    free(b.slots);
  }
  free(reacted);
  finish_births(s);
  return s->oom ? -1 : 0;
}

int orc_run(orc_sim *s, uint64_t n_events, int mode) {
  s->frozen = 1;
  for (uint64_t z = 0; z < n_events; z++) {
    if (s->event >= 0xFFFFFFFFull) return -1;
    double te;
    uint8_t due[MAX_SPECIES];
    if (next_event(s, &te, due)) return -1;
    double dt = te - s->t;
    uint8_t order[ORC_MAX_COLOURS];
    orc_stage_order_n(s->seed, s->event, s->n_col, order);
    int rc;
    if (mode == ORC_MODE_S) rc = first_order_ssa(s, dt);
    else rc = first_order_coloured(s, dt, order, mode == ORC_MODE_C_REV);
    if (rc) return -1;
    if (walk(s, due, order, mode)) return -1;
    for (int a = 1; a <= s->n_species; a++)
      if (due[a]) s->n_walks[a]++;
    s->t = te;
    s->event++;
    compact(s);
  }
  return 0;
}

int orc_walk_forced(orc_sim *s, uint64_t n_order, const uint32_t *order_ids,
                    const uint8_t *dirs, const uint8_t *fire) {
  s->frozen = 1;
  uint8_t *reacted = calloc(s->n_slots + 1, 1);
  if (!reacted) return -1;
  s->walk_slot0 = s->n_slots;
  for (uint64_t z = 0; z < n_order; z++) {
    uint32_t want = order_ids[z];
    uint64_t slot = s->n_slots;
    for (uint64_t q = 0; q < s->n_slots; q++)
      if (s->id[q] == want) { slot = q; break; }
    if (slot == s->n_slots) { free(reacted); return -1; }
    if (!s->alive[slot] || reacted[slot]) continue;
    if (!(s->D[s->sp[slot]] > 0.0)) continue;
    attempt(s, (uint32_t)slot, dirs[want] % 12, fire[want] ? 1 : 0, 0, reacted);
  }
  free(reacted);
  finish_births(s);
  return s->oom ? -1 : 0;
}

uint64_t orc_n_molecules(const orc_sim *s) { return s->n_alive; }
uint64_t orc_n_voxels(const orc_sim *s) { return s->nv; }

void orc_read(const orc_sim *s, uint16_t *occ, uint32_t *id, uint32_t *vox,
              uint16_t *sp, int32_t *dx, int32_t *dy, int32_t *dz) {
  if (occ) memcpy(occ, s->occ, s->nv * sizeof *occ);
  uint64_t w = 0;
  for (uint64_t q = 0; q < s->n_slots; q++) {
    if (!s->alive[q]) continue;
    if (id) id[w] = s->id[q];
    if (vox) vox[w] = s->vox[q];
    if (sp) sp[w] = s->sp[q];
    if (dx) dx[w] = (int32_t)s->dx[q];
    if (dy) dy[w] = (int32_t)s->dy[q];
    if (dz) dz[w] = (int32_t)s->dz[q];
    w++;
  }
}

void orc_counters(const orc_sim *s, uint64_t out[ORC_CNT_N]) {
  for (int a = 0; a < ORC_CNT_N; a++) out[a] = s->cnt[a];
}

void orc_reactions_fired(const orc_sim *s, uint64_t *out) {
  for (int r = 0; r < s->n_rx; r++) out[r] = s->fired[r];
}

uint64_t orc_species_count(const orc_sim *s, uint16_t species) {
  if (species < 1 || species >= MAX_SPECIES) return 0;
  return s->count[species];
}

uint64_t orc_event(const orc_sim *s) { return s->event; }
double orc_time(const orc_sim *s) { return s->t; }
uint32_t orc_next_id(const orc_sim *s) { return s->next_id; }
