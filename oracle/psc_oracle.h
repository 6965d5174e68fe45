/*
 * psc_oracle.h -- plain, slow, single-threaded CPU reference for the lattice
 * walk of pSpatiocyte (Miyauchi, Iwamoto, Arjunan, Takahashi, "pSpatiocyte: A
 * Parallel Stochastic Method for Particle Reaction-Diffusion Systems").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU path.
 *
 * What it computes (paper section in brackets):
 *   - HCP voxel lattice in twisted Cartesian coordinates, 12-neighbour stencil
 *     with even/odd layer parity               [2.1 Coordinate System, Fig. 3]
 *   - diffusion events of each species every tau = 2 r^2 / (3 D), molecules
 *     hop to a random neighbour only if it is vacant  [2.3 Diffusion, eq. 2]
 *   - first-order reactions once per diffusion event over the elapsed
 *     interval, P(no reaction) = exp(-dt a0), reaction chosen by cumulative
 *     propensity                              [2.4.1 First-Order, eqs. 3-5]
 *   - second-order reactions on collision with probability
 *     p = k / (6 sqrt2 (DA+DB) r)              [2.4.2 Second-Order, eq. 6]
 *     and one to eleven products (2.4: two reactants may coalesce or decay
 *     into several molecules; at most eleven, the neighbours left)
 *   - compartments (2): groups of voxels given per voxel; a move into
 *     another compartment fails like a move into an occupied voxel (2.3),
 *     so molecules stay in their compartment, products included
 *   - periodic boxes, or boxes closed by walls: the space beyond a face of a
 *     closed box is read as another compartment
 *   - the face-centred cubic lattice (ABC stacking of the same close-packed
 *     layers; 2.1 names both close packings)
 *
 * Two processing orders are provided:
 *   ORC_MODE_C     coloured stages: each event's molecules are processed by the
 *                  colour of their voxel in a per-event random stage order,
 *                  ascending id inside a stage; first-order reactions by the
 *                  per-molecule law.  This is the order the GPU path follows.
 *   ORC_MODE_C_REV the same with descending id inside each stage (the results
 *                  must not change: same-colour closed neighbourhoods are
 *                  disjoint).
 *   ORC_MODE_S     the paper's sequential order: species ascending, molecules
 *                  in ascending id (the list order of 2.3); first-order
 *                  reactions by Gillespie's direct method run over the
 *                  interval (2.4.1).
 *
 * Parity status: every function here is pinned by a test that does not
 * re-derive it from this file (geometry against Euclidean distances,
 * Philox4x32-10 against its published known-answer vectors and the 4x64
 * variant against numpy's Philox-4x64, the walk by brute force on 4x4x4 and
 * by diffusion / reaction statistics).
 */
#ifndef PSC_ORACLE_H
#define PSC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_MODE_C = 0, ORC_MODE_S = 1, ORC_MODE_C_REV = 2 };

/* box boundary: periodic (the default) or reflecting walls on all six faces;
 * with walls a hop towards a neighbour beyond a face is blocked (the attempt
 * counts, nothing moves, no collision) and such neighbours take no products */
enum { ORC_BOUNDARY_PERIODIC = 0, ORC_BOUNDARY_REFLECT = 1 };
#define ORC_OUTSIDE 0xFFFFFFFFu

/* lattice: hexagonal close packed (ABAB stacking, the default) or
 * face-centred cubic (ABC stacking in the same twisted coordinates; the i and
 * j edges multiples of 8, the k edge of 12); 16 stage colours on both */
enum { ORC_LATTICE_HCP = 0, ORC_LATTICE_FCC = 1 };
#define ORC_MAX_COLOURS 24

/* Philox counter "phase" word values */
enum { ORC_PHASE_WALK = 0, ORC_PHASE_FIRST = 1, ORC_PHASE_STAGE = 2,
       ORC_PHASE_PLACE = 3, ORC_PHASE_SSA = 4 };

/* counters returned by orc_counters (in this order) */
enum { ORC_CNT_ATTEMPTS = 0, ORC_CNT_HOPS, ORC_CNT_COLLISIONS,
       ORC_CNT_PLACE_FAIL, ORC_CNT_N };

typedef struct orc_sim orc_sim;

/* ---- primitives (exposed so the tests can pin them) ---------------------- */
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
uint32_t orc_neighbour(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, int n);
/* as orc_neighbour for either boundary; ORC_OUTSIDE beyond a wall */
uint32_t orc_neighbour_b(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, int n,
                         int boundary);
/* the general forms, for either lattice */
uint32_t orc_neighbour_l(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, int n,
                         int lattice, int boundary);
void orc_hop_vector_l(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, int n, int lattice,
                      int32_t out[3]);
void orc_position_l(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, double rv, int lattice,
                    double out[3]);
int orc_colour_l(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, int lattice);
int orc_n_colours(int lattice);
/* a uniform permutation of 0..n-1 (n <= ORC_MAX_COLOURS) for an event */
void orc_stage_order_n(uint64_t seed, uint64_t event, int n, uint8_t *out);
/* out[12 v + n] = orc_neighbour(v, n) for every voxel */
void orc_neighbour_table(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t *out);
/* out[12 v + n] = orc_neighbour_l(v, n, lattice, boundary) for every voxel */
void orc_neighbour_table_l(uint32_t ni, uint32_t nj, uint32_t nk, int lattice, int boundary,
                           uint32_t *out);
void orc_hop_vector(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, int n,
                    int32_t out[3]);
void orc_position(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v, double rv,
                  double out[3]);
int orc_colour(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t v);
void orc_stage_order(uint64_t seed, uint64_t event, uint8_t out[16]);
uint64_t orc_second_order_threshold(double k, double DA, double DB, double rv);
uint32_t orc_prob_to_u32(double p);
double orc_tau(double rv, double D);

/* ---- simulation ---------------------------------------------------------- */
orc_sim *orc_create(uint32_t ni, uint32_t nj, uint32_t nk, double rv,
                    uint64_t seed);
void orc_destroy(orc_sim *s);
/* ORC_BOUNDARY_PERIODIC (default) or ORC_BOUNDARY_REFLECT; 0 on success */
int orc_set_boundary(orc_sim *s, int boundary);
/* ORC_LATTICE_HCP (default) or ORC_LATTICE_FCC (ni, nj % 8 == 0, nk % 12 == 0);
 * 0 on success */
int orc_set_lattice(orc_sim *s, int lattice);
/* returns the new species id (1, 2, ...) or -1 */
int orc_add_species(orc_sim *s, double D);
/* returns the new reaction id (0, 1, ...) or -1.  First order: 0..11
 * products, the first in place, the others on vacant neighbours.  Second
 * order: 1..11 products, the first on the partner's voxel (partner's id),
 * the second on the mover's voxel (mover's id), the others on vacant
 * neighbours of the mover's voxel with ids assigned at the end of the walk in
 * ascending (mover id, product index) order; too few vacant neighbours: the
 * reaction fails with no change (a placement failure). */
int orc_add_reaction(orc_sim *s, int n_reac, const uint16_t *reac, int n_prod,
                     const uint16_t *prod, double k);
/* places `count` molecules of `species` uniformly at random; 0 on success */
int orc_place_uniform(orc_sim *s, uint16_t species, uint64_t count);
/* compartments: comp[v] (nv entries, copied) is the compartment of voxel v.
 * A hop into a voxel of another compartment is blocked like a hop beyond a
 * wall, and products go only to vacant neighbours of the same compartment.
 * Without this call every voxel is in compartment 0.  0 on success */
int orc_set_compartments(orc_sim *s, const uint8_t *comp);
/* as orc_place_uniform, keeping only draws whose voxel is in compartment c */
int orc_place_uniform_in(orc_sim *s, uint16_t species, uint64_t count, int c);
/* loads a full state; arrays are borrowed; 0 on success, -1 if inconsistent */
int orc_load(orc_sim *s, const uint16_t *occ, uint64_t n_mol, const uint32_t *id,
             const uint32_t *vox, const int32_t *dx, const int32_t *dy,
             const int32_t *dz, uint64_t event, uint32_t next_id);
/* runs n events in the given mode; 0 on success */
int orc_run(orc_sim *s, uint64_t n_events, int mode);

/* one walk with forced choices (no time advance): molecules are processed in
 * the order given by `order_ids`; molecule with id x uses direction dirs[x]
 * and fires a collision reaction iff fire[x] != 0.  Used by the exhaustive
 * small-lattice tests.  0 on success. */
int orc_walk_forced(orc_sim *s, uint64_t n_order, const uint32_t *order_ids,
                    const uint8_t *dirs, const uint8_t *fire);

uint64_t orc_n_molecules(const orc_sim *s);
uint64_t orc_n_voxels(const orc_sim *s);
/* copies the state out; molecules in ascending id; any pointer may be NULL */
void orc_read(const orc_sim *s, uint16_t *occ, uint32_t *id, uint32_t *vox,
              uint16_t *sp, int32_t *dx, int32_t *dy, int32_t *dz);
void orc_counters(const orc_sim *s, uint64_t out[ORC_CNT_N]);
/* fired counts per reaction id (second- and first-order) */
void orc_reactions_fired(const orc_sim *s, uint64_t *out);
uint64_t orc_species_count(const orc_sim *s, uint16_t species);
uint64_t orc_event(const orc_sim *s);
double orc_time(const orc_sim *s);
uint32_t orc_next_id(const orc_sim *s);

#ifdef __cplusplus
}
#endif
#endif
