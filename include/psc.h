/*
 * psc.h -- C ABI of libpsc, an MI355X (gfx950) engine for the lattice walk of
 * pSpatiocyte (Miyauchi, Iwamoto, Arjunan, Takahashi: "pSpatiocyte: A
 * Parallel Stochastic Method for Particle Reaction-Diffusion Systems").
 *
 * Model (paper section in brackets):
 *   - space is a hexagonal close-packed lattice of voxels of radius r (or,
 *     with PSC_LATTICE_FCC, a face-centred cubic one), held in twisted
 *     Cartesian coordinates (i, j, k); each voxel holds at most one molecule
 *     and has 12 neighbours at distance 2r                   [2.1, Fig. 3]
 *   - every species s with D_s > 0 has diffusion events every
 *     tau_s = 2 r^2 / (3 D_s); in an event each of its molecules picks one of
 *     its 12 neighbours at random and hops there only if it is vacant  [2.3]
 *   - a hop onto a molecule of a registered partner species fires the
 *     second-order reaction with p = k / (6 sqrt2 (DA + DB) r)    [2.4.2]
 *   - first-order reactions are applied once per diffusion event over the
 *     time elapsed since the previous event                      [2.2, 2.4.1]
 *
 * Conventions shared by every entry point:
 *   - Functions return psc_status: 0 on success, a negative code on error.
 *     Nothing is thrown or aborted across the ABI.  After an error other than
 *     PSC_EDEVICE the handle is unchanged; after PSC_EDEVICE it is poisoned
 *     (every later call but psc_destroy / psc_last_error returns
 *     PSC_EDEVICE).  psc_last_error(h) describes the last error on h.
 *   - Pointers in psc_state_view are HOST pointers.  They are borrowed for the
 *     duration of the call only.
 *   - Streams are hipStream_t passed as void*; NULL means the default stream.
 *   - One handle must not be used from two threads at once; distinct handles
 *     are independent.
 *   - Lattice dimensions must each be >= 4 and a multiple of 4 (the paper
 *     requires even counts, 2.1; multiples of 4 make the 16-colour stage
 *     schedule conflict-free on the periodic lattice; the FCC lattice also
 *     needs nk a multiple of 12 and ni, nj multiples of 8).  ni*nj*nk <= 2^32.
 *   - Boundaries are periodic unless PSC_BOUNDARY_WALLS closes the box.
 */
#ifndef PSC_H
#define PSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t psc_status;
#define PSC_OK 0
#define PSC_EINVAL (-1)     /* bad argument */
#define PSC_ESTATE (-2)     /* call not allowed in the handle's state */
#define PSC_ENOMEM (-3)     /* device or host allocation failed */
#define PSC_ECAPACITY (-4)  /* molecule capacity / vacant voxels exhausted */
#define PSC_EDEVICE (-5)    /* HIP error or device-side failure; poisoned */

/* species id 0 is the vacant voxel; registered species are 1, 2, ... */
#define PSC_MAX_SPECIES 63
#define PSC_MAX_REACTIONS 255
#define PSC_MAX_PRODUCTS 11

/* lattice flags */
#define PSC_TRACK_DISPLACEMENT 1u /* keep unwrapped per-molecule displacement */
#define PSC_BOUNDARY_WALLS 4u     /* close the box by walls on its six faces instead
                                     of wrapping it periodically: a move into
                                     another compartment fails like a move into an
                                     occupied voxel (2.3), and the space beyond a
                                     face is such a compartment.  A hop towards it
                                     counts as an attempt and is neither a hop nor
                                     a collision; first-order products are never
                                     placed there. */
#define PSC_LAYOUT_LINEAR 2u      /* keep the occupancy in linear order on the
                                     device instead of 4x4x4 bricks (a 128-byte
                                     line each); results are identical */
#define PSC_LATTICE_FCC 8u        /* face-centred cubic lattice instead of HCP:
                                     the same close-packed layers and twisted
                                     Cartesian coordinates (2.1), stacked ABC
                                     instead of ABAB, so the layer phase is
                                     k mod 3.  Voxel centres, neighbour rows and
                                     displacement units are as for HCP with that
                                     phase; the walk keeps 16 colour stages (a
                                     colouring periodic in 8 along i and j).
                                     nk must be a multiple of 12, ni and nj of
                                     8. */

/* Device memory allocator hooks.  alloc returns a device pointer of at least
 * `bytes` bytes usable on `stream` (or NULL on failure); free releases it.
 * When both are NULL the library uses hipMalloc / hipFree. */
typedef void *(*psc_alloc_fn)(size_t bytes, void *stream, void *user);
typedef void (*psc_free_fn)(void *ptr, void *user);

typedef struct psc_lattice psc_lattice;

typedef struct psc_lattice_desc {
  uint32_t ni, nj, nk;     /* voxels along the straight axis i and the two
                              zigzag axes j, k (2.1) */
  double voxel_radius;     /* r, metres, > 0 */
  uint64_t seed;           /* key of every random draw of this lattice */
  uint64_t max_molecules;  /* capacity: live molecules at any time */
  uint32_t flags;          /* PSC_TRACK_DISPLACEMENT | PSC_LAYOUT_LINEAR |
                              PSC_BOUNDARY_WALLS | PSC_LATTICE_FCC */
  int32_t device;          /* HIP device ordinal */
  psc_alloc_fn alloc;      /* optional allocator hooks (both or neither) */
  psc_free_fn free;
  void *alloc_user;
} psc_lattice_desc;

typedef struct psc_counters {
  uint64_t attempts;           /* hop attempts (one per participating
                                  molecule per diffusion event) */
  uint64_t hops;               /* attempts that moved */
  uint64_t collisions;         /* attempts whose target voxel was occupied */
  uint64_t placement_failures; /* reactions (first order, or collisions with
                                  more than two products) that found too few
                                  vacant neighbours for their products */
} psc_counters;

/* A full lattice state.  For psc_load_state every array holds n_molecules
 * entries (dx, dy, dz may be NULL = zero); ids strictly ascending, each below
 * next_id; occupancy[voxel[q]] == species[q]; every other voxel 0.
 * For psc_read_state the caller provides arrays of capacity n_molecules (set
 * n_molecules to that capacity; any array pointer may be NULL to skip it) and
 * the call sets n_molecules to the number of live molecules; molecules are
 * returned in ascending id. */
typedef struct psc_state_view {
  uint16_t *occupancy;       /* [ni*nj*nk], v = i + ni*(j + nj*k) */
  uint64_t n_molecules;
  uint32_t *id;
  uint32_t *voxel;
  uint16_t *species;
  int32_t *dx, *dy, *dz;     /* unwrapped displacement: dx in r, dy in r/sqrt3,
                                dz in 2 sqrt(2/3) r */
  uint64_t event;            /* diffusion events completed */
  uint32_t next_id;          /* id the next newborn molecule will take */
  double time;               /* read: simulated time of the last event, s */
  psc_counters counters;     /* read: cumulative counters */
  uint64_t *reactions_fired; /* read: [n_reactions] or NULL */
} psc_state_view;

/* ---- lattice life cycle --------------------------------------------------- */

/* Creates a lattice with no species.  EINVAL on bad dimensions, radius or
 * capacity; ENOMEM if the occupancy lattice cannot be allocated. */
psc_status psc_create_lattice(const psc_lattice_desc *desc, psc_lattice **out);

/* Frees every device and host resource of h (NULL is ignored).  Pending work
 * on the lattice's streams is waited for first. */
void psc_destroy(psc_lattice *h);

/* Message for the last error on h; for h == NULL, the last psc_create_lattice
 * failure of this thread.  The string lives until the next call on h. */
const char *psc_last_error(const psc_lattice *h);

/* ---- model (2.3, 2.4) ----------------------------------------------------- */

/* Registers a species with diffusion coefficient D (m^2/s).  D == 0 makes it
 * immobile (an obstacle unless it reacts).  EINVAL if D < 0 or not finite or
 * more than PSC_MAX_SPECIES species; ESTATE after the first psc_step. */
psc_status psc_add_species(psc_lattice *h, const char *name, double D,
                           uint16_t *out_id);

/* Registers a reaction.  n_r == 1: first-order, k in 1/s, 0..PSC_MAX_PRODUCTS
 * products: the first stays in the reactant's voxel (keeping its id), the
 * others go to distinct vacant neighbours (new ids), and the reaction fails
 * with no change if too few are vacant (2.4.1).  n_r == 2: second-order,
 * k in m^3/s, 1..PSC_MAX_PRODUCTS products (2.4: two reactants may coalesce
 * or decay into several molecules): on collision the first product takes the
 * partner's voxel and id, the second the mover's voxel and id (with one
 * product the mover's voxel is vacated), the others distinct vacant
 * neighbours of the mover's voxel with new ids, numbered at the end of the
 * event in ascending (mover id, product index) order; too few vacant
 * neighbours: no reaction and one placement failure (2.4.2).  EINVAL for a second pair
 * on the same unordered reactant pair, two immobile reactants, unknown
 * species, or k < 0; ESTATE after the first psc_step. */
psc_status psc_add_reaction(psc_lattice *h, const uint16_t *reactants,
                            uint32_t n_r, const uint16_t *products, uint32_t n_p,
                            double k, uint32_t *out_id);

/* How a registered reaction is applied.  Second order (2.4.2, eq. 6):
 * p = k / (6 sqrt2 (D_A + D_B) r); a collision with a registered partner fires
 * iff the draw r1 < threshold, or always once p >= 1 (clamped = 1, threshold
 * = 2^32).  First order (2.4.1): p = k in 1/s, threshold 0, clamped 0 (its
 * per-event probability depends on the event's interval).  Valid before and
 * after the first step; EINVAL for an unknown reaction id or out == NULL. */
typedef struct psc_reaction_info {
  uint32_t order;      /* 1 or 2 */
  uint32_t clamped;    /* 1: p > 1 was clamped to 1 */
  double p;            /* per-collision probability before clamping; k for order 1 */
  uint64_t threshold;  /* on a uniform 32-bit draw; 2^32 = always */
} psc_reaction_info;

psc_status psc_get_reaction_info(const psc_lattice *h, uint32_t reaction_id,
                                 psc_reaction_info *out);

/* ---- initial state -------------------------------------------------------- */

/* Places `count` molecules of `species` at uniformly random vacant voxels
 * (the paper's homogeneous start, 3.4).  The c-th call draws candidate voxel
 * floor(r * nv / 2^32) for attempt a from Philox(seed; c, a, 3, 0) word 0 and
 * keeps it if vacant; new molecules take ids next_id, next_id + 1, ...
 * ECAPACITY if there are too few vacant voxels or capacity; ESTATE after the
 * first psc_step. */
psc_status psc_place_uniform(psc_lattice *h, uint16_t species, uint64_t count);

/* Compartments (2): a cell is modelled as groups of voxels, and a move into
 * a voxel of another compartment fails as a move into an occupied one (2.3).
 * comp[v] (ni*nj*nk entries, linear order v = i + ni*(j + nj*k), copied) is
 * the compartment, 0..255, of voxel v; without this call every voxel is in
 * compartment 0.  A hop towards a voxel of another compartment counts as an
 * attempt and is neither a hop nor a collision (no reaction across a
 * compartment boundary); every product of a reaction stays in its
 * reactants' compartment (first-order and collision products take only
 * vacant neighbours of that compartment).  Molecules placed or loaded
 * before or after this call stay where they are.  EINVAL if comp is NULL;
 * ESTATE after the first psc_step. */
psc_status psc_set_compartments(psc_lattice *h, const uint8_t *comp);

/* As psc_place_uniform, keeping only candidate voxels that are vacant and in
 * `compartment` (the same draws: the c-th placement call, attempt a,
 * Philox(seed; c, a, 3, 0) word 0).  ECAPACITY if the compartment has too
 * few vacant voxels or capacity is exceeded; EINVAL for a compartment above
 * 255 or an unknown species; ESTATE after the first psc_step. */
psc_status psc_place_uniform_in(psc_lattice *h, uint16_t species, uint64_t count,
                                uint32_t compartment);

/* Replaces the whole state with a copy of `state` (see psc_state_view).
 * EINVAL if it is inconsistent; ECAPACITY if it exceeds max_molecules;
 * ESTATE after the first psc_step. */
psc_status psc_load_state(psc_lattice *h, const psc_state_view *state);

/* ---- running ---------------------------------------------------------------- */

/* Runs n_events diffusion events, asynchronously on `stream`.  The first
 * call freezes the model: probabilities become 32-bit integer thresholds
 * (computed in FP64 on the host) and the state moves to the device.
 * Device-side failures (capacity overflow) surface at the next
 * psc_read_state or psc_sync as ECAPACITY / EDEVICE. */
psc_status psc_step(psc_lattice *h, uint64_t n_events, void *stream);

/* Waits for the lattice's pending work; reports device-side failures. */
psc_status psc_sync(psc_lattice *h);

/* Copies the current state to host arrays (see psc_state_view) and waits.
 * ECAPACITY if the caller's arrays are too small (n_molecules is then set to
 * the required count and nothing else is written). */
psc_status psc_read_state(psc_lattice *h, psc_state_view *out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * read-back as psc_read_state, identical results, without any device
 * allocation.  psc_read_state converts a bricked occupancy through a
 * transient device buffer as large as the lattice; this call converts one
 * layer of bricks (4 k-layers, 4 ni nj voxels) at a time through a static
 * 32 MiB device buffer that each GPU holds until the process ends, and runs
 * its conversion kernels and copies on `stream` (NULL: the default stream),
 * then waits.  EINVAL (nothing read) if a layer of bricks exceeds the buffer:
 * ni * nj > 4194304 in the brick layout (any size with PSC_LAYOUT_LINEAR).
 * The buffer is shared by every call on one GPU and keeps the last call's
 * contents: calls that overlap on one GPU (from several threads, or on
 * different streams) race and must not be made. */
psc_status psc_read_state_noalloc(psc_lattice *h, psc_state_view *out, void *stream);

/* Cumulative counters and events completed, without reading the state
 * (waits for pending work). */
psc_status psc_read_counters(psc_lattice *h, psc_counters *out, uint64_t *event);

/* Statistics without reading the state (waits for pending work):
 * species_count[s] for s = 0..n_species (index 0 unused) = live molecules of
 * each species, kept exact on the device through every reaction;
 * disp_sum = sum over molecules of 3 dx^2 + dy^2 + 8 dz^2, i.e. 3 |d|^2 / r^2
 * for the unwrapped displacements (zero unless PSC_TRACK_DISPLACEMENT), so the
 * mean squared displacement is r^2 disp_sum / (3 n) (3.1, eq. 7);
 * n_walkers = molecules that can move.  Any pointer may be NULL. */
psc_status psc_read_stats(psc_lattice *h, uint64_t *species_count, uint64_t *disp_sum,
                          uint64_t *n_walkers);

/* Sizes needed to read the state. */
psc_status psc_query_sizes(const psc_lattice *h, uint64_t *n_voxels,
                           uint64_t *n_molecules, uint32_t *n_species,
                           uint32_t *n_reactions);

/* The same sizes under the name the scope of this library first gave them. */
psc_status psc_required_sizes(const psc_lattice *h, uint64_t *n_voxels,
                              uint64_t *n_molecules, uint32_t *n_species,
                              uint32_t *n_reactions);

/* Device bytes held by the lattice (for admission control). */
psc_status psc_device_bytes(const psc_lattice *h, uint64_t *bytes);

/* ---- launch shape (result-invariant) ---------------------------------------- */

/* Launch shape of the walk-stage kernel: molecules per thread per pass
 * (1, 2, 4, 8 or 16) and workgroups per launch (grid-striding beyond).  It
 * changes only how the work is spread over the GPU, never the result (the
 * molecules of one stage commute).  0 keeps the current value.  Unless set,
 * both are chosen at the first step from the molecules in the colour bins:
 * 4 items when a stage fills the GPU with 4-item chunks (512 workgroups),
 * else 2 or 1 items, and one chunk per workgroup for 1.25 times an average
 * bin (at most 65536 workgroups). */
typedef struct psc_launch {
  uint32_t items_per_thread;
  uint32_t stage_blocks;
} psc_launch;

psc_status psc_set_launch(psc_lattice *h, const psc_launch *l);
psc_status psc_get_launch(const psc_lattice *h, psc_launch *out);

/* Graph replay (result-invariant): 1 captures one event's launches (the
 * first-order pass, the 16 colour stages, the event end) as a HIP graph on
 * the lattice's first step after the call and replays it for every event,
 * instead of issuing the launches one by one; events whose first-order
 * decisions need a launch of their own (many expected candidates) are still
 * launched directly, and so is every event while per-launch timing is on.
 * For small lattices, whose events are short enough for the host's launch
 * rate to matter.  0 (the default) launches directly.  Other values:
 * PSC_EINVAL. */
psc_status psc_set_graph_replay(psc_lattice *h, int enable);

/* ---- measurement ------------------------------------------------------------ */

/* Per-kernel device time of the steps run while timing is on, measured with
 * HIP events recorded on the step's stream around every launch:
 * begin = stage order + first-order pass (with its separate decision launch
 * when an event expects many first-order candidates), stage = one colour
 * stage of the walk, end = flag sweep and numbering of collision newborns. */
typedef struct psc_kernel_times {
  double begin_ms, stage_ms, end_ms;
  uint64_t begin_launches, stage_launches, end_launches;
} psc_kernel_times;

/* Per-launch timing: 1 turns it on and clears the totals (waits for the
 * device), 0 turns it off and 2 turns it back on, both keeping the totals and
 * without waiting, so that a sample of the events of a timed run can be
 * measured without stalling it.  Timing adds two event records per launch;
 * leave it off for throughput runs.  Other values: PSC_EINVAL. */
psc_status psc_set_kernel_timing(psc_lattice *h, int enable);

/* Waits for the timed work and returns the totals since timing was last
 * turned on with 1. */
psc_status psc_get_kernel_times(psc_lattice *h, psc_kernel_times *out);

/* ---- ensembles ---------------------------------------------------------------
 * Many independent lattices (replicates of one model, or different models of
 * any sizes) advanced together: every event of every member is one batched
 * launch sequence (first-order pass of all members, the 16 colour stages of
 * all members as one work list each, event end), captured once as a HIP
 * graph and replayed.  Each member's result is bit-identical to stepping it
 * alone: the members share no state and every draw is keyed by the member's
 * own seed, event and molecule ids. */
typedef struct psc_ensemble psc_ensemble;

/* Groups 1..4096 distinct lattices of one device.  Members are frozen (their
 * state moves to the device) and, while grouped, may be read (psc_read_state,
 * psc_read_counters) but not stepped alone (ESTATE).  The members must
 * outlive the ensemble.  EINVAL on a bad member list. */
psc_status psc_ensemble_create(psc_lattice *const *members, uint32_t n, psc_ensemble **out);

/* Advances every member by n_events, asynchronously on `stream`. */
psc_status psc_ensemble_step(psc_ensemble *e, uint64_t n_events, void *stream);

/* Waits for the ensemble's work; reports device-side failures of members. */
psc_status psc_ensemble_sync(psc_ensemble *e);

/* Launch shape of the batched stage kernel (items per thread 1, 2, 4 or 8;
 * workgroups per launch).  Result-invariant. */
psc_status psc_ensemble_set_launch(psc_ensemble *e, const psc_launch *l);
psc_status psc_ensemble_get_launch(const psc_ensemble *e, psc_launch *out);

/* Autotuner: the next psc_ensemble_step times each candidate launch shape on
 * trial_events of its own events (plus one untimed event per candidate) and
 * runs the rest with the fastest.  The events count toward n_events and the
 * results are the same as with any shape. */
psc_status psc_ensemble_autotune(psc_ensemble *e, uint32_t trial_events);

/* The shape the autotuner chose and its time per event (0 before tuning). */
psc_status psc_ensemble_tuned(const psc_ensemble *e, psc_launch *chosen, double *ms_per_event);

/* Member i's state (as psc_read_state on that member, after waiting for the
 * ensemble's work).  EINVAL for i beyond the members. */
psc_status psc_ensemble_read(psc_ensemble *e, uint32_t i, psc_state_view *out, void *stream);

/* Releases the ensemble (members stay valid and can be stepped alone). */
void psc_ensemble_destroy(psc_ensemble *e);

/* Message for the last error on e; NULL: the last create failure. */
const char *psc_ensemble_last_error(const psc_ensemble *e);

/* ---- serving loop ---------------------------------------------------------------
 * Continuous batching of simulation jobs.  Jobs are submitted from any thread
 * and copied.  Builder threads admit queued jobs (first come, first served)
 * while their device memory fits the budget and build them; a worker thread
 * owns the batched steps: at every step boundary the built jobs join, all
 * resident jobs advance together as one batched ensemble by `quantum_events`
 * events (a job that reaches its last event idles for the rest of the
 * quantum), and finished jobs retire, which frees their memory for the
 * queue.  A job's result is bit-identical to running it alone. */
typedef struct psc_server psc_server;

typedef struct psc_server_options {
  int32_t device;           /* HIP device ordinal */
  uint64_t budget_bytes;    /* device memory the resident jobs may hold */
  uint32_t quantum_events;  /* events per step between admissions (>= 1) */
  uint32_t max_active;      /* resident jobs at most (1..4096) */
  uint32_t builders;        /* threads building admitted jobs (host placement
                               and the freeze) while the GPU steps the
                               resident ones; 0: 4, at most 64 */
} psc_server_options;

typedef struct psc_reaction_desc {
  uint32_t n_r, n_p;        /* as psc_add_reaction */
  uint16_t reactants[2];
  uint16_t products[PSC_MAX_PRODUCTS];
  double k;
} psc_reaction_desc;

typedef struct psc_place_desc {
  uint16_t species;         /* uniform placement, as psc_place_uniform */
  uint64_t count;
} psc_place_desc;

/* One job: a lattice (desc fields as psc_lattice_desc; allocator hooks and
 * device come from the server), species D[0..n_species) = ids 1..n,
 * reactions, placements in order, and the number of events to run. */
typedef struct psc_job_desc {
  uint32_t ni, nj, nk;
  double voxel_radius;
  uint64_t seed;
  uint64_t max_molecules;
  uint32_t flags;
  uint32_t n_species;
  const double *D;
  uint32_t n_reactions;
  const psc_reaction_desc *reactions;
  uint32_t n_place;
  const psc_place_desc *place;
  uint64_t n_events;
  uint32_t keep_state;      /* keep the final state until psc_server_release */
} psc_job_desc;

#define PSC_JOB_QUEUED 0
#define PSC_JOB_RUNNING 1
#define PSC_JOB_DONE 2
#define PSC_JOB_FAILED 3
#define PSC_JOB_CANCELLED 4

typedef struct psc_job_status {
  int32_t state;            /* PSC_JOB_* */
  psc_status error;         /* why a job failed (EINVAL: bad job; ENOMEM: does
                               not fit the budget; ECAPACITY; EDEVICE) */
  double submit_s, admit_s, done_s;  /* seconds since the server started */
  uint64_t events_done;
  psc_counters counters;
} psc_job_status;

typedef struct psc_server_stats {
  uint64_t submitted, admitted, done, failed, active, queued;
  uint64_t device_bytes_in_use;
  uint64_t attempts;        /* hop attempts of finished jobs */
  uint64_t quanta;          /* batched steps run */
  double busy_s;            /* time spent in batched steps */
  uint64_t peak_active;     /* most jobs resident at once */
  uint64_t cancelled;       /* jobs cancelled (psc_server_cancel) */
} psc_server_stats;

/* Device bytes the server reserves for a job (its admission cost), for a
 * server whose quantum is at most 1024 events: the lattice's buffers as
 * allocated at the freeze plus a bound on its event tape (which grows with
 * the job's events and its first-order reactions).  A job holds this much of
 * the budget from its admission until it is retired (or, with keep_state,
 * released), also when it fails. */
psc_status psc_server_job_bytes(const psc_job_desc *job, uint64_t *bytes);

/* Starts the worker.  EINVAL on bad options or device. */
psc_status psc_server_create(const psc_server_options *opt, psc_server **out);

/* psc_server_create with the default options: a quantum of 64 events, at
 * most 1024 resident jobs, 4 builder threads, on `device` under
 * `budget_bytes` of device memory. */
psc_status psc_server_start(uint64_t budget_bytes, int32_t device, psc_server **out);

/* Queues a copy of the job; *job_id identifies it.  A job that can never fit
 * the budget fails at once (ENOMEM); one the lattice rejects fails with that
 * status when it is admitted; other jobs are unaffected.  ESTATE once the
 * server is being destroyed. */
psc_status psc_server_submit(psc_server *s, const psc_job_desc *job, uint64_t *job_id);

/* Current status of a job (non-blocking) / wait until it is done, failed or
 * cancelled. */
psc_status psc_server_poll(psc_server *s, uint64_t job_id, psc_job_status *out);
psc_status psc_server_wait(psc_server *s, uint64_t job_id, psc_job_status *out);

/* Final state of a finished job submitted with keep_state (ESTATE otherwise),
 * as psc_read_state. */
psc_status psc_server_read_state(psc_server *s, uint64_t job_id, psc_state_view *out);

/* Cancels a job that has not finished: a queued job leaves the queue at once,
 * one being admitted or running is retired at the next step boundary (its
 * events so far are lost); its state becomes PSC_JOB_CANCELLED and its
 * memory returns to the budget.  Other jobs are unaffected.  ESTATE for a job
 * already done, failed or cancelled; EINVAL for an unknown id.  For a server
 * that must stop before its queue drains (psc_server_destroy runs every
 * submitted job to completion). */
psc_status psc_server_cancel(psc_server *s, uint64_t job_id);

/* Frees a finished job's kept state. */
psc_status psc_server_release(psc_server *s, uint64_t job_id);

psc_status psc_server_stats_get(psc_server *s, psc_server_stats *out);
const char *psc_server_last_error(const psc_server *s);

/* Runs every submitted job to completion, then stops the worker and frees
 * everything (kept states included). */
void psc_server_destroy(psc_server *s);

#ifdef __cplusplus
}
#endif
#endif
