// psc_internal.h -- host-side records of libpsc shared by the C ABI
// implementation (psc_host.cpp) and the serving loop (psc_server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "psc.h"
#include "psc_core.h"

namespace psc_detail {

struct SpeciesDef {
  std::string name;
  double D = 0.0;
  double tau = 0.0;  // 2 r^2 / (3 D), eq. (2) of 2.3; 0 if immobile
};

struct ReactionDef {
  uint32_t nr = 0, np = 0;
  uint16_t r[2] = {0, 0};
  uint16_t p[psc::kMaxProducts] = {};
  double k = 0.0;
};

}  // namespace psc_detail

struct psc_lattice {
  psc_lattice_desc desc{};
  uint64_t nv = 0;
  psc::Geo geo{};
  std::vector<psc_detail::SpeciesDef> species{1};  // index 0 = vacant
  std::vector<psc_detail::ReactionDef> rx;
  bool frozen = false;
  bool poisoned = false;
  std::string err;

  // state before the freeze (host)
  std::vector<uint16_t> occ;          // species per voxel (linear order)
  std::vector<uint8_t> comp;          // compartment per voxel, or empty (all 0)
  std::vector<uint32_t> mid, mvox;
  std::vector<int32_t> mdx, mdy, mdz;
  uint32_t next_id = 0;
  uint64_t event0 = 0;
  uint64_t place_calls = 0;

  // static molecules: immobile species that react with nothing never change,
  // so they stay out of the walk's bins
  std::vector<uint32_t> st_id, st_vox;
  std::vector<int32_t> st_d[3];

  // event tape (absolute event index)
  std::vector<uint64_t> n_walks;
  uint64_t tape_end = 0;
  double t_prev = 0.0;
  std::vector<double> tape_time;
  std::vector<uint64_t> tape_due;
  std::vector<uint32_t> tape_thr, tape_cmax;
  uint64_t events_done = 0;  // events enqueued on the device
  uint64_t walkers0 = 0;     // molecules binned at the freeze (sizes the decision launch)

  // first-order slots: for each species, its first-order reactions in
  // registration order
  std::vector<uint16_t> fo_first, fo_rx;
  std::vector<uint8_t> fo_n;
  uint32_t n_fo = 0;
  uint32_t fo_extra_max = 0;  // most newborns of one first-order firing

  // device
  struct Block {
    void *p;
    size_t bytes;
  };
  std::vector<Block> blocks;
  uint64_t device_bytes = 0;
  psc::LatDev L{};
  psc::LatDev *dL = nullptr;
  uint64_t *d_tape_due = nullptr;
  uint32_t *d_tape_thr = nullptr, *d_tape_cmax = nullptr;
  uint64_t d_tape_rows = 0;
  int grid = 1;
  int items = 4;
  bool items_set = false;
  bool grid_set = false;
  uint64_t version = 0;   // bumped whenever the device record changes
  bool in_ensemble = false;
  hipStream_t last_stream = nullptr;

  // one event's launches captured as a HIP graph and replayed per event
  // (events whose first-order decisions need a launch of their own are
  // launched directly); rebuilt when the launch shape changes
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_grid = 0, graph_items = 0;

  // the device's last-event counts (LatDev::recent), copied back without a
  // wait at the end of each step and read at the next one that finds the
  // copy done: they drop launches that recent events did not need
  uint32_t *h_recent = nullptr;  // pinned, [kRecentN]
  hipEvent_t recent_ev = nullptr;
  bool recent_pending = false;
  bool recent_valid = false;
  uint32_t recent[psc::kRecentN] = {};

  // per-launch timing: kind (0 begin, 1 stage, 2 end) and its event pair
  bool timing = false;
  struct Timed {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> event_pool;
};

struct psc_ensemble {
  std::vector<psc_lattice *> members;
  int device = 0;
  std::string err;
  bool poisoned = false;
  psc::LatDev *d_lats = nullptr;                 // device array of member records
  std::vector<uint64_t> versions;           // member record versions uploaded
  int grid = 1024;
  int items = 4;
  uint32_t stages = 16;                     // the most stage colours of any member
  // one captured event of the batched launches, replayed per event
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_grid = 0, graph_items = 0;
  bool use_graph = true;                    // replay a captured event (false: direct launches)
  uint32_t autotune_events = 0;             // > 0: tune on the next step
  psc_launch tuned{0, 0};
  double tuned_ms_per_event = 0.0;
};

namespace psc_detail {

psc_status fail(psc_lattice *h, psc_status code, const char *fmt, ...);
psc_status efail(psc_ensemble *E, psc_status code, const char *fmt, ...);
void extend_tape(psc_lattice *h, uint64_t end);
psc_status sync_tape(psc_lattice *h, hipStream_t stream);
psc_status check_device_error(psc_lattice *h);
// sums of the kStatRep replicas of n statistics counters (see kStatRep)
psc_status read_replicas(psc_lattice *h, const unsigned long long *dev, uint32_t n,
                         uint32_t stride, uint64_t *out);
// The state read-back of psc_read_state with a pluggable reader of the
// occupancy: it fills occp[nv] with the species of every voxel in the ABI's
// linear order (flags masked off) and returns a status.
typedef psc_status (*OccupancyReader)(psc_lattice *h, uint16_t *occp, void *ctx);
psc_status read_state_with(psc_lattice *h, psc_state_view *out, OccupancyReader read_occ,
                           void *ctx);
psc_status read_occupancy_transient(psc_lattice *h, uint16_t *occp, void *ctx);
psc_status ensure_member_records(psc_ensemble *E, hipStream_t stream, uint64_t n_events);
psc_status ensure_graph(psc_ensemble *E);
bool any_births(const psc_ensemble *E);
psc_status ensure_lattice_graph(psc_lattice *h);
// device bytes a lattice with this capacity and size will hold once frozen
// ncol: stage colours of the lattice (16)
uint64_t estimate_device_bytes(uint64_t voxels, uint64_t max_molecules, bool displacement,
                               uint32_t n_reactions, bool collision_births, uint32_t ncol);

}  // namespace psc_detail
