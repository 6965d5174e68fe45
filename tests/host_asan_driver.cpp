// Test helper (host only): drives libpsc's host code through its C ABI on
// the CPU, with the HIP runtime and the kernel launchers answered by
// host_stub_hip.cpp, under AddressSanitizer: model registration, placement,
// the freeze (every device buffer and table), launch-shape selection, the
// event tape and its growth, per-launch timing switched on and off as the
// benchmark does, every read-back, checkpoint loading, ensembles with graph
// capture and autotuning, and the serving loop with valid and invalid jobs.
// Exit status 0 when every launch check passed.  Not part of the library.
#include <cstdio>
#include <cstring>
#include <vector>

#include "psc.h"

extern "C" int stub_launch_errors();
extern "C" int stub_open_ends();
extern "C" unsigned long long stub_fused_openings();
extern "C" unsigned long long stub_launches();

#define OK(call)                                                         \
  do {                                                                   \
    psc_status s_ = (call);                                              \
    if (s_ != PSC_OK) {                                                  \
      fprintf(stderr, "%s failed: %d at line %d\n", #call, s_, __LINE__); \
      return 1;                                                          \
    }                                                                    \
  } while (0)

// many: with the four-product collision (its newborns numbered at the event end)
static psc_lattice *make(uint32_t ni, uint32_t nj, uint32_t nk, uint32_t flags, uint64_t seed,
                         uint64_t per_species, bool many = true) {
  psc_lattice_desc d{};
  d.ni = ni;
  d.nj = nj;
  d.nk = nk;
  d.voxel_radius = 4.4e-9;
  d.seed = seed;
  d.max_molecules = 8 * per_species + 1024;
  d.flags = flags;
  psc_lattice *h = nullptr;
  if (psc_create_lattice(&d, &h)) return nullptr;
  uint16_t sp[6];
  const double D[6] = {1e-12, 1e-12, 0.5e-12, 1e-12, 0.0, 2e-12};
  for (int s = 0; s < 6; ++s)
    if (psc_add_species(h, "s", D[s], &sp[s])) return nullptr;
  const uint16_t ab[2] = {1, 2}, c1[1] = {3}, cc[1] = {3}, ab2[2] = {1, 2}, a4[2] = {1, 4},
                 many_p[4] = {1, 2, 6, 6}, six[1] = {6}, d6[3] = {2, 6, 6};
  if (psc_add_reaction(h, ab, 2, c1, 1, 1e-18, nullptr)) return nullptr;        // A + B -> C
  if (psc_add_reaction(h, cc, 1, ab2, 2, 200.0, nullptr)) return nullptr;       // C -> A + B
  if (many && psc_add_reaction(h, a4, 2, many_p, 4, 1e-18, nullptr)) return nullptr;  // A + O -> 4 products
  if (psc_add_reaction(h, six, 1, nullptr, 0, 50.0, nullptr)) return nullptr;   // F -> 0
  if (psc_add_reaction(h, six, 1, d6, 3, 30.0, nullptr)) return nullptr;        // F -> B + F + F
  for (uint16_t s = 1; s <= 6; ++s)
    if (psc_place_uniform(h, s, s == 5 ? 0 : per_species)) return nullptr;
  return h;
}

static int read_all(psc_lattice *h) {
  uint64_t nv = 0, nm = 0;
  uint32_t ns = 0, nr = 0;
  OK(psc_query_sizes(h, &nv, &nm, &ns, &nr));
  std::vector<uint16_t> occ(nv), sp(nm);
  std::vector<uint32_t> id(nm), vox(nm);
  std::vector<int32_t> dx(nm), dy(nm), dz(nm);
  std::vector<uint64_t> fired(nr);
  psc_state_view v{};
  v.occupancy = occ.data();
  v.n_molecules = nm;
  v.id = id.data();
  v.voxel = vox.data();
  v.species = sp.data();
  v.dx = dx.data();
  v.dy = dy.data();
  v.dz = dz.data();
  v.reactions_fired = fired.data();
  OK(psc_read_state(h, &v, nullptr));
  // too small: ECAPACITY and the required count
  psc_state_view w{};
  w.id = id.data();
  w.n_molecules = 0;
  if (nm && psc_read_state(h, &w, nullptr) != PSC_ECAPACITY) return 1;
  std::vector<uint64_t> counts(ns + 1);
  uint64_t dsum = 0, walkers = 0;
  OK(psc_read_stats(h, counts.data(), &dsum, &walkers));
  psc_counters c{};
  uint64_t ev = 0;
  OK(psc_read_counters(h, &c, &ev));
  uint64_t bytes = 0;
  OK(psc_device_bytes(h, &bytes));
  return 0;
}

int main() {
  std::vector<psc_lattice *> lats;
  const uint32_t flag_sets[4] = {PSC_TRACK_DISPLACEMENT, 0, PSC_LAYOUT_LINEAR | PSC_BOUNDARY_WALLS,
                                 PSC_LATTICE_FCC | PSC_TRACK_DISPLACEMENT};
  for (int a = 0; a < 4; ++a) {
    const bool fcc = (flag_sets[a] & PSC_LATTICE_FCC) != 0;
    psc_lattice *h = make(fcc ? 16 : 32, fcc ? 16 : 24, fcc ? 24 : 16, flag_sets[a], 11 + a, 200);
    if (!h) {
      fprintf(stderr, "lattice %d: %s\n", a, psc_last_error(nullptr));
      return 1;
    }
    lats.push_back(h);
  }
  // before the freeze: host read-back
  if (read_all(lats[0])) return 1;
  // the benchmark's sequence: warm-up, timing cleared and off, timed events,
  // then launches timed one by one, switched on and off without waiting
  psc_lattice *h = lats[0];
  OK(psc_step(h, 10, nullptr));
  OK(psc_set_kernel_timing(h, 1));
  OK(psc_set_kernel_timing(h, 0));
  for (int r = 0; r < 4; ++r) {
    OK(psc_set_kernel_timing(h, 2));
    OK(psc_step(h, 1, nullptr));
    OK(psc_set_kernel_timing(h, 0));
    OK(psc_step(h, 49, nullptr));
  }
  psc_kernel_times kt{};
  OK(psc_get_kernel_times(h, &kt));
  if (kt.stage_launches != 4 * 16 || kt.begin_launches != 4 || kt.end_launches != 4) {
    fprintf(stderr, "kernel times: %llu stage launches\n", (unsigned long long)kt.stage_launches);
    return 1;
  }
  OK(psc_set_kernel_timing(h, 1));  // clears (waits), reuses the events
  OK(psc_step(h, 2, nullptr));
  OK(psc_get_kernel_times(h, &kt));
  OK(psc_set_kernel_timing(h, 0));
  // the tape grows past its first 1024 events, twice
  OK(psc_step(h, 3000, nullptr));
  psc_launch l{1, 7};
  OK(psc_set_launch(h, &l));
  OK(psc_step(h, 6, nullptr));
  // graph replay, rebuilt after a change of launch shape
  OK(psc_set_graph_replay(h, 1));
  OK(psc_step(h, 4, nullptr));
  psc_launch l2{2, 9};
  OK(psc_set_launch(h, &l2));
  OK(psc_step(h, 2, nullptr));
  if (psc_set_graph_replay(h, 5) != PSC_EINVAL) return 1;
  // (an even event count: with the launchers stubbed the molecules stay in
  // the bins of event parity 0, which the read-back then finds)
  for (psc_lattice *x : lats) {
    OK(psc_step(x, 4, nullptr));
    if (read_all(x)) return 1;
  }
  // a checkpoint loaded into a fresh lattice of the same model
  {
    uint64_t nv = 0, nm = 0;
    OK(psc_query_sizes(lats[1], &nv, &nm, nullptr, nullptr));
    std::vector<uint16_t> occ(nv), sp(nm);
    std::vector<uint32_t> id(nm), vox(nm);
    psc_state_view v{};
    v.occupancy = occ.data();
    v.n_molecules = nm;
    v.id = id.data();
    v.voxel = vox.data();
    v.species = sp.data();
    OK(psc_read_state(lats[1], &v, nullptr));
    psc_lattice *r = make(32, 24, 16, 0, 12, 0);
    if (!r) return 1;
    if (psc_load_state(r, &v)) {
      fprintf(stderr, "load_state: %s\n", psc_last_error(r));
      return 1;
    }
    OK(psc_step(r, 4, nullptr));
    if (read_all(r)) return 1;
    psc_destroy(r);
  }
  // no collision newborns: a step after one whose counts came back runs each
  // event's end with the next event's opening
  {
    psc_lattice *f = make(32, 24, 16, PSC_TRACK_DISPLACEMENT, 21, 200, false);
    if (!f) return 1;
    OK(psc_step(f, 2, nullptr));
    OK(psc_step(f, 6, nullptr));
    if (read_all(f)) return 1;
    psc_destroy(f);
  }
  // an ensemble of fresh lattices: graph capture, autotuning, direct steps
  {
    std::vector<psc_lattice *> mem;
    for (int a = 0; a < 3; ++a) mem.push_back(make(16, 16, 16, 0, 40 + a, 50));
    psc_ensemble *E = nullptr;
    OK(psc_ensemble_create(mem.data(), 3, &E));
    if (psc_step(mem[0], 1, nullptr) != PSC_ESTATE) return 1;
    OK(psc_ensemble_autotune(E, 1));
    OK(psc_ensemble_step(E, 40, nullptr));
    psc_launch el{2, 300};
    OK(psc_ensemble_set_launch(E, &el));
    OK(psc_ensemble_step(E, 3000, nullptr));
    OK(psc_ensemble_sync(E));
    psc_ensemble_destroy(E);
    for (auto *m : mem) {
      if (read_all(m)) return 1;
      psc_destroy(m);
    }
  }
  // the serving loop: valid, invalid and never-fitting jobs
  {
    psc_server_options o{0, 64ull << 20, 16, 64, 3};
    psc_server *S = nullptr;
    OK(psc_server_create(&o, &S));
    const double D[3] = {1e-12, 0.5e-12, 1e-12};
    psc_reaction_desc rx[2]{};
    rx[0].n_r = 2;
    rx[0].n_p = 1;
    rx[0].reactants[0] = 1;
    rx[0].reactants[1] = 2;
    rx[0].products[0] = 3;
    rx[0].k = 1e-18;
    rx[1].n_r = 1;
    rx[1].n_p = 2;
    rx[1].reactants[0] = 3;
    rx[1].products[0] = 1;
    rx[1].products[1] = 2;
    rx[1].k = 100.0;
    psc_place_desc pl[2] = {{1, 100}, {2, 100}};
    std::vector<uint64_t> ids;
    for (int a = 0; a < 8; ++a) {
      psc_job_desc j{};
      j.ni = j.nj = j.nk = (a == 5) ? 6 : 16;   // job 5 is invalid
      j.voxel_radius = 4.4e-9;
      j.seed = 100 + a;
      j.max_molecules = 1024;
      j.n_species = 3;
      j.D = D;
      j.n_reactions = 2;
      j.reactions = rx;
      j.n_place = 2;
      j.place = pl;
      j.n_events = 50 + 10 * a;
      j.keep_state = a % 2;
      if (a == 7) j.ni = j.nj = j.nk = 512, j.max_molecules = 1 << 24;  // never fits
      uint64_t id = 0;
      OK(psc_server_submit(S, &j, &id));
      ids.push_back(id);
    }
    for (uint64_t id : ids) {
      psc_job_status st{};
      OK(psc_server_wait(S, id, &st));
      if (st.state == PSC_JOB_DONE && (id % 2 == 0)) {
        std::vector<uint16_t> occ(16 * 16 * 16);
        psc_state_view v{};
        v.occupancy = occ.data();
        v.n_molecules = 0;
        OK(psc_server_read_state(S, id, &v));
      }
    }
    // long jobs cancelled while queued or running
    std::vector<uint64_t> longs;
    for (int a = 0; a < 4; ++a) {
      psc_job_desc j{};
      j.ni = j.nj = j.nk = 16;
      j.voxel_radius = 4.4e-9;
      j.seed = 300 + a;
      j.max_molecules = 1024;
      j.n_species = 3;
      j.D = D;
      j.n_reactions = 2;
      j.reactions = rx;
      j.n_place = 2;
      j.place = pl;
      j.n_events = 50000;
      uint64_t id = 0;
      OK(psc_server_submit(S, &j, &id));
      longs.push_back(id);
    }
    // (with the launchers stubbed a job may finish before its cancellation:
    // then the cancellation is refused and the job is done)
    uint64_t n_cancelled = 0;
    for (uint64_t id : longs) {
      const psc_status cs = psc_server_cancel(S, id);
      if (cs != PSC_OK && cs != PSC_ESTATE) return 1;
      if (psc_server_cancel(S, id) != PSC_ESTATE) return 1;
      psc_job_status st{};
      OK(psc_server_wait(S, id, &st));
      if (st.state != (cs == PSC_OK ? PSC_JOB_CANCELLED : PSC_JOB_DONE)) return 1;
      n_cancelled += cs == PSC_OK;
    }
    for (uint64_t id : ids) (void)psc_server_release(S, id);
    psc_server_stats ss{};
    OK(psc_server_stats_get(S, &ss));
    if (ss.device_bytes_in_use != 0 || ss.failed != 2 || ss.cancelled != n_cancelled) {
      fprintf(stderr, "server: %llu bytes in use, %llu failed\n",
              (unsigned long long)ss.device_bytes_in_use, (unsigned long long)ss.failed);
      return 1;
    }
    psc_server_destroy(S);
  }
  for (psc_lattice *x : lats) psc_destroy(x);
  printf("launches %llu, launch check failures %d, event ends left open %d, fused openings %llu\n",
         stub_launches(), stub_launch_errors(), stub_open_ends(), stub_fused_openings());
  // the steps above run the fused event end and opening (a step after one
  // whose counts came back)
  return stub_launch_errors() || stub_open_ends() || stub_fused_openings() == 0 ? 1 : 0;
}
