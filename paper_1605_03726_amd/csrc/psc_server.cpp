// psc_server.cpp -- continuous-batching serving loop of libpsc.
//
// Jobs (one lattice + model + initial state + a number of diffusion events
// each) are submitted from any thread.  A builder thread admits queued jobs
// while their estimated device memory fits the budget and builds them (host
// placement, the freeze on a stream of its own).  A worker thread owns the
// batched steps: at every step boundary the built jobs join, all resident
// jobs advance together as one batched ensemble by a quantum of events (a
// job that reaches its last event idles for the rest of the quantum), and
// finished jobs retire, freeing their memory for the queue.  A job's result does not depend on what it ran with:
// every draw is keyed by the job's own seed, event and molecule ids.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "psc_internal.h"

using namespace psc;
using namespace psc_detail;

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
  uint64_t id = 0;
  psc_lattice_desc desc{};
  std::vector<double> D;
  std::vector<psc_reaction_desc> rx;
  std::vector<psc_place_desc> place;
  uint64_t n_events = 0;
  bool keep_state = false;
  psc_job_status st{};
  psc_lattice *lat = nullptr;
  uint64_t est_bytes = 0;
  bool charged = false;  // est_bytes counted in the server's used bytes
  bool cancel = false;   // cancelled while being admitted or running
};

}  // namespace

struct psc_server {
  psc_server_options opt{};
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job *> queue;          // submitted, waiting for admission
  std::deque<Job *> ready;          // admitted and built, joining at the next step boundary
  uint64_t building = 0;            // admitted, being built
  std::map<uint64_t, Job *> jobs;   // every job ever submitted, by id
  std::vector<Job *> active;
  uint64_t next_job = 1;
  uint64_t used_bytes = 0;
  bool stopping = false;
  psc_server_stats stats{};
  std::thread worker;               // owns the batched steps
  std::vector<std::thread> builders; // build admitted jobs meanwhile
  std::condition_variable cv_build;
  hipStream_t stream = nullptr;
  psc_ensemble ens;                  // the resident jobs, rebuilt on change
  uint64_t ens_capacity = 0;
  bool ens_dirty = true;
  std::string err;
};

namespace {

double seconds(const psc_server *S) {
  return std::chrono::duration<double>(Clock::now() - S->t0).count();
}

// builds the job's lattice on the host (model, placement), freezes it on the
// device; returns a status for the job
psc_status build_job(Job *j, hipStream_t stream) {
  psc_lattice *h = nullptr;
  psc_status st = psc_create_lattice(&j->desc, &h);
  if (st) return st;
  j->lat = h;
  for (size_t s = 0; s < j->D.size(); ++s) {
    st = psc_add_species(h, "", j->D[s], nullptr);
    if (st) return st;
  }
  for (auto &r : j->rx) {
    st = psc_add_reaction(h, r.reactants, r.n_r, r.products, r.n_p, r.k, nullptr);
    if (st) return st;
  }
  for (auto &p : j->place) {
    st = psc_place_uniform(h, p.species, p.count);
    if (st) return st;
  }
  st = psc_step(h, 0, stream);  // freeze: the state moves to the device
  if (st) return st;
  h->L.stop_event = h->events_done + j->n_events;
  if (hipMemcpy(h->dL, &h->L, sizeof(LatDev), hipMemcpyHostToDevice) != hipSuccess)
    return PSC_EDEVICE;
  h->version++;
  return PSC_OK;
}

void finish_job(psc_server *S, Job *j, int state, psc_status code) {
  // called with the lock held
  j->st.state = state;
  j->st.error = code;
  j->st.done_s = seconds(S);
  if (state == PSC_JOB_DONE) S->stats.done++;
  else if (state == PSC_JOB_CANCELLED) S->stats.cancelled++;
  else S->stats.failed++;
  S->cv_done.notify_all();
}

// the admission cost of a job is charged when it is admitted and returned
// when its lattice is released, whether or not the lattice was ever built
// (called with the lock held)
void charge(psc_server *S, Job *j) {
  S->used_bytes += j->est_bytes;
  j->charged = true;
  S->stats.device_bytes_in_use = S->used_bytes;
}

void release_lattice(psc_server *S, Job *j) {
  if (j->lat) {
    psc_destroy(j->lat);
    j->lat = nullptr;
  }
  if (j->charged) {
    S->used_bytes -= std::min(S->used_bytes, j->est_bytes);
    j->charged = false;
    S->stats.device_bytes_in_use = S->used_bytes;
  }
}

// Admission (first come, first served): the builder thread takes the job at
// the head of the queue once it fits the budget beside the jobs resident,
// ready or being built (a job always fits an idle server: larger ones are
// refused at submission), and builds it -- placement on the host, the
// freeze on its own stream -- while the worker keeps stepping the resident
// jobs; built jobs join at the next step boundary.
bool can_admit(const psc_server *S) {
  if (S->queue.empty()) return false;
  const uint64_t resident = S->active.size() + S->ready.size() + S->building;
  if (resident >= S->opt.max_active) return false;
  return resident == 0 || S->used_bytes + S->queue.front()->est_bytes <= S->opt.budget_bytes;
}

void builder_main(psc_server *S) {
  (void)hipSetDevice(S->opt.device);
  hipStream_t stream = nullptr;  // this builder's own: a freeze waits for it alone
  const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    S->cv_build.wait(lk, [&] { return can_admit(S) || (S->stopping && S->queue.empty()); });
    if (!can_admit(S)) break;  // stopping, nothing queued
    Job *j = S->queue.front();
    S->queue.pop_front();
    S->stats.queued = S->queue.size();
    charge(S, j);
    S->building++;
    lk.unlock();
    const psc_status st = have_stream ? build_job(j, stream) : PSC_EDEVICE;
    lk.lock();
    S->building--;
    if (j->cancel) {
      release_lattice(S, j);
      finish_job(S, j, PSC_JOB_CANCELLED, PSC_OK);
    } else if (st) {
      if (j->lat && j->lat->poisoned) S->err = j->lat->err;
      release_lattice(S, j);
      finish_job(S, j, PSC_JOB_FAILED, st);
    } else {
      S->ready.push_back(j);
    }
    S->cv_work.notify_one();
  }
  lk.unlock();
  if (have_stream) (void)hipStreamDestroy(stream);
}

void worker_main(psc_server *S) {
  (void)hipSetDevice(S->opt.device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    // ---- built jobs join at the step boundary ----
    while (!S->ready.empty()) {
      Job *j = S->ready.front();
      S->ready.pop_front();
      if (j->cancel) {
        release_lattice(S, j);
        finish_job(S, j, PSC_JOB_CANCELLED, PSC_OK);
        S->cv_build.notify_one();
        continue;
      }
      j->st.state = PSC_JOB_RUNNING;
      j->st.admit_s = seconds(S);
      S->stats.admitted++;
      S->active.push_back(j);
      S->stats.peak_active = std::max<uint64_t>(S->stats.peak_active, S->active.size());
      S->ens_dirty = true;
    }
    S->stats.active = S->active.size();
    S->stats.queued = S->queue.size();
    S->stats.device_bytes_in_use = S->used_bytes;
    if (S->active.empty()) {
      if (S->stopping && S->queue.empty() && S->ready.empty() && S->building == 0) break;
      S->cv_work.wait(lk);
      continue;
    }
    // ---- one quantum of events for every resident job ----
    if (S->ens_dirty) {
      psc_ensemble &E = S->ens;
      E.members.clear();
      for (Job *j : S->active) E.members.push_back(j->lat);
      E.versions.assign(E.members.size(), ~0ull);
      if (E.members.size() > S->ens_capacity) {
        if (E.d_lats) (void)hipFree(E.d_lats);
        E.d_lats = nullptr;
        S->ens_capacity = std::max<uint64_t>(E.members.size(), 2 * S->ens_capacity);
        if (hipMalloc(&E.d_lats, member_records_bytes((uint32_t)S->ens_capacity)) != hipSuccess) {
          S->err = "device allocation of the member records failed";
          for (Job *j : S->active) {
            release_lattice(S, j);
            finish_job(S, j, PSC_JOB_FAILED, PSC_ENOMEM);
          }
          S->active.clear();
          S->ens_capacity = 0;
          continue;
        }
      }
      uint64_t mol = 0;
      E.stages = 0;
      for (auto *h : E.members) {
        mol += h->desc.max_molecules;
        E.stages = std::max(E.stages, n_colours(h->geo));
      }
      E.grid = (int)std::min<uint64_t>(std::max<uint64_t>(mol / E.stages / 1024, 64), 2048);
      E.items = 4;
      S->ens_dirty = false;
    }
    uint64_t q = S->opt.quantum_events;
    lk.unlock();
    psc_ensemble &E = S->ens;
    psc_status st = ensure_member_records(&E, S->stream, q);
    const bool births = any_births(&E);
    const double tb = seconds(S);
    // direct launches: a server shares its process with other threads, and
    // capturing a graph would forbid their legacy-stream work meanwhile
    for (uint64_t e = 0; e < q && !st; ++e)
      if (launch_event_multi(E.d_lats, (uint32_t)E.members.size(), E.stages, E.grid, E.items,
                             births, S->stream) != hipSuccess)
        st = PSC_EDEVICE;
    if (!st && hipStreamSynchronize(S->stream) != hipSuccess) st = PSC_EDEVICE;
    const double te = seconds(S);
    lk.lock();
    S->stats.quanta++;
    S->stats.busy_s += te - tb;
    // ---- retire finished jobs ----
    std::vector<Job *> still;
    for (Job *j : S->active) {
      psc_lattice *h = j->lat;
      h->events_done = std::min(h->events_done + q, h->L.stop_event);
      if (j->cancel) {
        release_lattice(S, j);
        finish_job(S, j, PSC_JOB_CANCELLED, PSC_OK);
        S->ens_dirty = true;
        continue;
      }
      psc_status js = st;
      if (!js) js = check_device_error(h);
      if (js) {
        release_lattice(S, j);
        finish_job(S, j, PSC_JOB_FAILED, js);
        S->ens_dirty = true;
        continue;
      }
      if (h->events_done < h->L.stop_event) {
        still.push_back(j);
        continue;
      }
      psc_counters c{};
      uint64_t ev = 0;
      psc_read_counters(h, &c, &ev);
      j->st.counters = c;
      j->st.events_done = ev;
      S->stats.attempts += c.attempts;
      if (!j->keep_state) release_lattice(S, j);
      finish_job(S, j, PSC_JOB_DONE, PSC_OK);
      S->ens_dirty = true;
    }
    S->active.swap(still);
    S->cv_build.notify_one();  // memory and slots may have freed
  }
}

}  // namespace

extern "C" {

psc_status psc_server_create(const psc_server_options *opt, psc_server **out) {
  if (!opt || !out) return PSC_EINVAL;
  *out = nullptr;
  if (opt->device < 0 || opt->budget_bytes == 0 || opt->quantum_events == 0 ||
      opt->max_active == 0 || opt->max_active > max_members() || opt->builders > 64)
    return PSC_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || opt->device >= ndev) return PSC_EINVAL;
  psc_server *S = new (std::nothrow) psc_server();
  if (!S) return PSC_ENOMEM;
  S->opt = *opt;
  S->t0 = Clock::now();
  if (hipSetDevice(opt->device) != hipSuccess ||
      hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
    delete S;
    return PSC_EDEVICE;
  }
  S->ens.device = opt->device;
  S->ens.use_graph = false;
  if (S->opt.builders == 0) S->opt.builders = 4;
  S->worker = std::thread(worker_main, S);
  for (uint32_t b = 0; b < S->opt.builders; ++b) S->builders.emplace_back(builder_main, S);
  *out = S;
  return PSC_OK;
}

// device bytes of a job's event tape: per event the due mask (8 B), the
// largest first-order threshold (4 B) and one threshold per first-order
// reaction (4 B each).  The tape grows by doubling from 1024 rows and the
// server asks for a quantum beyond the job's last event, so it ends below
// 2 (n_events + max(quantum, 1024)) rows; superseded tapes stay allocated
// until the lattice is destroyed, at most as many rows again.  Each
// allocation is rounded up to 256 B (three per growth, at most 64 growths).
uint64_t tape_bytes(const psc_job_desc *d, uint32_t quantum) {
  uint32_t n_fo = 0;
  for (uint32_t r = 0; d->reactions && r < d->n_reactions; ++r) n_fo += d->reactions[r].n_r == 1;
  const uint64_t rows = 2 * (d->n_events + std::max<uint64_t>(quantum, 1024));
  return 2 * rows * (12 + 4 * (uint64_t)n_fo) + 64 * 3 * 256;
}

uint64_t job_bytes(const psc_job_desc *d, uint32_t quantum) {
  const uint64_t nv = (uint64_t)d->ni * d->nj * d->nk;
  bool collision_births = false;
  for (uint32_t r = 0; d->reactions && r < d->n_reactions; ++r)
    collision_births |= d->reactions[r].n_r == 2 && d->reactions[r].n_p > 2;
  return estimate_device_bytes(nv, d->max_molecules, (d->flags & PSC_TRACK_DISPLACEMENT) != 0,
                               d->n_reactions, collision_births,
                               (d->flags & PSC_LATTICE_FCC) ? kColoursFcc : kColoursHcp) +
         tape_bytes(d, quantum);
}

psc_status psc_server_start(uint64_t budget_bytes, int32_t device, psc_server **out) {
  const psc_server_options o{device, budget_bytes, 64, 1024, 4};
  return psc_server_create(&o, out);
}

psc_status psc_server_job_bytes(const psc_job_desc *d, uint64_t *bytes) {
  if (!d || !bytes) return PSC_EINVAL;
  *bytes = job_bytes(d, 1024);
  return PSC_OK;
}

psc_status psc_server_submit(psc_server *S, const psc_job_desc *d, uint64_t *job_id) {
  if (!S || !d || !job_id) return PSC_EINVAL;
  Job *j = new (std::nothrow) Job();
  if (!j) return PSC_ENOMEM;
  j->desc.ni = d->ni;
  j->desc.nj = d->nj;
  j->desc.nk = d->nk;
  j->desc.voxel_radius = d->voxel_radius;
  j->desc.seed = d->seed;
  j->desc.max_molecules = d->max_molecules;
  j->desc.flags = d->flags;
  j->desc.device = S->opt.device;
  if (d->n_species && d->D) j->D.assign(d->D, d->D + d->n_species);
  if (d->n_reactions && d->reactions) j->rx.assign(d->reactions, d->reactions + d->n_reactions);
  if (d->n_place && d->place) j->place.assign(d->place, d->place + d->n_place);
  j->n_events = d->n_events;
  j->keep_state = d->keep_state != 0;
  j->est_bytes = job_bytes(d, S->opt.quantum_events);
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stopping) {
    delete j;
    return PSC_ESTATE;
  }
  j->id = S->next_job++;
  j->st.state = PSC_JOB_QUEUED;
  j->st.submit_s = seconds(S);
  S->jobs[j->id] = j;
  S->stats.submitted++;
  if (j->est_bytes > S->opt.budget_bytes) {
    // can never fit: rejected at once, the others are unaffected
    finish_job(S, j, PSC_JOB_FAILED, PSC_ENOMEM);
  } else {
    S->queue.push_back(j);
    S->stats.queued = S->queue.size();
    S->cv_build.notify_one();
  }
  *job_id = j->id;
  return PSC_OK;
}

psc_status psc_server_poll(psc_server *S, uint64_t job_id, psc_job_status *out) {
  if (!S || !out) return PSC_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->jobs.find(job_id);
  if (it == S->jobs.end()) return PSC_EINVAL;
  *out = it->second->st;
  return PSC_OK;
}

psc_status psc_server_wait(psc_server *S, uint64_t job_id, psc_job_status *out) {
  if (!S) return PSC_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(job_id);
  if (it == S->jobs.end()) return PSC_EINVAL;
  Job *j = it->second;
  S->cv_done.wait(lk, [&] {
    return j->st.state == PSC_JOB_DONE || j->st.state == PSC_JOB_FAILED ||
           j->st.state == PSC_JOB_CANCELLED;
  });
  if (out) *out = j->st;
  return PSC_OK;
}

psc_status psc_server_read_state(psc_server *S, uint64_t job_id, psc_state_view *out) {
  if (!S || !out) return PSC_EINVAL;
  psc_lattice *h = nullptr;
  {
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->jobs.find(job_id);
    if (it == S->jobs.end()) return PSC_EINVAL;
    if (it->second->st.state != PSC_JOB_DONE || !it->second->lat) return PSC_ESTATE;
    h = it->second->lat;
  }
  return psc_read_state(h, out, nullptr);
}

psc_status psc_server_cancel(psc_server *S, uint64_t job_id) {
  if (!S) return PSC_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->jobs.find(job_id);
  if (it == S->jobs.end()) return PSC_EINVAL;
  Job *j = it->second;
  const int state = j->st.state;
  if (state == PSC_JOB_DONE || state == PSC_JOB_FAILED || state == PSC_JOB_CANCELLED || j->cancel)
    return PSC_ESTATE;
  auto q = std::find(S->queue.begin(), S->queue.end(), j);
  if (q != S->queue.end()) {
    // still waiting for admission: it never holds memory
    S->queue.erase(q);
    S->stats.queued = S->queue.size();
    finish_job(S, j, PSC_JOB_CANCELLED, PSC_OK);
    return PSC_OK;
  }
  // being built, ready or running: retired at the next step boundary (or
  // once built)
  j->cancel = true;
  S->cv_work.notify_one();
  return PSC_OK;
}

psc_status psc_server_release(psc_server *S, uint64_t job_id) {
  if (!S) return PSC_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->jobs.find(job_id);
  if (it == S->jobs.end()) return PSC_EINVAL;
  if (it->second->st.state != PSC_JOB_DONE && it->second->st.state != PSC_JOB_FAILED &&
      it->second->st.state != PSC_JOB_CANCELLED)
    return PSC_ESTATE;
  release_lattice(S, it->second);
  S->cv_build.notify_one();
  return PSC_OK;
}

psc_status psc_server_stats_get(psc_server *S, psc_server_stats *out) {
  if (!S || !out) return PSC_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  *out = S->stats;
  return PSC_OK;
}

const char *psc_server_last_error(const psc_server *S) { return S ? S->err.c_str() : ""; }

void psc_server_destroy(psc_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stopping = true;
    S->cv_work.notify_all();
    S->cv_build.notify_all();
  }
  for (auto &t : S->builders)
    if (t.joinable()) t.join();
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->cv_work.notify_all();  // the worker may wait for the last built job
  }
  if (S->worker.joinable()) S->worker.join();
  (void)hipSetDevice(S->opt.device);
  if (S->ens.exec) (void)hipGraphExecDestroy(S->ens.exec);
  if (S->ens.graph) (void)hipGraphDestroy(S->ens.graph);
  if (S->ens.cap_stream) (void)hipStreamDestroy(S->ens.cap_stream);
  if (S->ens.d_lats) (void)hipFree(S->ens.d_lats);
  S->ens.members.clear();
  for (auto &kv : S->jobs) {
    if (kv.second->lat) psc_destroy(kv.second->lat);
    delete kv.second;
  }
  if (S->stream) (void)hipStreamDestroy(S->stream);
  delete S;
}

}  // extern "C"
