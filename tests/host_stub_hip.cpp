// Test helper (host only): the HIP runtime calls of libpsc's host code
// answered from host memory, and the kernel launchers replaced by host
// checks, so that psc_host.cpp and psc_server.cpp can run on the CPU under
// AddressSanitizer.  "Device" buffers are ordinary heap blocks: every copy
// and fill the host code makes into or out of them is bounds-checked by the
// sanitizer, and every launch checks its arguments against the lattice
// record.  Not part of the library.
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <mutex>
#include <set>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "psc_core.h"

// the serving loop launches from two threads
static std::atomic<int> g_launch_errors{0};
static std::atomic<unsigned long long> g_launches{0};
// lattices whose last directly launched event left its end to the next
// event's opening
static std::mutex g_open_mu;
static std::set<const psc::LatDev *> g_open_ends;
static std::atomic<unsigned long long> g_fused_openings{0};

static void bad(const char *what) {
  fprintf(stderr, "launch check failed: %s\n", what);
  ++g_launch_errors;
}

extern "C" {

int stub_launch_errors() { return g_launch_errors.load(); }
// lattices whose event end is still left open (every step must close its last event)
int stub_open_ends();
unsigned long long stub_launches() { return g_launches.load(); }

hipError_t hipMalloc(void **p, size_t n) {
  *p = calloc(1, n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p) {
  free(p);
  return hipSuccess;
}
hipError_t hipMallocAsync(void **p, size_t n, hipStream_t) { return hipMalloc(p, n); }
hipError_t hipFreeAsync(void *p, hipStream_t) { return hipFree(p); }
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
  memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) {
  memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemset(void *d, int v, size_t n) {
  memset(d, v, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) {
  memset(d, v, n);
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDeviceCount(int *n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  *s = (hipStream_t)malloc(16);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  free((void *)s);
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) {
  *e = (hipEvent_t)malloc(16);
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  free((void *)e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventQuery(hipEvent_t e) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipHostMalloc(void **p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void *p) { return hipFree(p); }
hipError_t hipEventSynchronize(hipEvent_t e) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
  *ms = 0.01f;
  return a && b ? hipSuccess : hipErrorInvalidValue;
}
const char *hipGetErrorString(hipError_t) { return "stub"; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
  *g = (hipGraph_t)malloc(16);
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t, hipGraphNode_t *, char *, size_t) {
  *x = (hipGraphExec_t)malloc(16);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) { return x ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGraphDestroy(hipGraph_t g) {
  free((void *)g);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  free((void *)x);
  return hipSuccess;
}

}  // extern "C"

namespace psc {

// every array of the record the kernels index by colour or stage holds
// kMaxColours entries; touching the last one makes the sanitizer check it
static void check_record(const LatDev *L) {
  if (!L) return bad("null record");
  if (L->ncol == 0 || L->ncol > (uint32_t)kMaxColours) bad("colour count");
  volatile uint32_t x = 0;
  x += L->perm[kMaxColours - 1];
  x += L->sdesc[kMaxColours - 1].x;
  for (int b = 0; b < 2; ++b) x += L->bins[b].count[kMaxColours - 1];
  x += L->cnt[kStatRep * kCntStride - 1] != 0;
  x += L->sp_count[kStatRep * kSpStride - 1] != 0;
  x += L->fired[(uint64_t)kStatRep * L->fired_stride - 1] != 0;
  x += L->hot[(1ull << L->hot_bits) / 16 - 1];
  x += L->nbr_cnt[(1ull << L->nbr_bits) - 1];
  x += (uint32_t)L->tape_due[L->tape_horizon - 1];
  x += L->tape_cmax[L->tape_horizon - 1];
  x += L->recent[kRecentN - 1];
  x += L->fire_vox[L->cap - 1];
  x += L->stage_tab[L->stage_tab_words - 1];
  if (L->n_fo) x += L->tape_thr[L->tape_horizon * L->n_fo - 1];
  (void)x;
}

hipError_t launch_scan(const LatDev *dL, int grid, hipStream_t) {
  ++g_launches;
  if (grid < 1 || grid > 65536) bad("scan grid");
  check_record(dL);
  return hipSuccess;
}
hipError_t launch_begin(const LatDev *dL, const BeginShape &b, uint32_t stages, hipStream_t, bool,
                        const LatDev *Lh, const uint32_t *perm, uint64_t e) {
  {
    std::lock_guard<std::mutex> g(g_open_mu);
    if (g_open_ends.count(dL)) bad("an opening launched while the last event's end is left open");
  }
  if (Lh && std::memcmp(dL, Lh, sizeof(LatDev)) != 0) bad("stale host record at begin");
  if (Lh && (!perm || e >= Lh->tape_horizon)) bad("first-order stage arguments");
  if (perm)
    for (uint32_t g = 0; g < stages; ++g)
      if (perm[g] >= (uint32_t)kMaxColours) bad("stage order");
  ++g_launches;
  if (b.decide < 0 || b.decide > 1024) bad("decide grid");
  if (b.births < 0 || b.births > 2048) bad("births grid");
  if (b.apply < 0 || b.apply > 1024) bad("apply grid");
  if (stages == 0 || stages > (uint32_t)kMaxColours) bad("stages");
  check_record(dL);
  return hipSuccess;
}
hipError_t launch_stage(const LatDev *dL, uint32_t g, int grid, int items, bool, bool,
                        hipStream_t) {
  ++g_launches;
  if (g >= (uint32_t)kMaxColours) bad("stage index");
  if (grid < 1 || grid > 65536) bad("stage grid");
  if (items != 1 && items != 2 && items != 4 && items != 8 && items != 16) bad("items");
  check_record(dL);
  return hipSuccess;
}
hipError_t launch_end(const LatDev *dL, bool births, hipStream_t, bool) {
  if (births != (dL->wb_count != nullptr)) bad("end births");
  ++g_launches;
  check_record(dL);
  return hipSuccess;
}
hipError_t launch_event(const LatDev *dL, int grid, int items, bool disp, bool fcc,
                        const BeginShape &b, bool births, hipStream_t s) {
  launch_begin(dL, b, kMaxColours, s);
  for (uint32_t g = 0; g < (uint32_t)kMaxColours; ++g) launch_stage(dL, g, grid, items, disp, fcc, s);
  return launch_end(dL, births, s);
}
hipError_t launch_stage_direct(const LatDev &L, uint32_t c, uint64_t e, uint64_t due,
                               uint32_t cmax_next, int grid, int items, bool, bool, hipStream_t) {
  ++g_launches;
  if (c >= (uint32_t)kMaxColours) bad("stage colour");
  if (e >= L.tape_horizon) bad("stage event beyond the tape");
  // the tape words must be those on the device
  if (due != L.tape_due[e]) bad("stage due word");
  if (cmax_next != ((L.n_fo && e + 1 < L.tape_horizon) ? L.tape_cmax[e + 1] : 0u))
    bad("stage next-event threshold");
  if (grid < 1 || grid > 65536) bad("stage grid");
  if (items != 1 && items != 2 && items != 4) bad("direct items");
  check_record(&L);
  return hipSuccess;
}
static bool take_open_end(const LatDev *dL) {
  std::lock_guard<std::mutex> g(g_open_mu);
  return g_open_ends.erase(dL) != 0;
}
hipError_t launch_event_direct(const LatDev *dL, const LatDev &L, uint64_t e, uint64_t due,
                               uint32_t cmax_next, int grid, int items, bool disp, bool fcc,
                               const BeginShape &b, bool births, bool births_defer,
                               hipStream_t s, bool open_with_end, bool close) {
  // the record handed to the stages by value must be the one on the device
  if (std::memcmp(dL, &L, sizeof(LatDev)) != 0) bad("stale host record");
  // an end left open is picked up by the very next event, and only then
  if (take_open_end(dL) != open_with_end) bad("event end left open or picked up out of turn");
  uint32_t perm[kMaxColours];
  stage_order_of(L.key0, L.key1, e, kMaxColours, perm);
  if (open_with_end) {
    if (births || b.decide || b.births || b.apply) bad("fused end and opening with launches of their own");
    ++g_fused_openings;
    ++g_launches;
    check_record(dL);
  } else {
    launch_begin(dL, b, kMaxColours, s, items > 4, &L, perm, e);
  }
  for (uint32_t g = 0; g < (uint32_t)kMaxColours; ++g) {
    if (items <= 4) launch_stage_direct(L, perm[g], e, due, cmax_next, grid, items, disp, fcc, s);
    else launch_stage(dL, g, grid, items, disp, fcc, s);
  }
  if (close) return launch_end(dL, births, s, births_defer);
  std::lock_guard<std::mutex> g(g_open_mu);
  g_open_ends.insert(dL);
  return hipSuccess;
}
hipError_t launch_event_multi(const LatDev *lats, uint32_t R, uint32_t stages, int grid,
                              int items, bool births, hipStream_t) {
  ++g_launches;
  if (R == 0 || R > 4096 || stages > (uint32_t)kMaxColours || grid < 1 || items < 1) bad("multi");
  bool any = false;
  for (uint32_t r = 0; r < R; ++r) {
    check_record(&lats[r]);
    any |= lats[r].wb_count != nullptr;
  }
  if (births != any) bad("multi births");
  return hipSuccess;
}
hipError_t launch_msd(const LatDev *dL, unsigned long long *out, hipStream_t) {
  ++g_launches;
  check_record(dL);
  out[0] = 0;
  out[1] = 0;
  return hipSuccess;
}
// the conversion itself, on the host: the buffers must hold nv words
hipError_t launch_relayout(const Geo &g, uint64_t nv, const uint16_t *src, uint16_t *dst,
                           bool to_layout_order, hipStream_t) {
  ++g_launches;
  for (uint64_t u = 0; u < nv; ++u) {
    const uint32_t lin = linear_of(g, coord_of(g, (uint32_t)u));
    if (to_layout_order) dst[u] = src[lin];
    else dst[lin] = src[u];
  }
  return hipSuccess;
}
uint32_t max_members() { return 4096; }
int stage_items() { return 4; }
int stage_threads() { return 256; }

}  // namespace psc

extern "C" unsigned long long stub_fused_openings() { return g_fused_openings.load(); }

extern "C" int stub_open_ends() {
  std::lock_guard<std::mutex> g(g_open_mu);
  return (int)g_open_ends.size();
}
