// psc_host.cpp -- host core of libpsc: model registry, the FP64 -> uint32
// "freeze" of every probability, the diffusion-event tape, uniform placement,
// state upload / read-back, and the C ABI declared in include/psc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "psc_internal.h"

using namespace psc;
using namespace psc_detail;

static_assert(kMaxReactions == PSC_MAX_REACTIONS && kMaxSpecies == PSC_MAX_SPECIES &&
                  kMaxProducts == PSC_MAX_PRODUCTS,
              "the kernels' limits are the ABI's");

namespace {

thread_local std::string g_create_error;


// interval between diffusion events of a species, tau = 2 r^2 / (3 D) (2.3)
double diffusion_interval(double rv, double D) {
  double num = 2.0 * rv;
  num = num * rv;
  const double den = 3.0 * D;
  return num / den;
}

// collision reaction probability, p = k / (6 sqrt2 (DA + DB) r) (2.4.2, eq. 6),
// as a threshold on a uniform 32-bit word: fire iff r1 < thr, or always
void second_order_threshold(double k, double DA, double DB, double rv, uint32_t *thr,
                            uint8_t *always) {
  double den = 6.0 * std::sqrt(2.0);
  den = den * (DA + DB);
  den = den * rv;
  const double p = k / den;
  if (p >= 1.0) {
    *thr = 0xFFFFFFFFu;
    *always = 1;
    return;
  }
  *always = 0;
  *thr = p > 0.0 ? (uint32_t)std::floor(p * 4294967296.0) : 0u;
}

// probability -> threshold on a uniform 32-bit word (capped at 2^32 - 1)
uint32_t prob_threshold(double p) {
  if (!(p > 0.0)) return 0u;
  const double x = p * 4294967296.0;
  if (x >= 4294967295.0) return 0xFFFFFFFFu;
  return (uint32_t)std::floor(x);
}

// words per replica of the per-reaction firing counters: the reactions
// rounded up to a whole 128-byte line
uint32_t fired_stride(uint32_t n_rx) { return (std::max<uint32_t>(n_rx, 1) + 15u) & ~15u; }

uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

}  // namespace


namespace psc_detail {

psc_status fail(psc_lattice *h, psc_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  h->err = buf;
  if (code == PSC_EDEVICE) h->poisoned = true;
  return code;
}

#define HIP_OK(h, call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail((h), PSC_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// A transient device buffer, freed when the scope ends (also on the early
// returns of a failed HIP call).  Stream-ordered: allocated and freed in the
// order of `stream`, so that neither waits for work on other streams (a
// plain hipFree waits for the whole device -- in the serving loop, for the
// batched step running meanwhile).
struct DevTemp {
  void *p = nullptr;
  hipStream_t stream = nullptr;
  explicit DevTemp(hipStream_t s = nullptr) : stream(s) {}
  ~DevTemp() {
    if (p) (void)hipFreeAsync(p, stream);
  }
  hipError_t alloc(size_t bytes) { return hipMallocAsync(&p, bytes, stream); }
};

void *dev_alloc(psc_lattice *h, size_t bytes) {
  if (bytes == 0) bytes = 16;
  bytes = (bytes + 255) & ~size_t(255);
  void *p = nullptr;
  if (h->desc.alloc) {
    p = h->desc.alloc(bytes, nullptr, h->desc.alloc_user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) {
    h->blocks.push_back({p, bytes});
    h->device_bytes += bytes;
  }
  return p;
}

void dev_free_all(psc_lattice *h) {
  for (auto &b : h->blocks) {
    if (h->desc.free) h->desc.free(b.p, h->desc.alloc_user);
    else (void)hipFree(b.p);
  }
  h->blocks.clear();
  h->device_bytes = 0;
}

bool mobile(const psc_lattice *h, uint16_t s) { return h->species[s].D > 0.0; }

// ---- the event tape ---------------------------------------------------------
// Next event time t_e = min over mobile species of (n_s + 1) tau_s, computed
// by multiplication (no accumulated drift); due species are those attaining
// it (2.2).  For each first-order species, the chance that one molecule reacts
// during dt_e = t_e - t_{e-1} is q = 1 - exp(-K dt) (K = sum of its rate
// constants, eq. 4 with the propensity of one molecule), shared among its
// reactions in proportion to k_j (eq. 5); the cumulative sums become 32-bit
// thresholds.
void extend_tape(psc_lattice *h, uint64_t end) {
  const size_t S = h->species.size();
  if (h->n_walks.size() != S) h->n_walks.assign(S, 0);
  while (h->tape_end < end) {
    double tmin = std::numeric_limits<double>::infinity();
    for (size_t s = 1; s < S; ++s) {
      if (!mobile(h, (uint16_t)s)) continue;
      const double ts = (double)(h->n_walks[s] + 1) * h->species[s].tau;
      if (ts < tmin) tmin = ts;
    }
    uint64_t due = 0;
    for (size_t s = 1; s < S; ++s) {
      if (!mobile(h, (uint16_t)s)) continue;
      if ((double)(h->n_walks[s] + 1) * h->species[s].tau == tmin) due |= 1ull << s;
    }
    const double dt = tmin - h->t_prev;
    uint32_t cmax = 0;
    for (size_t s = 1; s < S; ++s) {
      const uint32_t n = h->fo_n[s];
      if (!n) continue;
      double K = 0.0;
      for (uint32_t a = 0; a < n; ++a) K += h->rx[h->fo_rx[h->fo_first[s] + a]].k;
      const double q = -std::expm1(-K * dt);
      double acc = 0.0;
      uint32_t C = 0;
      for (uint32_t a = 0; a < n; ++a) {
        const double kj = h->rx[h->fo_rx[h->fo_first[s] + a]].k;
        acc = acc + q * kj / K;
        C = prob_threshold(acc);
        h->tape_thr.push_back(C);
      }
      cmax = std::max(cmax, C);
    }
    h->tape_due.push_back(due);
    h->tape_cmax.push_back(cmax);
    h->tape_time.push_back(tmin);
    for (size_t s = 1; s < S; ++s)
      if ((due >> s) & 1ull) h->n_walks[s]++;
    h->t_prev = tmin;
    h->tape_end++;
  }
}

// time of the last of the first e events (the clock alone, before the freeze)
double clock_time(const psc_lattice *h, uint64_t e) {
  const size_t S = h->species.size();
  std::vector<uint64_t> nw(S, 0);
  double t = 0.0;
  for (uint64_t z = 0; z < e; ++z) {
    double tmin = std::numeric_limits<double>::infinity();
    for (size_t s = 1; s < S; ++s)
      if (mobile(h, (uint16_t)s)) tmin = std::min(tmin, (double)(nw[s] + 1) * h->species[s].tau);
    if (tmin == std::numeric_limits<double>::infinity()) return 0.0;
    for (size_t s = 1; s < S; ++s)
      if (mobile(h, (uint16_t)s) && (double)(nw[s] + 1) * h->species[s].tau == tmin) nw[s]++;
    t = tmin;
  }
  return t;
}

// uploads tape rows [0, tape_end) when the device copy is too short
psc_status sync_tape(psc_lattice *h, hipStream_t stream) {
  if (h->d_tape_rows >= h->tape_end) return PSC_OK;
  HIP_OK(h, hipStreamSynchronize(stream));
  const uint64_t rows = h->tape_end;
  auto *due = (uint64_t *)dev_alloc(h, rows * sizeof(uint64_t));
  auto *thr = (uint32_t *)dev_alloc(h, std::max<uint64_t>(1, rows * h->n_fo) * sizeof(uint32_t));
  auto *cmax = (uint32_t *)dev_alloc(h, rows * sizeof(uint32_t));
  if (!due || !thr || !cmax) return fail(h, PSC_ENOMEM, "tape allocation failed");
  HIP_OK(h, hipMemcpy(due, h->tape_due.data(), rows * sizeof(uint64_t), hipMemcpyHostToDevice));
  if (h->n_fo)
    HIP_OK(h, hipMemcpy(thr, h->tape_thr.data(), rows * h->n_fo * sizeof(uint32_t),
                        hipMemcpyHostToDevice));
  HIP_OK(h, hipMemcpy(cmax, h->tape_cmax.data(), rows * sizeof(uint32_t), hipMemcpyHostToDevice));
  // the previous tape stays allocated until destroy (it is small and may
  // still be referenced by work captured earlier)
  h->d_tape_due = due;
  h->d_tape_thr = thr;
  h->d_tape_cmax = cmax;
  h->d_tape_rows = rows;
  h->L.tape_due = due;
  h->L.tape_thr = thr;
  h->L.tape_cmax = cmax;
  h->L.tape_horizon = rows;
  HIP_OK(h, hipMemcpy(h->dL, &h->L, sizeof(LatDev), hipMemcpyHostToDevice));
  h->version++;
  return PSC_OK;
}

template <class T>
T *alloc_n(psc_lattice *h, uint64_t n) {
  return (T *)dev_alloc(h, (size_t)std::max<uint64_t>(n, 1) * sizeof(T));
}

// ---- freeze: model tables, buffers, upload ---------------------------------------
psc_status freeze(psc_lattice *h, hipStream_t stream) {
  const size_t S = h->species.size();
  bool any_mobile = false;
  for (size_t s = 1; s < S; ++s) any_mobile |= mobile(h, (uint16_t)s);
  if (!any_mobile) return fail(h, PSC_EINVAL, "no mobile species: no diffusion events");

  // model tables
  std::vector<uint8_t> sp_flags(64, 0);
  std::vector<int16_t> pair(64 * 64, -1);
  const uint32_t R = (uint32_t)h->rx.size();
  std::vector<uint32_t> thr(std::max<uint32_t>(R, 1), 0);
  std::vector<uint8_t> always(std::max<uint32_t>(R, 1), 0), nprod(std::max<uint32_t>(R, 1), 0);
  std::vector<uint16_t> prod(std::max<uint32_t>(R, 1) * 12, 0);
  std::vector<bool> reactant(S, false);
  h->fo_first.assign(64, 0);
  h->fo_n.assign(64, 0);
  h->fo_rx.clear();
  for (size_t s = 1; s < S; ++s) {
    if (mobile(h, (uint16_t)s)) sp_flags[s] |= kSpMobile;
    h->fo_first[s] = (uint16_t)h->fo_rx.size();
    for (uint32_t r = 0; r < R; ++r)
      if (h->rx[r].nr == 1 && h->rx[r].r[0] == s) {
        h->fo_rx.push_back((uint16_t)r);
        h->fo_n[s]++;
      }
    if (h->fo_n[s]) sp_flags[s] |= kSpFirstOrder;
  }
  h->n_fo = (uint32_t)h->fo_rx.size();
  h->fo_extra_max = 0;
  for (uint32_t r = 0; r < R; ++r)
    if (h->rx[r].nr == 1 && h->rx[r].np > 1)
      h->fo_extra_max = std::max<uint32_t>(h->fo_extra_max, h->rx[r].np - 1);
  for (uint32_t r = 0; r < R; ++r) {
    const ReactionDef &d = h->rx[r];
    nprod[r] = (uint8_t)d.np;
    for (uint32_t a = 0; a < d.np; ++a) prod[r * 12 + a] = d.p[a];
    for (uint32_t a = 0; a < d.nr; ++a) reactant[d.r[a]] = true;
    if (d.nr == 2) {
      const uint16_t A = d.r[0], B = d.r[1];
      pair[A * 64 + B] = pair[B * 64 + A] = (int16_t)r;
      second_order_threshold(d.k, h->species[A].D, h->species[B].D, h->desc.voxel_radius,
                             &thr[r], &always[r]);
    }
  }

  // split molecules into the walk's bins and the static list
  Geo lin_geo = h->geo;  // decodes the ABI's linear indices
  lin_geo.brick = 0;
  h->st_id.clear();
  h->st_vox.clear();
  for (auto &d : h->st_d) d.clear();
  const uint64_t nmol = h->mid.size();
  std::vector<uint8_t> colour(nmol);
  const uint32_t ncol = n_colours(h->geo);
  uint64_t bin_count[kMaxColours] = {0};
  std::vector<uint64_t> walkers;
  walkers.reserve(nmol);
  for (uint64_t q = 0; q < nmol; ++q) {
    const uint16_t s = h->occ[h->mvox[q]];
    if (!mobile(h, s) && !reactant[s]) {
      h->st_id.push_back(h->mid[q]);
      h->st_vox.push_back(h->mvox[q]);
      h->st_d[0].push_back(h->mdx[q]);
      h->st_d[1].push_back(h->mdy[q]);
      h->st_d[2].push_back(h->mdz[q]);
      continue;
    }
    colour[q] = (uint8_t)colour_of(lin_geo, coord_of(lin_geo, h->mvox[q]));
    bin_count[colour[q]]++;
    walkers.push_back(q);
  }

  // buffers
  const uint64_t cap = std::max<uint64_t>(h->desc.max_molecules, 1);
  const bool disp = (h->desc.flags & PSC_TRACK_DISPLACEMENT) != 0;
  LatDev &L = h->L;
  L.stop_event = ~0ull;
  L.geo = h->geo;
  L.nv = h->nv;
  L.key0 = (uint32_t)h->desc.seed;
  L.key1 = (uint32_t)(h->desc.seed >> 32);
  L.occ = alloc_n<uint16_t>(h, h->nv);
  L.cap = cap;
  L.ncol = ncol;
  for (int b = 0; b < 2; ++b) {
    L.bins[b].vox = alloc_n<uint32_t>(h, ncol * cap);
    L.bins[b].id = alloc_n<uint32_t>(h, ncol * cap);
    L.bins[b].sp = alloc_n<uint16_t>(h, ncol * cap);
    L.bins[b].disp = disp ? alloc_n<int32_t>(h, 3 * ncol * cap) : nullptr;
    L.bins[b].count = alloc_n<uint32_t>(h, kMaxColours);
    L.cand_pos[b] = alloc_n<uint32_t>(h, cap);
    L.cand_id[b] = alloc_n<uint32_t>(h, cap);
    L.cand_col[b] = alloc_n<uint8_t>(h, cap);
    if (!L.bins[b].vox || !L.bins[b].id || !L.bins[b].sp || (disp && !L.bins[b].disp) ||
        !L.bins[b].count ||
        !L.cand_pos[b] || !L.cand_id[b] || !L.cand_col[b])
      return fail(h, PSC_ENOMEM, "device allocation of molecule bins failed");
  }
  L.cand_count = alloc_n<uint32_t>(h, 2);
  L.cand_cap = cap;
  L.flag_vox[0] = alloc_n<uint32_t>(h, cap);
  L.flag_vox[1] = alloc_n<uint32_t>(h, cap);
  L.flag_count = alloc_n<uint32_t>(h, 2);
  L.flag_cap = cap;
  L.birth_cap = std::min<uint64_t>(pow2_at_least(cap), 1ull << 27);
  L.birth_key = alloc_n<uint64_t>(h, L.birth_cap);
  L.birth_vox = alloc_n<uint32_t>(h, L.birth_cap);
  L.birth_sp = alloc_n<uint16_t>(h, L.birth_cap);
  L.birth_count = alloc_n<uint32_t>(h, 1);
  bool collision_births = false;
  for (const auto &d : h->rx) collision_births |= d.nr == 2 && d.np > 2;
  if (collision_births) {
    L.wb_cap = L.birth_cap;
    L.wb_vox = alloc_n<uint32_t>(h, L.wb_cap);
    L.wb_key = alloc_n<uint64_t>(h, L.wb_cap);
    L.wb_count = alloc_n<uint32_t>(h, 1);
  }
  if (collision_births || h->fo_extra_max) {
    L.rank_hist = alloc_n<uint32_t>(h, kRankBucketsMax);
    L.rank_off = alloc_n<uint32_t>(h, kRankBucketsMax + 1);
    L.rank_keys = alloc_n<uint64_t>(h, L.birth_cap);
    if (!L.rank_hist || !L.rank_off || !L.rank_keys)
      return fail(h, PSC_ENOMEM, "device allocation of the newborn ranking failed");
  }
  {
    uint32_t bits = 16;
    while (bits < 24 && (1ull << bits) < cap / 4) ++bits;
    L.hot_bits = bits;
  }
  L.hot = alloc_n<uint32_t>(h, (1ull << L.hot_bits) / 16);
  L.end_done = alloc_n<uint32_t>(h, 1);
  L.nbr_bits = 12;
  while (L.nbr_bits < 22 && (1ull << L.nbr_bits) < 8 * cap) ++L.nbr_bits;
  L.nbr_cnt = alloc_n<uint32_t>(h, 1ull << L.nbr_bits);
  L.fire_pos = alloc_n<uint32_t>(h, cap);
  L.fire_vox = alloc_n<uint32_t>(h, cap);
  L.fire_id = alloc_n<uint32_t>(h, cap);
  L.fire_col = alloc_n<uint8_t>(h, cap);
  L.fire_rx = alloc_n<uint8_t>(h, cap);
  L.fire_count = alloc_n<uint32_t>(h, 1);
  L.recent = alloc_n<uint32_t>(h, kRecentN);
  L.n_species = (uint32_t)(S - 1);
  L.n_rx = R;
  L.n_fo = h->n_fo;
  auto *d_flags = alloc_n<uint8_t>(h, 64);
  auto *d_pair = alloc_n<int16_t>(h, 64 * 64);
  auto *d_thr = alloc_n<uint32_t>(h, thr.size());
  auto *d_always = alloc_n<uint8_t>(h, always.size());
  auto *d_nprod = alloc_n<uint8_t>(h, nprod.size());
  auto *d_prod = alloc_n<uint16_t>(h, prod.size());
  const StageTabLayout tl = stage_tab_layout((uint32_t)(S - 1), R);
  auto *d_tab = alloc_n<uint32_t>(h, tl.words);
  auto *d_fo_first = alloc_n<uint16_t>(h, 64);
  auto *d_fo_n = alloc_n<uint8_t>(h, 64);
  auto *d_fo_rx = alloc_n<uint16_t>(h, std::max<size_t>(h->fo_rx.size(), 1));
  L.ev = alloc_n<uint64_t>(h, 1);
  L.perm = alloc_n<uint32_t>(h, kMaxColours);
  L.sdesc = alloc_n<uint4>(h, kMaxColours);
  L.next_id = alloc_n<uint32_t>(h, 1);
  L.cnt = alloc_n<unsigned long long>(h, kStatRep * kCntStride);
  L.sp_count = alloc_n<unsigned long long>(h, kStatRep * kSpStride);
  L.fired_stride = fired_stride(R);
  L.fired = alloc_n<unsigned long long>(h, (uint64_t)kStatRep * L.fired_stride);
  L.error = alloc_n<uint32_t>(h, 1);
  h->dL = alloc_n<LatDev>(h, 1);
  if (!L.occ || !L.cand_count || !L.flag_vox[0] || !L.flag_vox[1] || !L.flag_count || !L.birth_key || !L.birth_vox ||
      !L.birth_sp || !L.birth_count || !L.fire_pos || !L.fire_id || !L.fire_col || !L.fire_count ||
      !L.fire_rx || !L.fire_vox || !L.recent || !d_flags || !d_pair || !d_thr || !d_always || !d_nprod ||
      !d_prod || !d_tab ||
      !d_fo_first || !d_fo_n || !d_fo_rx || !L.ev || !L.perm || !L.sdesc || !L.next_id || !L.cnt || !L.sp_count ||
      !L.fired || !L.error || !h->dL || !L.hot || !L.end_done || !L.nbr_cnt ||
      (collision_births && (!L.wb_vox || !L.wb_key || !L.wb_count)))
    return fail(h, PSC_ENOMEM, "device allocation failed");
  L.sp_flags = d_flags;
  L.pair_rx = d_pair;
  L.rx_thr = d_thr;
  L.rx_always = d_always;
  L.rx_nprod = d_nprod;
  L.rx_prod = d_prod;
  L.stage_tab = d_tab;
  L.stage_tab_words = tl.words;
  L.fo_first = d_fo_first;
  L.fo_n = d_fo_n;
  L.fo_rx = d_fo_rx;

  auto up = [&](void *dst, const void *src, size_t bytes) {
    return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  };
  HIP_OK(h, up(d_flags, sp_flags.data(), 64));
  HIP_OK(h, up(d_pair, pair.data(), pair.size() * sizeof(int16_t)));
  HIP_OK(h, up(d_thr, thr.data(), thr.size() * sizeof(uint32_t)));
  HIP_OK(h, up(d_always, always.data(), always.size()));
  HIP_OK(h, up(d_nprod, nprod.data(), nprod.size()));
  HIP_OK(h, up(d_prod, prod.data(), prod.size() * sizeof(uint16_t)));
  {
    std::vector<uint32_t> tab(tl.words, 0);
    std::memcpy(tab.data() + tl.pair, pair.data(), S * 64 * sizeof(int16_t));
    if (R) {
      std::memcpy(tab.data() + tl.thr, thr.data(), R * sizeof(uint32_t));
      std::memcpy(tab.data() + tl.prod, prod.data(), R * 12 * sizeof(uint16_t));
      std::memcpy(tab.data() + tl.nprod, nprod.data(), R);
      std::memcpy(tab.data() + tl.always, always.data(), R);
    }
    HIP_OK(h, up(d_tab, tab.data(), tab.size() * sizeof(uint32_t)));
  }
  HIP_OK(h, up(d_fo_first, h->fo_first.data(), 64 * sizeof(uint16_t)));
  HIP_OK(h, up(d_fo_n, h->fo_n.data(), 64));
  if (!h->fo_rx.empty()) HIP_OK(h, up(d_fo_rx, h->fo_rx.data(), h->fo_rx.size() * sizeof(uint16_t)));
  // the device words carry the compartment of every voxel beside its species
  // (the host copy keeps species only: a failed freeze leaves it unchanged)
  std::vector<uint16_t> with_comp;
  const uint16_t *words = h->occ.data();
  if (!h->comp.empty()) {
    with_comp.resize(h->nv);
    for (uint64_t v = 0; v < h->nv; ++v)
      with_comp[v] = (uint16_t)(h->occ[v] | (h->comp[v] << kCompShift));
    words = with_comp.data();
  }
  if (h->geo.brick) {
    DevTemp tmp(stream);
    if (tmp.alloc(h->nv * sizeof(uint16_t)) != hipSuccess)
      return fail(h, PSC_ENOMEM, "transient device buffer for the layout change failed");
    HIP_OK(h, hipMemcpyAsync(tmp.p, words, h->nv * sizeof(uint16_t), hipMemcpyHostToDevice,
                             stream));
    HIP_OK(h, launch_relayout(h->geo, h->nv, (const uint16_t *)tmp.p, L.occ, true, stream));
    HIP_OK(h, hipStreamSynchronize(stream));
  } else {
    HIP_OK(h, up(L.occ, words, h->nv * sizeof(uint16_t)));
  }

  // bins of the current event parity, by colour (counting sort)
  const int cur = (int)(h->event0 & 1);
  {
    std::vector<uint32_t> vox(walkers.size()), id(walkers.size());
    std::vector<uint16_t> spc(walkers.size());
    std::vector<int32_t> d3(disp ? 3 * walkers.size() : 0);
    uint64_t start[kMaxColours + 1] = {0};
    for (uint32_t c = 0; c < ncol; ++c) start[c + 1] = start[c] + bin_count[c];
    uint64_t fill[kMaxColours];
    for (uint32_t c = 0; c < ncol; ++c) fill[c] = start[c];
    for (uint64_t q : walkers) {
      const uint64_t at = fill[colour[q]]++;
      vox[at] = to_layout(h->geo, h->mvox[q]);
      id[at] = h->mid[q];
      spc[at] = words[h->mvox[q]];  // species and compartment
      if (disp) {
        d3[3 * at + 0] = h->mdx[q];
        d3[3 * at + 1] = h->mdy[q];
        d3[3 * at + 2] = h->mdz[q];
      }
    }
    uint32_t counts[kMaxColours] = {0};
    for (uint32_t c = 0; c < ncol; ++c) {
      if (bin_count[c] > cap) return fail(h, PSC_ECAPACITY, "more molecules than max_molecules");
      counts[c] = (uint32_t)bin_count[c];
      if (!bin_count[c]) continue;
      HIP_OK(h, up(L.bins[cur].vox + c * cap, vox.data() + start[c], bin_count[c] * 4));
      HIP_OK(h, up(L.bins[cur].id + c * cap, id.data() + start[c], bin_count[c] * 4));
      HIP_OK(h, up(L.bins[cur].sp + c * cap, spc.data() + start[c], bin_count[c] * 2));
      if (disp) {
        std::vector<int32_t> plane(bin_count[c]);
        for (int a = 0; a < 3; ++a) {
          for (uint64_t z = 0; z < bin_count[c]; ++z) plane[z] = d3[3 * (start[c] + z) + a];
          HIP_OK(h, up(L.bins[cur].disp + (a * ncol + c) * cap, plane.data(), bin_count[c] * 4));
        }
      }
    }
    HIP_OK(h, up(L.bins[cur].count, counts, sizeof counts));
    HIP_OK(h, hipMemset(L.bins[cur ^ 1].count, 0, kMaxColours * sizeof(uint32_t)));
  }
  HIP_OK(h, hipMemset(L.cand_count, 0, 2 * sizeof(uint32_t)));
  HIP_OK(h, hipMemset(L.flag_count, 0, 2 * sizeof(uint32_t)));
  HIP_OK(h, hipMemset(L.sdesc, 0, kMaxColours * sizeof(uint4)));  // empty until a first-order pass
  if (L.wb_count) HIP_OK(h, hipMemset(L.wb_count, 0, sizeof(uint32_t)));
  HIP_OK(h, hipMemset(L.birth_count, 0, sizeof(uint32_t)));
  HIP_OK(h, hipMemset(L.fire_count, 0, sizeof(uint32_t)));
  HIP_OK(h, hipMemset(L.recent, 0, kRecentN * sizeof(uint32_t)));
  h->recent_valid = false;   // counts of the state before this one do not apply
  h->recent_pending = false;
  HIP_OK(h, hipMemset(L.cnt, 0, kStatRep * kCntStride * sizeof(unsigned long long)));
  {
    // the initial counts in replica 0, the other replicas at zero
    std::vector<unsigned long long> counts(kStatRep * kSpStride, 0);
    for (uint64_t q = 0; q < nmol; ++q) counts[h->occ[h->mvox[q]]]++;
    HIP_OK(h, up(L.sp_count, counts.data(), counts.size() * sizeof(unsigned long long)));
  }
  HIP_OK(h, hipMemset(L.fired, 0, (uint64_t)kStatRep * L.fired_stride * sizeof(unsigned long long)));
  HIP_OK(h, hipMemset(L.error, 0, sizeof(uint32_t)));
  HIP_OK(h, hipMemset(L.end_done, 0, sizeof(uint32_t)));
  if (L.rank_hist) HIP_OK(h, hipMemset(L.rank_hist, 0, kRankBucketsMax * sizeof(uint32_t)));
  HIP_OK(h, hipMemset(L.nbr_cnt, 0, (1ull << L.nbr_bits) * sizeof(uint32_t)));
  HIP_OK(h, hipMemset(L.hot, 0, (1ull << L.hot_bits) / 4));
  HIP_OK(h, up(L.ev, &h->event0, sizeof(uint64_t)));
  HIP_OK(h, up(L.next_id, &h->next_id, sizeof(uint32_t)));

  // tape covering the events already done (a loaded state may start late)
  extend_tape(h, h->event0 + 1024);
  h->events_done = h->event0;
  HIP_OK(h, up(h->dL, &L, sizeof(LatDev)));
  psc_status st = sync_tape(h, stream);
  if (st) return st;

  // launch shape of the stage kernel from the molecules binned now (an
  // average colour bin holds 1/16 of them): a stage that cannot
  // fill the GPU with 4-item chunks (two workgroups per CU) takes one- or
  // two-item chunks to shorten its chain of dependent accesses.  Every chunk
  // gets a workgroup of its own, so that all of a stage's probes are in
  // flight at once (three waves per SIMD; a grid-striding second pass costs
  // about a sixth of the walk), with a quarter more workgroups than the
  // average bin needs: bins differ and grow, and a workgroup without a chunk
  // exits at once.
  h->walkers0 = walkers.size();
  if (!h->grid_set) {
    const uint64_t expect = std::max<uint64_t>(walkers.size() / ncol, 1);
    const uint64_t T = (uint64_t)stage_threads();
    if (!h->items_set) h->items = expect >= 512 * 4 * T ? 4 : (expect >= 512 * 2 * T ? 2 : 1);
    const uint64_t chunk = T * (uint64_t)h->items;
    h->grid = (int)std::min<uint64_t>(
        std::max<uint64_t>((5 * expect / 4 + chunk - 1) / chunk, 1), 65536);
  }
  HIP_OK(h, launch_scan(h->dL, std::min(h->grid * 4, 4096), stream));
  h->frozen = true;
  // the host copy of the walkers is no longer authoritative
  std::vector<uint16_t>().swap(h->occ);
  std::vector<uint8_t>().swap(h->comp);  // the device words hold it now
  std::vector<uint32_t>().swap(h->mid);
  std::vector<uint32_t>().swap(h->mvox);
  std::vector<int32_t>().swap(h->mdx);
  std::vector<int32_t>().swap(h->mdy);
  std::vector<int32_t>().swap(h->mdz);
  return PSC_OK;
}

uint64_t estimate_device_bytes(uint64_t voxels, uint64_t max_molecules, bool displacement,
                               uint32_t n_reactions, bool collision_births, uint32_t ncol) {
  auto r = [](uint64_t b) { return (std::max<uint64_t>(b, 16) + 255) & ~uint64_t(255); };
  const uint64_t cap = std::max<uint64_t>(max_molecules, 1);
  uint64_t t = r(voxels * 2);
  for (int b = 0; b < 2; ++b) {
    t += r(ncol * cap * 4) * 2 + r(ncol * cap * 2) + r(kMaxColours * 4);
    if (displacement) t += r(3 * ncol * cap * 4);
    t += r(cap * 4) * 2 + r(cap);
  }
  t += r(8) + 2 * r(cap * 4) + r(8) + r(256);
  const uint64_t bcap = std::min<uint64_t>(pow2_at_least(cap), 1ull << 27);
  t += r(bcap * 8) + r(bcap * 4) + r(bcap * 2) + r(4);
  if (collision_births) t += r(bcap * 4) + r(bcap * 8) + r(4);
  // the newborn ranking (first-order reactions with several products are
  // not known here: counted whenever the model has reactions)
  if (n_reactions) t += r(kRankBucketsMax * 4) + r((kRankBucketsMax + 1) * 4) + r(bcap * 8);
  uint32_t hb = 16;
  while (hb < 24 && (1ull << hb) < cap / 4) ++hb;
  t += r((1ull << hb) / 4) + r(4);
  uint32_t nb = 12;
  while (nb < 22 && (1ull << nb) < 8 * cap) ++nb;
  t += r((1ull << nb) * 4);
  t += r(cap * 4) * 3 + r(cap) * 2 + r(4);
  const uint64_t R = std::max<uint32_t>(n_reactions, 1);
  t += r(64) + r(64 * 64 * 2) + r(R * 4) + r(R) * 2 + r(R * 24) + r(128) + r(64);
  t += r(kStageTabWordsMax * 4);
  t += r(kStatRep * kSpStride * 8) + r(kStatRep * kCntStride * 8) +
       r((uint64_t)kStatRep * fired_stride((uint32_t)R) * 8);
  t += r(8) + r(64) + r(4) + r(4) + r(sizeof(LatDev));
  return t;
}

// out[a] = the sum over the kStatRep replicas of counter a (a < n), each
// replica `stride` words after the previous one
psc_status read_replicas(psc_lattice *h, const unsigned long long *dev, uint32_t n,
                         uint32_t stride, uint64_t *out) {
  std::vector<unsigned long long> all((uint64_t)kStatRep * stride);
  HIP_OK(h, hipMemcpy(all.data(), dev, all.size() * sizeof(unsigned long long),
                      hipMemcpyDeviceToHost));
  for (uint32_t a = 0; a < n; ++a) {
    uint64_t sum = 0;
    for (uint32_t r = 0; r < kStatRep; ++r) sum += all[(uint64_t)r * stride + a];
    out[a] = sum;
  }
  return PSC_OK;
}

// one event of the lattice (first-order pass in k_begin, the 16 stages, the
// event end) captured on a private stream; every launch reads the event's
// index and descriptors from the device, so one graph serves every event
psc_status ensure_lattice_graph(psc_lattice *h) {
  if (h->exec && h->graph_grid == h->grid && h->graph_items == h->items) return PSC_OK;
  if (h->exec) {
    HIP_OK(h, hipGraphExecDestroy(h->exec));
    h->exec = nullptr;
  }
  if (h->graph) {
    HIP_OK(h, hipGraphDestroy(h->graph));
    h->graph = nullptr;
  }
  if (!h->cap_stream) HIP_OK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  HIP_OK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  const hipError_t le = launch_event(h->dL, h->grid, h->items, h->L.bins[0].disp != nullptr,
                                     h->geo.fcc != 0, BeginShape{}, h->L.wb_count != nullptr,
                                     h->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(h->cap_stream, &g);
  if (le != hipSuccess || ce != hipSuccess)
    return fail(h, PSC_EDEVICE, "capturing the lattice's event failed: %s / %s",
                hipGetErrorString(le), hipGetErrorString(ce));
  h->graph = g;
  HIP_OK(h, hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0));
  h->graph_grid = h->grid;
  h->graph_items = h->items;
  return PSC_OK;
}

psc_status check_device_error(psc_lattice *h) {
  uint32_t e = 0;
  HIP_OK(h, hipMemcpy(&e, h->L.error, sizeof e, hipMemcpyDeviceToHost));
  if (!e) return PSC_OK;
  if (e & (kErrBinOverflow | kErrCandOverflow | kErrFlagOverflow | kErrBirthOverflow | kErrIds))
    return fail(h, PSC_EDEVICE, "device capacity exceeded (error bits 0x%x); state is invalid", e);
  return fail(h, PSC_EDEVICE, "device error bits 0x%x", e);
}

}  // namespace psc_detail

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

psc_status psc_create_lattice(const psc_lattice_desc *desc, psc_lattice **out) {
  if (!out) return PSC_EINVAL;
  *out = nullptr;
  if (!desc) {
    g_create_error = "desc is NULL";
    return PSC_EINVAL;
  }
  const uint32_t ni = desc->ni, nj = desc->nj, nk = desc->nk;
  if (ni < 4 || nj < 4 || nk < 4 || ni % 4 || nj % 4 || nk % 4) {
    g_create_error = "dimensions must be >= 4 and multiples of 4";
    return PSC_EINVAL;
  }
  const uint64_t nv = (uint64_t)ni * nj * nk;
  if (nv > (1ull << 32)) {
    g_create_error = "more than 2^32 voxels";
    return PSC_EINVAL;
  }
  if (!(desc->voxel_radius > 0.0) || !std::isfinite(desc->voxel_radius)) {
    g_create_error = "voxel_radius must be positive";
    return PSC_EINVAL;
  }
  if (desc->max_molecules == 0 || desc->max_molecules > nv || desc->max_molecules >= 0xFFFFFFFFull) {
    g_create_error = "max_molecules must be in [1, voxels]";
    return PSC_EINVAL;
  }
  if ((desc->alloc == nullptr) != (desc->free == nullptr)) {
    g_create_error = "alloc and free hooks come together";
    return PSC_EINVAL;
  }
  if (desc->flags &
      ~(PSC_TRACK_DISPLACEMENT | PSC_LAYOUT_LINEAR | PSC_BOUNDARY_WALLS | PSC_LATTICE_FCC)) {
    g_create_error = "unknown flags";
    return PSC_EINVAL;
  }
  if ((desc->flags & PSC_LATTICE_FCC) && (nk % 12 || ni % 8 || nj % 8)) {
    g_create_error = "an FCC lattice needs nk a multiple of 12 (stacking period 3, bricks of 4) "
                     "and ni, nj multiples of 8 (the stage colouring's period)";
    return PSC_EINVAL;
  }
  if (desc->device < 0) {
    g_create_error = "device ordinal must be >= 0";
    return PSC_EINVAL;
  }
  psc_lattice *h = new (std::nothrow) psc_lattice();
  if (!h) return PSC_ENOMEM;
  h->desc = *desc;
  h->nv = nv;
  h->geo.ni = ni;
  h->geo.nj = nj;
  h->geo.nk = nk;
  h->geo.dni = make_div(ni);
  h->geo.dnj = make_div(nj);
  h->geo.brick = (desc->flags & PSC_LAYOUT_LINEAR) ? 0u : 1u;
  h->geo.walls = (desc->flags & PSC_BOUNDARY_WALLS) ? 1u : 0u;
  h->geo.fcc = (desc->flags & PSC_LATTICE_FCC) ? 1u : 0u;
  h->geo.nbi = ni / 4;
  h->geo.nbj = nj / 4;
  h->geo.dnbi = make_div(ni / 4);
  h->geo.dnbj = make_div(nj / 4);
  try {
    h->occ.assign(nv, 0);
  } catch (...) {
    delete h;
    g_create_error = "host allocation of the lattice failed";
    return PSC_ENOMEM;
  }
  *out = h;
  return PSC_OK;
}

void psc_destroy(psc_lattice *h) {
  if (!h) return;
  if (h->frozen && !h->poisoned) {
    (void)hipSetDevice(h->desc.device);
    (void)hipDeviceSynchronize();
  }
  for (auto &t : h->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto &e : h->event_pool) (void)hipEventDestroy(e);
  if (h->recent_ev) (void)hipEventDestroy(h->recent_ev);
  if (h->h_recent) (void)hipHostFree(h->h_recent);
  if (h->exec) (void)hipGraphExecDestroy(h->exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  dev_free_all(h);
  delete h;
}

const char *psc_last_error(const psc_lattice *h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

psc_status psc_add_species(psc_lattice *h, const char *name, double D, uint16_t *out_id) {
  if (!h) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  if (h->frozen) return fail(h, PSC_ESTATE, "model is frozen after the first step");
  if (!(D >= 0.0) || !std::isfinite(D)) return fail(h, PSC_EINVAL, "D must be finite and >= 0");
  if (h->species.size() > (size_t)PSC_MAX_SPECIES)
    return fail(h, PSC_EINVAL, "at most %d species", PSC_MAX_SPECIES);
  SpeciesDef s;
  s.name = name ? name : "";
  s.D = D;
  s.tau = D > 0.0 ? diffusion_interval(h->desc.voxel_radius, D) : 0.0;
  h->species.push_back(s);
  if (out_id) *out_id = (uint16_t)(h->species.size() - 1);
  return PSC_OK;
}

psc_status psc_add_reaction(psc_lattice *h, const uint16_t *reactants, uint32_t n_r,
                            const uint16_t *products, uint32_t n_p, double k, uint32_t *out_id) {
  if (!h) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  if (h->frozen) return fail(h, PSC_ESTATE, "model is frozen after the first step");
  if (h->rx.size() >= (size_t)PSC_MAX_REACTIONS)
    return fail(h, PSC_EINVAL, "at most %d reactions", PSC_MAX_REACTIONS);
  if (!reactants || n_r < 1 || n_r > 2) return fail(h, PSC_EINVAL, "1 or 2 reactants");
  if (n_p && !products) return fail(h, PSC_EINVAL, "products is NULL");
  if (!(k >= 0.0) || !std::isfinite(k)) return fail(h, PSC_EINVAL, "k must be finite and >= 0");
  const uint16_t S = (uint16_t)(h->species.size() - 1);
  for (uint32_t a = 0; a < n_r; ++a)
    if (reactants[a] < 1 || reactants[a] > S) return fail(h, PSC_EINVAL, "unknown reactant");
  for (uint32_t a = 0; a < n_p; ++a)
    if (products[a] < 1 || products[a] > S) return fail(h, PSC_EINVAL, "unknown product");
  if (n_r == 1 && n_p > (uint32_t)PSC_MAX_PRODUCTS)
    return fail(h, PSC_EINVAL, "first-order reactions take 0..%d products", PSC_MAX_PRODUCTS);
  if (n_r == 2) {
    if (n_p < 1 || n_p > (uint32_t)PSC_MAX_PRODUCTS)
      return fail(h, PSC_EINVAL, "second-order reactions take 1..%d products", PSC_MAX_PRODUCTS);
    const uint16_t A = reactants[0], B = reactants[1];
    if (!(h->species[A].D + h->species[B].D > 0.0))
      return fail(h, PSC_EINVAL, "two immobile reactants never collide");
    for (auto &r : h->rx)
      if (r.nr == 2 && ((r.r[0] == A && r.r[1] == B) || (r.r[0] == B && r.r[1] == A)))
        return fail(h, PSC_EINVAL, "reactant pair already has a reaction");
  }
  ReactionDef d;
  d.nr = n_r;
  d.np = n_p;
  for (uint32_t a = 0; a < n_r; ++a) d.r[a] = reactants[a];
  for (uint32_t a = 0; a < n_p; ++a) d.p[a] = products[a];
  d.k = k;
  h->rx.push_back(d);
  if (out_id) *out_id = (uint32_t)(h->rx.size() - 1);
  return PSC_OK;
}

psc_status psc_get_reaction_info(const psc_lattice *h, uint32_t reaction_id,
                                 psc_reaction_info *out) {
  if (!h || !out || reaction_id >= h->rx.size()) return PSC_EINVAL;
  const ReactionDef &d = h->rx[reaction_id];
  *out = psc_reaction_info{};
  out->order = d.nr;
  if (d.nr == 1) {
    out->p = d.k;
    return PSC_OK;
  }
  double den = 6.0 * std::sqrt(2.0);
  den = den * (h->species[d.r[0]].D + h->species[d.r[1]].D);
  den = den * h->desc.voxel_radius;
  out->p = d.k / den;
  uint32_t thr = 0;
  uint8_t always = 0;
  second_order_threshold(d.k, h->species[d.r[0]].D, h->species[d.r[1]].D,
                         h->desc.voxel_radius, &thr, &always);
  out->clamped = out->p > 1.0 ? 1u : 0u;
  out->threshold = always ? (1ull << 32) : (uint64_t)thr;
  return PSC_OK;
}

psc_status psc_place_uniform(psc_lattice *h, uint16_t species, uint64_t count) {
  if (!h) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  if (h->frozen) return fail(h, PSC_ESTATE, "placement only before the first step");
  if (species < 1 || species >= h->species.size()) return fail(h, PSC_EINVAL, "unknown species");
  const uint64_t have = h->mid.size();
  if (count > h->nv - have) return fail(h, PSC_ECAPACITY, "too few vacant voxels");
  if (have + count > h->desc.max_molecules)
    return fail(h, PSC_ECAPACITY, "placement exceeds max_molecules");
  if ((uint64_t)h->next_id + count >= 0xFFFFFFFFull) return fail(h, PSC_ECAPACITY, "ids exhausted");
  const uint32_t call = (uint32_t)h->place_calls;
  const uint32_t k0 = (uint32_t)h->desc.seed, k1 = (uint32_t)(h->desc.seed >> 32);
  uint64_t attempt = 0;
  const bool disp = (h->desc.flags & PSC_TRACK_DISPLACEMENT) != 0;
  (void)disp;
  for (uint64_t q = 0; q < count; ++q) {
    for (;;) {
      const U4 r = philox(call, (uint32_t)attempt, kPhasePlace, 0, k0, k1);
      ++attempt;
      const uint32_t v = (uint32_t)(((uint64_t)r.x * h->nv) >> 32);
      if (h->occ[v] == 0) {
        h->occ[v] = species;
        h->mid.push_back(h->next_id++);
        h->mvox.push_back(v);
        h->mdx.push_back(0);
        h->mdy.push_back(0);
        h->mdz.push_back(0);
        break;
      }
    }
  }
  h->place_calls++;
  return PSC_OK;
}

psc_status psc_set_compartments(psc_lattice *h, const uint8_t *comp) {
  if (!h) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  if (h->frozen) return fail(h, PSC_ESTATE, "compartments only before the first step");
  if (!comp) return fail(h, PSC_EINVAL, "comp is NULL");
  try {
    h->comp.assign(comp, comp + h->nv);
  } catch (...) {
    return fail(h, PSC_ENOMEM, "host allocation of the compartment map failed");
  }
  return PSC_OK;
}

psc_status psc_place_uniform_in(psc_lattice *h, uint16_t species, uint64_t count,
                                uint32_t compartment) {
  if (!h) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  if (h->frozen) return fail(h, PSC_ESTATE, "placement only before the first step");
  if (species < 1 || species >= h->species.size()) return fail(h, PSC_EINVAL, "unknown species");
  if (compartment >= (uint32_t)kMaxCompartments)
    return fail(h, PSC_EINVAL, "compartments are 0..%d", kMaxCompartments - 1);
  auto comp_of = [&](uint64_t v) -> uint32_t { return h->comp.empty() ? 0u : h->comp[v]; };
  uint64_t vacant = 0;
  for (uint64_t v = 0; v < h->nv; ++v) vacant += h->occ[v] == 0 && comp_of(v) == compartment;
  if (count > vacant) return fail(h, PSC_ECAPACITY, "too few vacant voxels in compartment %u",
                                  compartment);
  if (h->mid.size() + count > h->desc.max_molecules)
    return fail(h, PSC_ECAPACITY, "placement exceeds max_molecules");
  if ((uint64_t)h->next_id + count >= 0xFFFFFFFFull) return fail(h, PSC_ECAPACITY, "ids exhausted");
  const uint32_t call = (uint32_t)h->place_calls;
  const uint32_t k0 = (uint32_t)h->desc.seed, k1 = (uint32_t)(h->desc.seed >> 32);
  uint64_t attempt = 0;
  for (uint64_t q = 0; q < count; ++q) {
    for (;;) {
      const U4 r = philox(call, (uint32_t)attempt, kPhasePlace, 0, k0, k1);
      ++attempt;
      const uint32_t v = (uint32_t)(((uint64_t)r.x * h->nv) >> 32);
      if (h->occ[v] == 0 && comp_of(v) == compartment) {
        h->occ[v] = species;
        h->mid.push_back(h->next_id++);
        h->mvox.push_back(v);
        h->mdx.push_back(0);
        h->mdy.push_back(0);
        h->mdz.push_back(0);
        break;
      }
    }
  }
  h->place_calls++;
  return PSC_OK;
}

psc_status psc_load_state(psc_lattice *h, const psc_state_view *st) {
  if (!h || !st) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  if (h->frozen) return fail(h, PSC_ESTATE, "load_state only before the first step");
  if (!st->occupancy || (st->n_molecules && (!st->id || !st->voxel)))
    return fail(h, PSC_EINVAL, "occupancy, id and voxel arrays are required");
  if (st->n_molecules > h->desc.max_molecules)
    return fail(h, PSC_ECAPACITY, "state exceeds max_molecules");
  const uint16_t S = (uint16_t)(h->species.size() - 1);
  uint64_t occupied = 0;
  for (uint64_t v = 0; v < h->nv; ++v) {
    if (st->occupancy[v] > S) return fail(h, PSC_EINVAL, "occupancy holds an unknown species");
    occupied += st->occupancy[v] != 0;
  }
  if (occupied != st->n_molecules)
    return fail(h, PSC_EINVAL, "occupied voxels (%llu) != molecules (%llu)",
                (unsigned long long)occupied, (unsigned long long)st->n_molecules);
  std::vector<uint8_t> seen(h->nv, 0);
  for (uint64_t q = 0; q < st->n_molecules; ++q) {
    if (q && st->id[q] <= st->id[q - 1]) return fail(h, PSC_EINVAL, "ids must ascend");
    if (st->id[q] >= st->next_id || st->next_id == 0xFFFFFFFFu)
      return fail(h, PSC_EINVAL, "id >= next_id");
    if (st->voxel[q] >= h->nv || st->occupancy[st->voxel[q]] == 0)
      return fail(h, PSC_EINVAL, "molecule on an empty voxel");
    if (st->species && st->species[q] != st->occupancy[st->voxel[q]])
      return fail(h, PSC_EINVAL, "species disagrees with occupancy");
    if (seen[st->voxel[q]]++) return fail(h, PSC_EINVAL, "two molecules on one voxel");
  }
  h->occ.assign(st->occupancy, st->occupancy + h->nv);
  h->mid.assign(st->id, st->id + st->n_molecules);
  h->mvox.assign(st->voxel, st->voxel + st->n_molecules);
  const uint64_t n = st->n_molecules;
  h->mdx.assign(n, 0);
  h->mdy.assign(n, 0);
  h->mdz.assign(n, 0);
  if (st->dx) h->mdx.assign(st->dx, st->dx + n);
  if (st->dy) h->mdy.assign(st->dy, st->dy + n);
  if (st->dz) h->mdz.assign(st->dz, st->dz + n);
  h->next_id = st->next_id;
  h->event0 = st->event;
  return PSC_OK;
}

psc_status psc_step(psc_lattice *h, uint64_t n_events, void *stream_) {
  if (!h) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  if (h->in_ensemble && n_events)
    return fail(h, PSC_ESTATE, "the lattice is stepped by its ensemble");
  hipStream_t stream = (hipStream_t)stream_;
  if (!h->frozen) {
    // the device is first touched here: creation, the model and the initial
    // state are host-only
    int ndev = 0;
    const hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || h->desc.device >= ndev)
      return fail(h, PSC_EINVAL, "no HIP device %d (%d devices, %s)", h->desc.device, ndev,
                  hipGetErrorString(e));
  }
  HIP_OK(h, hipSetDevice(h->desc.device));
  if (!h->frozen) {
    psc_status st = freeze(h, stream);
    if (st) return st;
  }
  if (n_events == 0) return PSC_OK;
  const uint64_t end = h->events_done + n_events;
  if (end >= 0xFFFFFFFFull) return fail(h, PSC_EINVAL, "event index exceeds 2^32");
  if (end > h->tape_end) {
    extend_tape(h, std::max(end, h->tape_end * 2));
    psc_status st = sync_tape(h, stream);
    if (st) return st;
  }
  // The device's counts of the last event before the previous step ended,
  // if their copy is done (no wait): launches sized for the expectations
  // below are dropped when recent events did not need them.  Only the speed
  // depends on it: a short path handles any count, more slowly.
  if (h->recent_pending && hipEventQuery(h->recent_ev) == hipSuccess) {
    for (int k = 0; k < kRecentN; ++k) h->recent[k] = h->h_recent[k];
    h->recent_valid = true;
    h->recent_pending = false;
  }
  // First-order decisions run inside k_begin (one workgroup) unless an event
  // expects many candidates (the event's largest threshold times the
  // walkers): then a launch of their own spreads them over workgroups.
  auto decide_grid = [&](uint64_t e) -> int {
    if (!h->n_fo) return 0;
    const double expect = (double)h->tape_cmax[e] * (1.0 / 4294967296.0) * (double)h->walkers0;
    if (expect < 4096.0) return 0;
    return (int)std::min(std::ceil(expect / 512.0), 1024.0);
  };
  // Newborns of the first-order pass are ranked by k_begin alone up to the
  // LDS limit (2048); an event whose bound on them (its expected candidates
  // times the most extra products of a firing) reaches twice that gets the
  // grid-wide ranking, a thread per bounded newborn.  Events under the bound
  // that exceed the limit fall back to k_begin's slower sort.
  auto births_grid = [&](uint64_t e) -> int {
    if (!h->fo_extra_max) return 0;
    // the last event's newborns fit k_begin's ranking with room to spare
    if (h->recent_valid && h->recent[kRecentFoBirths] <= 1024) return 0;
    const double expect = (double)h->tape_cmax[e] * (1.0 / 4294967296.0) *
                          (double)h->walkers0 * (double)h->fo_extra_max;
    if (expect < 4096.0) return 0;
    return (int)std::min(std::ceil(expect / 256.0), 2048.0);
  };
  // An event whose decisions get a launch of their own may fire more
  // first-order reactions than k_begin has threads (the candidates bound the
  // firings; only the device knows how many fire): it gets one application
  // launch per stage, a workgroup per kFoTile expected candidates, which
  // find the list empty when k_begin applied it itself.
  auto apply_grid = [&](uint64_t e) -> int {
    if (!h->n_fo) return 0;
    // the last event's firings took half of k_begin's threads or fewer
    if (h->recent_valid && h->recent[kRecentFire] <= 512) return 0;
    const double expect = (double)h->tape_cmax[e] * (1.0 / 4294967296.0) * (double)h->walkers0;
    if (expect < 4096.0) return 0;
    return (int)std::min(std::max(std::ceil(expect / kFoTile), 1.0), 1024.0);
  };
  auto shape = [&](uint64_t e) {
    BeginShape b;
    b.decide = decide_grid(e);
    b.births = births_grid(e);
    b.apply = apply_grid(e);
    return b;
  };
  const uint64_t e0 = h->events_done;
  const bool disp = h->L.bins[0].disp != nullptr, births = h->L.wb_count != nullptr;
  // collision newborns beyond the event end's own ranking get the grid-wide
  // numbering unless the last event's fitted with room to spare
  const bool births_defer = !(h->recent_valid && h->recent[kRecentColBirths] <= 1024);
  // the tape words the walk of event e reads (as the device reads them)
  auto due_of = [&](uint64_t e) -> uint64_t { return h->tape_due[e]; };
  auto cmax_after = [&](uint64_t e) -> uint32_t {
    return (h->L.n_fo && e + 1 < h->L.tape_horizon) ? h->tape_cmax[e + 1] : 0u;
  };
  if (!h->timing && h->use_graph) {
    psc_status st = ensure_lattice_graph(h);
    if (st) return st;
    for (uint64_t e = 0; e < n_events; ++e) {
      const BeginShape b = shape(e0 + e);
      if (b.decide || b.births || b.apply)
        HIP_OK(h, launch_event(h->dL, h->grid, h->items, disp, h->geo.fcc != 0, b, births,
                               stream));
      else HIP_OK(h, hipGraphLaunch(h->exec, stream));
    }
  } else if (!h->timing) {
    // An event's end is left to the next event's opening (one kernel for
    // both) when neither needs launches of its own: no collision newborns to
    // number, and a next opening that k_begin does alone.  One workgroup
    // then sweeps the end's lists of reacted partners, each entry a scattered
    // read and write of the lattice, so only while the last event's list was
    // short, or of moderate length on a lattice small enough (2^27 voxels,
    // 256 MB of words) that those accesses stay in the caches.  On the 2^32
    // MAPK lattice (~8,000 partners per event) the end is faster over many
    // workgroups; on a crowded 256^3 lattice (up to 11,000) the single
    // launch wins.  The last event of the call always ends in its own launch.
    auto plain = [](const BeginShape &b) { return b.decide == 0 && b.births == 0 && b.apply == 0; };
    const uint32_t partners = h->recent[kRecentFlags];
    const bool fuse = h->recent_valid && (partners <= 1024 ||
                                          (h->nv <= (1ull << 27) && partners <= 16384));
    bool open_with_end = false;
    BeginShape b = shape(e0);
    for (uint64_t e = 0; e < n_events; ++e) {
      const BeginShape next = e + 1 < n_events ? shape(e0 + e + 1) : BeginShape{};
      const bool leave_end = fuse && !births && e + 1 < n_events && plain(next);
      HIP_OK(h, launch_event_direct(h->dL, h->L, e0 + e, due_of(e0 + e), cmax_after(e0 + e),
                                    h->grid, h->items, disp, h->geo.fcc != 0, b, births,
                                    births_defer, stream, open_with_end, !leave_end));
      open_with_end = leave_end;
      b = next;
    }
  } else {
    auto ev = [&](hipEvent_t *out) -> hipError_t {
      if (!h->event_pool.empty()) {
        *out = h->event_pool.back();
        h->event_pool.pop_back();
        return hipSuccess;
      }
      return hipEventCreate(out);
    };
    for (uint64_t e = 0; e < n_events; ++e) {
      const int stages = (int)n_colours(h->geo);
      uint32_t perm[kMaxColours];
      stage_order_of(h->L.key0, h->L.key1, e0 + e, (uint32_t)stages, perm);
      for (int g = -1; g <= stages; ++g) {
        psc_lattice::Timed t;
        t.kind = g < 0 ? 0 : (g < stages ? 1 : 2);
        HIP_OK(h, ev(&t.a));
        HIP_OK(h, ev(&t.b));
        HIP_OK(h, hipEventRecord(t.a, stream));
        if (g < 0)
          HIP_OK(h, launch_begin(h->dL, shape(e0 + e), (uint32_t)stages, stream, h->items > 4,
                                 &h->L, perm, e0 + e));
        else if (g < stages && h->items <= 4)
          HIP_OK(h, launch_stage_direct(h->L, perm[g], e0 + e, due_of(e0 + e),
                                        cmax_after(e0 + e), h->grid, h->items,
                                        h->L.bins[0].disp != nullptr, h->geo.fcc != 0, stream));
        else if (g < stages)
          HIP_OK(h, launch_stage(h->dL, (uint32_t)g, h->grid, h->items,
                                 h->L.bins[0].disp != nullptr, h->geo.fcc != 0, stream));
        else HIP_OK(h, launch_end(h->dL, births, stream, births_defer));
        HIP_OK(h, hipEventRecord(t.b, stream));
        h->timed.push_back(t);
      }
    }
  }
  h->events_done = end;
  h->last_stream = stream;
  // copy the last event's counts back for the next step (no wait)
  if (!h->recent_pending) {
    if (!h->h_recent) {
      HIP_OK(h, hipHostMalloc((void **)&h->h_recent, kRecentN * sizeof(uint32_t),
                              hipHostMallocDefault));
      HIP_OK(h, hipEventCreateWithFlags(&h->recent_ev, hipEventDisableTiming));
    }
    HIP_OK(h, hipMemcpyAsync(h->h_recent, h->L.recent, kRecentN * sizeof(uint32_t),
                             hipMemcpyDeviceToHost, stream));
    HIP_OK(h, hipEventRecord(h->recent_ev, stream));
    h->recent_pending = true;
  }
  return PSC_OK;
}

psc_status psc_sync(psc_lattice *h) {
  if (!h) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  if (!h->frozen) return PSC_OK;
  HIP_OK(h, hipSetDevice(h->desc.device));
  HIP_OK(h, hipDeviceSynchronize());
  return check_device_error(h);
}

psc_status psc_query_sizes(const psc_lattice *hc, uint64_t *n_voxels, uint64_t *n_molecules,
                           uint32_t *n_species, uint32_t *n_reactions) {
  psc_lattice *h = const_cast<psc_lattice *>(hc);
  if (!h) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  if (n_voxels) *n_voxels = h->nv;
  if (n_species) *n_species = (uint32_t)(h->species.size() - 1);
  if (n_reactions) *n_reactions = (uint32_t)h->rx.size();
  if (n_molecules) {
    if (!h->frozen) {
      *n_molecules = h->mid.size();
    } else {
      HIP_OK(h, hipSetDevice(h->desc.device));
      HIP_OK(h, hipDeviceSynchronize());
      uint32_t counts[kMaxColours];
      HIP_OK(h, hipMemcpy(counts, h->L.bins[h->events_done & 1].count, sizeof counts,
                          hipMemcpyDeviceToHost));
      uint64_t n = h->st_id.size();
      for (uint32_t c = 0; c < h->L.ncol; ++c) n += counts[c];
      *n_molecules = n;  // upper bound: dead entries are dropped by the walk
    }
  }
  return PSC_OK;
}

psc_status psc_required_sizes(const psc_lattice *h, uint64_t *n_voxels, uint64_t *n_molecules,
                              uint32_t *n_species, uint32_t *n_reactions) {
  return psc_query_sizes(h, n_voxels, n_molecules, n_species, n_reactions);
}

psc_status psc_read_counters(psc_lattice *h, psc_counters *out, uint64_t *event) {
  if (!h || !out) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  if (event) *event = h->frozen ? h->events_done : h->event0;
  if (!h->frozen) {
    *out = psc_counters{0, 0, 0, 0};
    return PSC_OK;
  }
  HIP_OK(h, hipSetDevice(h->desc.device));
  HIP_OK(h, hipDeviceSynchronize());
  psc_status st = check_device_error(h);
  if (st) return st;
  uint64_t cnt[4];
  psc_status rs = read_replicas(h, h->L.cnt, 4, kCntStride, cnt);
  if (rs) return rs;
  *out = psc_counters{cnt[0], cnt[1], cnt[2], cnt[3]};
  return PSC_OK;
}

psc_status psc_read_stats(psc_lattice *h, uint64_t *species_count, uint64_t *disp_sum,
                          uint64_t *n_walkers) {
  if (!h) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  if (!h->frozen) {
    if (species_count) {
      for (size_t s = 0; s < h->species.size(); ++s) species_count[s] = 0;
      for (uint64_t q = 0; q < h->mid.size(); ++q) species_count[h->occ[h->mvox[q]]]++;
    }
    uint64_t acc = 0;
    for (uint64_t q = 0; q < h->mid.size(); ++q) {
      const int64_t X = h->mdx[q], Y = h->mdy[q], Z = h->mdz[q];
      acc += (uint64_t)(3 * X * X + Y * Y + 8 * Z * Z);
    }
    if (disp_sum) *disp_sum = acc;
    if (n_walkers) *n_walkers = h->mid.size();
    return PSC_OK;
  }
  HIP_OK(h, hipSetDevice(h->desc.device));
  HIP_OK(h, hipDeviceSynchronize());
  psc_status st = check_device_error(h);
  if (st) return st;
  if (species_count) {
    uint64_t c[64];
    psc_status rs = read_replicas(h, h->L.sp_count, 64, kSpStride, c);
    if (rs) return rs;
    for (size_t s = 0; s < h->species.size(); ++s) species_count[s] = c[s];
  }
  if (disp_sum || n_walkers) {
    unsigned long long out[2] = {0, 0};
    DevTemp d;
    HIP_OK(h, d.alloc(sizeof out));
    HIP_OK(h, hipMemset(d.p, 0, sizeof out));
    HIP_OK(h, launch_msd(h->dL, (unsigned long long *)d.p, nullptr));
    HIP_OK(h, hipMemcpy(out, d.p, sizeof out, hipMemcpyDeviceToHost));
    // static molecules never move, but a loaded state may give them a
    // displacement
    for (size_t q = 0; q < h->st_id.size(); ++q) {
      const int64_t X = h->st_d[0][q], Y = h->st_d[1][q], Z = h->st_d[2][q];
      out[0] += (uint64_t)(3 * X * X + Y * Y + 8 * Z * Z);
    }
    if (disp_sum) *disp_sum = out[0];
    if (n_walkers) *n_walkers = out[1];
  }
  return PSC_OK;
}

psc_status psc_set_launch(psc_lattice *h, const psc_launch *l) {
  if (!h || !l) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  const int it = (int)l->items_per_thread;
  if (it != 0 && it != 1 && it != 2 && it != 4 && it != 8 && it != 16)
    return fail(h, PSC_EINVAL, "items_per_thread must be 1, 2, 4, 8 or 16");
  if (l->stage_blocks > 65536) return fail(h, PSC_EINVAL, "stage_blocks must be <= 65536");
  if (it) {
    h->items = it;
    h->items_set = true;
  }
  if (l->stage_blocks) {
    h->grid = (int)l->stage_blocks;
    h->grid_set = true;
  }
  return PSC_OK;
}

psc_status psc_get_launch(const psc_lattice *h, psc_launch *out) {
  if (!h || !out) return PSC_EINVAL;
  out->items_per_thread = (uint32_t)h->items;
  out->stage_blocks = (uint32_t)h->grid;
  return PSC_OK;
}

psc_status psc_set_graph_replay(psc_lattice *h, int enable) {
  if (!h) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  if (enable != 0 && enable != 1) return fail(h, PSC_EINVAL, "graph replay must be 0 or 1");
  h->use_graph = enable != 0;
  return PSC_OK;
}

psc_status psc_set_kernel_timing(psc_lattice *h, int enable) {
  if (!h) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  if (enable < 0 || enable > 2) return fail(h, PSC_EINVAL, "timing mode must be 0, 1 or 2");
  // 0 and 2 only switch recording (no synchronisation): a caller may time a
  // sample of the events of a run without stalling it
  if (enable == 1 && !h->timed.empty()) {
    HIP_OK(h, hipSetDevice(h->desc.device));
    HIP_OK(h, hipDeviceSynchronize());
    for (auto &t : h->timed) {
      h->event_pool.push_back(t.a);
      h->event_pool.push_back(t.b);
    }
    h->timed.clear();
  }
  h->timing = enable != 0;
  return PSC_OK;
}

psc_status psc_get_kernel_times(psc_lattice *h, psc_kernel_times *out) {
  if (!h || !out) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  *out = psc_kernel_times{0, 0, 0, 0, 0, 0};
  if (h->timed.empty()) return PSC_OK;
  HIP_OK(h, hipSetDevice(h->desc.device));
  HIP_OK(h, hipEventSynchronize(h->timed.back().b));
  for (auto &t : h->timed) {
    float ms = 0.f;
    HIP_OK(h, hipEventElapsedTime(&ms, t.a, t.b));
    if (t.kind == 0) {
      out->begin_ms += ms;
      out->begin_launches++;
    } else if (t.kind == 1) {
      out->stage_ms += ms;
      out->stage_launches++;
    } else {
      out->end_ms += ms;
      out->end_launches++;
    }
  }
  return PSC_OK;
}

psc_status psc_device_bytes(const psc_lattice *h, uint64_t *bytes) {
  if (!h || !bytes) return PSC_EINVAL;
  *bytes = h->device_bytes;
  return PSC_OK;
}

psc_status psc_read_state(psc_lattice *h, psc_state_view *out, void *stream_) {
  (void)stream_;
  return read_state_with(h, out, read_occupancy_transient, nullptr);
}

}  // extern "C"

namespace psc_detail {

// Occupancy in the ABI's linear order, species only, through a transient
// device buffer of the lattice's size when the device layout is bricked.
psc_status read_occupancy_transient(psc_lattice *h, uint16_t *occp, void *) {
  const LatDev &L = h->L;
  if (h->geo.brick) {
    DevTemp tmp;
    if (tmp.alloc(h->nv * sizeof(uint16_t)) != hipSuccess)
      return fail(h, PSC_ENOMEM, "transient device buffer for the layout change failed");
    HIP_OK(h, launch_relayout(h->geo, h->nv, L.occ, (uint16_t *)tmp.p, false, nullptr));
    HIP_OK(h, hipMemcpy(occp, tmp.p, h->nv * sizeof(uint16_t), hipMemcpyDeviceToHost));
  } else {
    HIP_OK(h, hipMemcpy(occp, L.occ, h->nv * sizeof(uint16_t), hipMemcpyDeviceToHost));
  }
  for (uint64_t v = 0; v < h->nv; ++v) occp[v] &= kSpeciesBits;
  return PSC_OK;
}

psc_status read_state_with(psc_lattice *h, psc_state_view *out, OccupancyReader read_occ,
                           void *ctx) {
  if (!h || !out) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  const bool want_mol = out->id || out->voxel || out->species || out->dx || out->dy || out->dz;
  if (!h->frozen) {
    const uint64_t n = h->mid.size();
    std::vector<uint64_t> order(n);
    for (uint64_t q = 0; q < n; ++q) order[q] = q;
    std::sort(order.begin(), order.end(),
              [&](uint64_t a, uint64_t b) { return h->mid[a] < h->mid[b]; });
    if (want_mol && out->n_molecules < n) {
      out->n_molecules = n;
      return fail(h, PSC_ECAPACITY, "output arrays too small");
    }
    if (out->occupancy) std::memcpy(out->occupancy, h->occ.data(), h->nv * sizeof(uint16_t));
    for (uint64_t z = 0; z < n; ++z) {
      const uint64_t q = order[z];
      if (out->id) out->id[z] = h->mid[q];
      if (out->voxel) out->voxel[z] = h->mvox[q];
      if (out->species) out->species[z] = h->occ[h->mvox[q]];
      if (out->dx) out->dx[z] = h->mdx[q];
      if (out->dy) out->dy[z] = h->mdy[q];
      if (out->dz) out->dz[z] = h->mdz[q];
    }
    out->n_molecules = n;
    out->event = h->event0;
    out->next_id = h->next_id;
    out->time = clock_time(h, h->event0);
    out->counters = psc_counters{0, 0, 0, 0};
    if (out->reactions_fired)
      for (size_t r = 0; r < h->rx.size(); ++r) out->reactions_fired[r] = 0;
    return PSC_OK;
  }
  HIP_OK(h, hipSetDevice(h->desc.device));
  HIP_OK(h, hipDeviceSynchronize());
  psc_status st = check_device_error(h);
  if (st) return st;
  const LatDev &L = h->L;
  const int cur = (int)(h->events_done & 1);
  uint32_t counts[kMaxColours];
  HIP_OK(h, hipMemcpy(counts, L.bins[cur].count, sizeof counts, hipMemcpyDeviceToHost));
  const bool disp = L.bins[cur].disp != nullptr;
  std::vector<uint32_t> vox, id;
  std::vector<int32_t> d3[3];
  for (uint32_t c = 0; c < L.ncol; ++c) {
    const uint32_t n = counts[c];
    if (!n) continue;
    const size_t at = vox.size();
    vox.resize(at + n);
    id.resize(at + n);
    HIP_OK(h, hipMemcpy(vox.data() + at, L.bins[cur].vox + c * L.cap, n * 4, hipMemcpyDeviceToHost));
    HIP_OK(h, hipMemcpy(id.data() + at, L.bins[cur].id + c * L.cap, n * 4, hipMemcpyDeviceToHost));
    if (disp)
      for (int a = 0; a < 3; ++a) {
        d3[a].resize(at + n);
        HIP_OK(h, hipMemcpy(d3[a].data() + at, L.bins[cur].disp + (a * L.ncol + c) * L.cap, n * 4,
                            hipMemcpyDeviceToHost));
      }
  }
  // gather live walkers and static molecules, ascending id
  std::vector<uint64_t> order;
  order.reserve(vox.size() + h->st_id.size());
  for (uint64_t q = 0; q < vox.size(); ++q)
    if (id[q] != kDeadId) order.push_back(q);
  const uint64_t nwalk = vox.size();
  for (uint64_t q = 0; q < h->st_id.size(); ++q) order.push_back(nwalk + q);
  auto id_of = [&](uint64_t q) { return q < nwalk ? id[q] : h->st_id[q - nwalk]; };
  for (uint64_t q = 0; q < nwalk; ++q) vox[q] = to_linear(h->geo, vox[q]);
  auto vox_of = [&](uint64_t q) { return q < nwalk ? vox[q] : h->st_vox[q - nwalk]; };
  std::sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) { return id_of(a) < id_of(b); });
  const uint64_t n = order.size();
  if (want_mol && out->n_molecules < n) {
    out->n_molecules = n;
    return fail(h, PSC_ECAPACITY, "output arrays too small");
  }
  std::vector<uint16_t> occ;
  uint16_t *occp = out->occupancy;
  if (!occp && out->species) {
    occ.resize(h->nv);
    occp = occ.data();
  }
  if (occp) {
    st = read_occ(h, occp, ctx);
    if (st) return st;
  }
  for (uint64_t z = 0; z < n; ++z) {
    const uint64_t q = order[z];
    const uint32_t v = vox_of(q);
    if (out->id) out->id[z] = id_of(q);
    if (out->voxel) out->voxel[z] = v;
    if (out->species) out->species[z] = occp[v];
    for (int a = 0; a < 3; ++a) {
      int32_t *dst = a == 0 ? out->dx : (a == 1 ? out->dy : out->dz);
      if (!dst) continue;
      if (q >= nwalk) dst[z] = h->st_d[a][q - nwalk];  // static molecules never move
      else dst[z] = disp ? d3[a][q] : 0;
    }
  }
  out->n_molecules = n;
  out->event = h->events_done;
  HIP_OK(h, hipMemcpy(&out->next_id, L.next_id, sizeof(uint32_t), hipMemcpyDeviceToHost));
  out->time = h->events_done ? h->tape_time[h->events_done - 1] : 0.0;
  uint64_t cnt[4];
  st = read_replicas(h, L.cnt, 4, kCntStride, cnt);
  if (st) return st;
  out->counters = psc_counters{cnt[0], cnt[1], cnt[2], cnt[3]};
  if (out->reactions_fired && !h->rx.empty()) {
    st = read_replicas(h, L.fired, (uint32_t)h->rx.size(), L.fired_stride,
                       out->reactions_fired);
    if (st) return st;
  }
  return PSC_OK;
}

}  // namespace psc_detail

extern "C" {

}  // extern "C"

// =============================================================================
// ensembles: many independent lattices advanced together
// =============================================================================

namespace psc_detail {

psc_status efail(psc_ensemble *E, psc_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  E->err = buf;
  if (code == PSC_EDEVICE) E->poisoned = true;
  return code;
}

#define EHIP_OK(E, call)                                                              \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return efail((E), PSC_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

psc_status ensure_member_records(psc_ensemble *E, hipStream_t stream, uint64_t n_events) {
  // every member's tape must cover the coming events; records re-uploaded
  // when a member's record changed
  bool dirty = false;
  for (size_t r = 0; r < E->members.size(); ++r) {
    psc_lattice *h = E->members[r];
    if (h->poisoned) return efail(E, PSC_EDEVICE, "member %zu is poisoned: %s", r, h->err.c_str());
    const uint64_t end = h->events_done + n_events;
    if (end >= 0xFFFFFFFFull) return efail(E, PSC_EINVAL, "event index exceeds 2^32");
    if (end > h->tape_end) {
      extend_tape(h, std::max(end, h->tape_end * 2));
      psc_status st = sync_tape(h, stream);
      if (st) return efail(E, st, "member %zu: %s", r, h->err.c_str());
    }
    if (E->versions[r] != h->version) dirty = true;
  }
  if (!dirty) return PSC_OK;
  EHIP_OK(E, hipStreamSynchronize(stream));
  std::vector<LatDev> recs(E->members.size());
  for (size_t r = 0; r < E->members.size(); ++r) {
    recs[r] = E->members[r]->L;
    E->versions[r] = E->members[r]->version;
  }
  EHIP_OK(E, hipMemcpy(E->d_lats, recs.data(), recs.size() * sizeof(LatDev),
                       hipMemcpyHostToDevice));
  return PSC_OK;
}

// some member numbers newborns of many-product collisions at its event end
bool any_births(const psc_ensemble *E) {
  for (const psc_lattice *h : E->members)
    if (h->L.wb_count) return true;
  return false;
}

psc_status ensure_graph(psc_ensemble *E) {
  if (E->exec && E->graph_grid == E->grid && E->graph_items == E->items) return PSC_OK;
  if (E->exec) {
    EHIP_OK(E, hipGraphExecDestroy(E->exec));
    E->exec = nullptr;
  }
  if (E->graph) {
    EHIP_OK(E, hipGraphDestroy(E->graph));
    E->graph = nullptr;
  }
  if (!E->cap_stream) EHIP_OK(E, hipStreamCreateWithFlags(&E->cap_stream, hipStreamNonBlocking));
  EHIP_OK(E, hipStreamBeginCapture(E->cap_stream, hipStreamCaptureModeThreadLocal));
  const hipError_t le = launch_event_multi(E->d_lats, (uint32_t)E->members.size(), E->stages,
                                           E->grid, E->items, any_births(E), E->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(E->cap_stream, &g);
  if (le != hipSuccess || ce != hipSuccess)
    return efail(E, PSC_EDEVICE, "capturing the ensemble event failed: %s / %s",
                 hipGetErrorString(le), hipGetErrorString(ce));
  E->graph = g;
  EHIP_OK(E, hipGraphInstantiate(&E->exec, E->graph, nullptr, nullptr, 0));
  E->graph_grid = E->grid;
  E->graph_items = E->items;
  return PSC_OK;
}

psc_status run_events(psc_ensemble *E, uint64_t n, hipStream_t stream) {
  if (E->use_graph) {
    psc_status st = ensure_graph(E);
    if (st) return st;
    for (uint64_t e = 0; e < n; ++e) EHIP_OK(E, hipGraphLaunch(E->exec, stream));
  } else {
    for (uint64_t e = 0; e < n; ++e)
      EHIP_OK(E, launch_event_multi(E->d_lats, (uint32_t)E->members.size(), E->stages, E->grid,
                                    E->items, any_births(E), stream));
  }
  for (psc_lattice *h : E->members) h->events_done += n;
  return PSC_OK;
}

}  // namespace psc_detail

extern "C" {

psc_status psc_ensemble_create(psc_lattice *const *members, uint32_t n, psc_ensemble **out) {
  if (!out) return PSC_EINVAL;
  *out = nullptr;
  if (!members || n == 0 || n > max_members()) {
    g_create_error = "an ensemble has 1.." + std::to_string(max_members()) + " members";
    return PSC_EINVAL;
  }
  for (uint32_t a = 0; a < n; ++a) {
    if (!members[a] || members[a]->poisoned || members[a]->in_ensemble) {
      g_create_error = "member " + std::to_string(a) + " is missing, poisoned or in an ensemble";
      return PSC_EINVAL;
    }
    for (uint32_t b = 0; b < a; ++b)
      if (members[a] == members[b]) {
        g_create_error = "a lattice appears twice";
        return PSC_EINVAL;
      }
    if (members[a]->desc.device != members[0]->desc.device) {
      g_create_error = "members must share one device";
      return PSC_EINVAL;
    }
  }
  psc_ensemble *E = new (std::nothrow) psc_ensemble();
  if (!E) return PSC_ENOMEM;
  E->members.assign(members, members + n);
  E->device = members[0]->desc.device;
  E->versions.assign(n, ~0ull);
  // freeze every member (state moves to the device)
  for (uint32_t a = 0; a < n; ++a) {
    psc_status st = psc_step(members[a], 0, nullptr);
    if (st) {
      g_create_error = "member " + std::to_string(a) + ": " + members[a]->err;
      delete E;
      return st;
    }
  }
  if (hipSetDevice(E->device) != hipSuccess ||
      hipMalloc(&E->d_lats, member_records_bytes(n)) != hipSuccess) {
    g_create_error = "device allocation of the member records failed";
    delete E;
    return PSC_ENOMEM;
  }
  // default launch: about two passes' worth of chunks for the whole ensemble
  uint64_t mol = 0;
  E->stages = 0;
  for (auto *h : E->members) {
    mol += h->desc.max_molecules;
    E->stages = std::max(E->stages, n_colours(h->geo));
  }
  const uint64_t chunks = std::max<uint64_t>(mol / E->stages / (256ull * 4), 1);
  E->grid = (int)std::min<uint64_t>(std::max<uint64_t>(chunks, 256), 4096);
  for (auto *h : E->members) h->in_ensemble = true;
  *out = E;
  return PSC_OK;
}

void psc_ensemble_destroy(psc_ensemble *E) {
  if (!E) return;
  if (!E->poisoned) {
    (void)hipSetDevice(E->device);
    (void)hipDeviceSynchronize();
  }
  if (E->exec) (void)hipGraphExecDestroy(E->exec);
  if (E->graph) (void)hipGraphDestroy(E->graph);
  if (E->cap_stream) (void)hipStreamDestroy(E->cap_stream);
  if (E->d_lats) (void)hipFree(E->d_lats);
  for (auto *h : E->members) h->in_ensemble = false;
  delete E;
}

const char *psc_ensemble_last_error(const psc_ensemble *E) {
  return E ? E->err.c_str() : g_create_error.c_str();
}

psc_status psc_ensemble_set_launch(psc_ensemble *E, const psc_launch *l) {
  if (!E || !l) return PSC_EINVAL;
  const int it = (int)l->items_per_thread;
  if (it != 0 && it != 1 && it != 2 && it != 4 && it != 8)
    return efail(E, PSC_EINVAL, "items_per_thread must be 1, 2, 4 or 8");
  if (l->stage_blocks > 65536) return efail(E, PSC_EINVAL, "stage_blocks must be <= 65536");
  if (it) E->items = it;
  if (l->stage_blocks) E->grid = (int)l->stage_blocks;
  return PSC_OK;
}

psc_status psc_ensemble_get_launch(const psc_ensemble *E, psc_launch *out) {
  if (!E || !out) return PSC_EINVAL;
  out->items_per_thread = (uint32_t)E->items;
  out->stage_blocks = (uint32_t)E->grid;
  return PSC_OK;
}

psc_status psc_ensemble_autotune(psc_ensemble *E, uint32_t trial_events) {
  if (!E) return PSC_EINVAL;
  E->autotune_events = trial_events;
  return PSC_OK;
}

psc_status psc_ensemble_tuned(const psc_ensemble *E, psc_launch *chosen, double *ms_per_event) {
  if (!E) return PSC_EINVAL;
  if (chosen) *chosen = E->tuned;
  if (ms_per_event) *ms_per_event = E->tuned_ms_per_event;
  return PSC_OK;
}

psc_status psc_ensemble_step(psc_ensemble *E, uint64_t n_events, void *stream_) {
  if (!E) return PSC_EINVAL;
  if (E->poisoned) return PSC_EDEVICE;
  hipStream_t stream = (hipStream_t)stream_;
  EHIP_OK(E, hipSetDevice(E->device));
  psc_status st = ensure_member_records(E, stream, n_events);
  if (st) return st;
  uint64_t left = n_events;
  if (E->autotune_events && left) {
    // spend the first events timing candidate shapes (the shape never
    // changes results, so these events are ordinary events of the run)
    static const int kItems[] = {2, 4, 8};
    static const int kGrids[] = {256, 512, 1024, 2048, 4096};
    hipEvent_t a, b;
    EHIP_OK(E, hipEventCreate(&a));
    EHIP_OK(E, hipEventCreate(&b));
    double best = 1e300;
    int best_items = E->items, best_grid = E->grid;
    for (int it : kItems)
      for (int gr : kGrids) {
        const uint64_t k = std::min<uint64_t>(E->autotune_events, left);
        if (k == 0) break;
        E->items = it;
        E->grid = gr;
        // one untimed event absorbs the graph rebuild
        st = run_events(E, 1, stream);
        if (st) return st;
        left -= 1;
        const uint64_t kt = std::min<uint64_t>(k, left);
        if (kt == 0) break;
        EHIP_OK(E, hipEventRecord(a, stream));
        st = run_events(E, kt, stream);
        if (st) return st;
        EHIP_OK(E, hipEventRecord(b, stream));
        EHIP_OK(E, hipEventSynchronize(b));
        float ms = 0.f;
        EHIP_OK(E, hipEventElapsedTime(&ms, a, b));
        left -= kt;
        const double per = ms / (double)kt;
        if (per < best) {
          best = per;
          best_items = it;
          best_grid = gr;
        }
      }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    E->items = best_items;
    E->grid = best_grid;
    E->tuned = psc_launch{(uint32_t)best_items, (uint32_t)best_grid};
    E->tuned_ms_per_event = best;
    E->autotune_events = 0;
  }
  return run_events(E, left, stream);
}

psc_status psc_ensemble_read(psc_ensemble *E, uint32_t i, psc_state_view *out, void *stream) {
  if (!E || !out) return PSC_EINVAL;
  if (E->poisoned) return PSC_EDEVICE;
  if (i >= E->members.size()) return efail(E, PSC_EINVAL, "member %u of %zu", i, E->members.size());
  psc_status st = psc_ensemble_sync(E);
  if (st) return st;
  st = psc_read_state(E->members[i], out, stream);
  if (st) return efail(E, st, "member %u: %s", i, E->members[i]->err.c_str());
  return PSC_OK;
}

psc_status psc_ensemble_sync(psc_ensemble *E) {
  if (!E) return PSC_EINVAL;
  if (E->poisoned) return PSC_EDEVICE;
  EHIP_OK(E, hipSetDevice(E->device));
  EHIP_OK(E, hipDeviceSynchronize());
  for (size_t r = 0; r < E->members.size(); ++r) {
    psc_status st = check_device_error(E->members[r]);
    if (st) return efail(E, st, "member %zu: %s", r, E->members[r]->err.c_str());
  }
  return PSC_OK;
}

}  // extern "C"
