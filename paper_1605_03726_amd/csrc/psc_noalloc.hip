// psc_noalloc.hip -- psc_read_state_noalloc: the state read-back of
// psc_read_state without any device allocation, for callers that cannot
// allocate.  psc_read_state converts the bricked occupancy to the ABI's
// linear order through a transient device buffer as large as the lattice;
// this variant converts one layer of bricks (4 k-layers, a contiguous range
// in both orders) at a time through a fixed static device buffer and copies
// each converted range straight into the caller's array.
#include <mutex>
#include <vector>

#include "psc_internal.h"

using namespace psc;
using namespace psc_detail;

// Staging buffer of every GPU the library runs on (held until the process
// ends).  Host code never passes `scratch` itself to a kernel or a copy: it
// uses the device address that hipGetSymbolAddress gives on each device.
static constexpr uint64_t kScratchWords = (32ull << 20) / sizeof(uint16_t);  // 32 MiB
static __device__ __align__(256) uint16_t scratch[kScratchWords];

namespace {

std::mutex g_scratch_mu;
std::vector<uint16_t *> g_scratch_ptr;  // by device ordinal; null until looked up

// the device address of `scratch` on `device` (current), looked up once
hipError_t scratch_on(int device, uint16_t **out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if ((size_t)device >= g_scratch_ptr.size()) g_scratch_ptr.resize(device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (uint16_t *)p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// dst[linear(u) - lin0] = the species at layout index u, for the n layout indices
// u = first, first + 1, ... (a range that is also contiguous in linear
// order, starting at lin0)
__global__ void __launch_bounds__(256) k_range_to_linear(Geo g, const uint16_t *__restrict__ occ,
                                                         uint64_t first, uint64_t n, uint64_t lin0,
                                                         uint16_t *__restrict__ dst) {
  for (uint64_t z = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; z < n;
       z += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t u = (uint32_t)(first + z);
    const uint64_t lin = g.brick ? (uint64_t)linear_of(g, coord_of(g, u)) : (uint64_t)u;
    dst[lin - lin0] = (uint16_t)(occ[u] & kSpeciesBits);
  }
}

struct NoallocCtx {
  hipStream_t stream;
  uint16_t *buf;  // device address of `scratch` on the lattice's device
};

// Ranges: with bricks, one layer of bricks (4 ni nj voxels) is contiguous in
// layout order (bricks in k-major order) and covers k-layers 4 kb .. 4 kb + 3,
// which are contiguous in linear order too; as many whole layers as fit the
// buffer go per copy.  Without bricks the orders coincide and any range will
// do.
psc_status read_occupancy_scratch(psc_lattice *h, uint16_t *occp, void *vctx) {
  const NoallocCtx &c = *(const NoallocCtx *)vctx;
  const uint64_t unit = h->geo.brick ? 4ull * h->geo.ni * h->geo.nj : 1ull;
  const uint64_t per = (kScratchWords / unit) * unit;
  for (uint64_t first = 0; first < h->nv; first += per) {
    const uint64_t n = std::min<uint64_t>(per, h->nv - first);
    const int grid = (int)std::min<uint64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_range_to_linear, dim3(grid), dim3(256), 0, c.stream, h->geo, h->L.occ,
                       first, n, first, c.buf);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(occp + first, c.buf, n * sizeof(uint16_t), hipMemcpyDeviceToHost,
                         c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess)
      return fail(h, PSC_EDEVICE, "occupancy read through the static buffer failed: %s",
                  hipGetErrorString(e));
  }
  return PSC_OK;
}

}  // namespace

extern "C" {

psc_status psc_read_state_noalloc(psc_lattice *h, psc_state_view *out, void *stream) {
  if (!h || !out) return PSC_EINVAL;
  if (h->poisoned) return PSC_EDEVICE;
  NoallocCtx ctx{(hipStream_t)stream, nullptr};
  if (h->frozen) {
    const uint64_t unit = h->geo.brick ? 4ull * h->geo.ni * h->geo.nj : 1ull;
    if (unit > kScratchWords)
      return fail(h, PSC_EINVAL,
                  "a layer of bricks of this lattice (4 ni nj = %llu voxels) exceeds the "
                  "static staging buffer of %llu voxels; use psc_read_state",
                  (unsigned long long)unit, (unsigned long long)kScratchWords);
    const hipError_t e0 = hipSetDevice(h->desc.device);
    const hipError_t e = e0 == hipSuccess ? scratch_on(h->desc.device, &ctx.buf) : e0;
    if (e != hipSuccess)
      return fail(h, PSC_EDEVICE, "device address of the static staging buffer: %s",
                  hipGetErrorString(e));
  }
  return read_state_with(h, out, read_occupancy_scratch, &ctx);
}

}  // extern "C"
