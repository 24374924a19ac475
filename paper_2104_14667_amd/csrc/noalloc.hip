// Compositing of device-resident members into caller-owned accumulators,
// without any allocation: the accumulation kernel step of the paper's two
// listings (Section 4) over rasters already in device memory, as
// composite_add_device runs it, for callers that cannot allocate device memory
// (code under stream capture, tight serving loops).
//
// The compositing kernel reads its members through a device table of pointers.
// composite_add_device keeps that table in memory its context allocates; here
// it lives in one file-scope device array of fixed size, `scratch`, that every
// call on a GPU shares.  The table is written by a small kernel that takes up
// to kTableChunk pointers as its argument, so the call enqueues kernels only:
// no allocation, no host-to-device copy from pageable memory, no memset.

#include <hip/hip_runtime.h>

#include <mutex>

#include "composite.h"
#include "kernels.h"

// The member table of every call on this GPU (each GPU holds its own copy,
// until the process ends).  In host code this name is not a device address:
// kernels get the address from hipGetSymbolAddress (scratch_of below).
static __device__ __align__(256) const uint8_t *scratch[CMP_STATIC_MAX_MEMBERS];

namespace {

constexpr int kTableChunk = 256;  // pointers per table-writing launch (2 KiB of arguments)
constexpr int kMaxDevices = 64;

static_assert(CMP_STATIC_MAX_MEMBERS % kTableChunk == 0, "whole table chunks");

struct TableChunk {
  const uint8_t *p[kTableChunk];
};

__global__ __launch_bounds__(kTableChunk) void k_table(TableChunk c, const uint8_t **dst, int cnt) {
  const int i = threadIdx.x;
  if (i < cnt) dst[i] = c.p[i];
}

std::mutex g_mu;
const uint8_t **g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_of(const uint8_t ***out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CMP_EDEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CMP_EDEVICE;
    g_scratch[dev] = static_cast<const uint8_t **>(p);
  }
  *out = g_scratch[dev];
  return CMP_OK;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

extern "C" int composite_accumulate_static(const uint8_t *const *dev_maps, int32_t n, int32_t W,
                                           int32_t H, uint32_t outputs, int32_t count_bits,
                                           void *dev_count, uint32_t *dev_sum, uint8_t *dev_max,
                                           int32_t set, void *stream) {
  // every check before anything is enqueued
  if (W < 1 || H < 1 || n < 0 || (set != 0 && set != 1)) return CMP_EINVAL;
  if (outputs == 0 || (outputs & ~(uint32_t)(CMP_COUNT | CMP_SUM | CMP_MAX))) return CMP_EINVAL;
  const int64_t npix = (int64_t)W * H;
  if (npix > (int64_t(1) << 32) - 16) return CMP_EINVAL;
  if (outputs & CMP_COUNT) {
    if (count_bits != 16 && count_bits != 32) return CMP_EINVAL;
    if (!dev_count || !aligned16(dev_count)) return CMP_EINVAL;
  }
  if ((outputs & CMP_SUM) && (!dev_sum || !aligned16(dev_sum))) return CMP_EINVAL;
  if ((outputs & CMP_MAX) && (!dev_max || !aligned16(dev_max))) return CMP_EINVAL;
  if (n > 0 && !dev_maps) return CMP_EINVAL;
  for (int32_t i = 0; i < n; ++i)
    if (!dev_maps[i]) return CMP_EINVAL;
  if (n > CMP_STATIC_MAX_MEMBERS) return CMP_ERANGE;
  if (n == 0 && !set) return CMP_OK;

  const uint8_t **tab = nullptr;
  int rc = scratch_of(&tab);
  if (rc != CMP_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool c16 = (outputs & CMP_COUNT) && count_bits == 16;

  if (n == 0) {
    // the composite of the empty set: every selected output is zero
    const int64_t cb = c16 ? 2 : 4;
    if ((outputs & CMP_COUNT) && cmp::launch_fill(dev_count, 0, npix * cb, s) != hipSuccess)
      return CMP_EDEVICE;
    if ((outputs & CMP_SUM) && cmp::launch_fill(dev_sum, 0, npix * 4, s) != hipSuccess)
      return CMP_EDEVICE;
    if ((outputs & CMP_MAX) && cmp::launch_fill(dev_max, 0, npix, s) != hipSuccess)
      return CMP_EDEVICE;
    return CMP_OK;
  }

  // the member table, written on the caller's stream ahead of the kernel
  for (int32_t i0 = 0; i0 < n; i0 += kTableChunk) {
    const int cnt = n - i0 < kTableChunk ? n - i0 : kTableChunk;
    TableChunk c;
    for (int k = 0; k < kTableChunk; ++k) c.p[k] = k < cnt ? dev_maps[i0 + k] : nullptr;
    k_table<<<1, kTableChunk, 0, s>>>(c, tab + i0, cnt);
    if (hipGetLastError() != hipSuccess) return CMP_EDEVICE;
  }
  cmp::Outputs o;
  o.count16 = c16;
  o.set = set != 0;
  if (outputs & CMP_COUNT) o.count = dev_count;
  if (outputs & CMP_SUM) o.sum = dev_sum;
  if (outputs & CMP_MAX) o.max = dev_max;
  if (cmp::launch_composite_linear(tab, n, npix, o, outputs, false, s) != hipSuccess) return CMP_EDEVICE;
  return CMP_OK;
}
