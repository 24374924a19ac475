// Internal launch interface of the compositing kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmp {

// Members composited by one pass; sums of up to this many uint8 values fit the
// 16-bit lanes the kernels accumulate in (256 * 255 < 65536).
constexpr int kGroup = 256;

enum : uint32_t { kCount = 1, kSum = 2, kMax = 4 };

// Where a launch writes the composite and, when the *_in pointers are set,
// where it reads the previous values from (two accumulators used in turn);
// otherwise the update is in place.  A launch that writes an output reads it
// from its *_in pointer if any *_in pointer is set.  With set, the previous
// values are all zero (cleared accumulators): nothing is read, the new values
// are written (an add only; the *_in pointers are ignored).
struct Outputs {
  void *count = nullptr;     // uint16_t* or uint32_t*
  uint32_t *sum = nullptr;
  uint8_t *max = nullptr;
  bool count16 = false;
  bool set = false;
  const void *count_in = nullptr;
  const uint32_t *sum_in = nullptr;
  const uint8_t *max_in = nullptr;
};

// Geometry of the tiled staging layout: tiles of tw bytes x th rows, stored
// tile after tile in row-major tile order, each tile row-major.
struct Tiling {
  int32_t W = 0, H = 0, tw = 0, th = 0;
  int64_t ntx() const { return (W + tw - 1) / tw; }
  int64_t nty() const { return (H + th - 1) / th; }
  int64_t plane() const { return ntx() * nty() * (int64_t)tw * th; }
};

// count/sum += (or -=) the members' contribution, max = max(max, members),
// for `outs` (kCount|kSum|kMax) over n members given by a device table of
// device pointers, each W*H row-major bytes (npix = W*H), any alignment.
hipError_t launch_composite_linear(const uint8_t *const *d_tab, int n, int64_t npix,
                                   const Outputs &o, uint32_t outs, bool sub,
                                   hipStream_t s);

// Same for members stored in the tiled layout (W must be a multiple of 16).
hipError_t launch_composite_tiled(const uint8_t *const *d_tab, int n, const Tiling &t,
                                  const Outputs &o, uint32_t outs, bool sub,
                                  hipStream_t s);

// Repacks n row-major members (src + i*src_stride) into the tiled layout
// (dst + i*dst_stride).  Padding bytes of edge tiles are written as zero.
hipError_t launch_repack_tiled(const uint8_t *src, int64_t src_stride, uint8_t *dst,
                               int64_t dst_stride, int n, const Tiling &t,
                               hipStream_t s);

// Fills `bytes` bytes at p (16-byte aligned) with `value`.  A kernel, not a
// memset, so it is safe inside captured graphs.
hipError_t launch_fill(void *p, uint8_t value, int64_t bytes, hipStream_t s);

// Copies the window (x0, y0, w, h) of a row-major W-wide array of elem-byte
// elements to dst, dst_pitch bytes between rows (device memory).
hipError_t launch_pack_window(const void *src, int elem, int32_t W, int32_t x0,
                              int32_t y0, int32_t w, int32_t h, void *dst,
                              int64_t dst_pitch, hipStream_t s);

// Histogram of a count array (uint16 or uint32, npix values) into nbins
// uint64 device counters (zeroed by the caller) plus one overflow counter at
// bins[nbins].  Bins live in LDS per workgroup when nbins <= kLdsBins.
constexpr int kLdsBins = 8192;
hipError_t launch_histogram(const void *count, bool count16, int64_t npix, int32_t nbins,
                            unsigned long long *bins, int cus, hipStream_t s);

}  // namespace cmp
