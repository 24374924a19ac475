// Utility kernels for gfx950: the fill that clears accumulators inside
// captured graphs, the window copy into device memory (the retrieval of
// results, Section 1), and the overlap-class histogram of a count composite
// (Figure 1, lower-left panel).

#include "kernels.h"

#include <algorithm>

namespace cmp {
namespace {

__global__ __launch_bounds__(256) void k_fill(uint8_t *__restrict__ p, uint32_t word,
                                              int64_t nvec, int64_t bytes) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nvec) reinterpret_cast<uint4 *>(p)[v] = make_uint4(word, word, word, word);
  if (v == 0)
    for (int64_t b = nvec * 16; b < bytes; ++b) p[b] = (uint8_t)word;
}

// Row y of the window: w elements of source row y0 + y from column x0.  VEC:
// the source and destination rows all start on 16-byte boundaries, so each
// thread moves 16 bytes and the row's last (w * sizeof(T)) % 16 bytes go
// element by element; otherwise one element per thread.
template <class T, bool VEC>
__global__ __launch_bounds__(256) void k_pack(const T *__restrict__ src, int32_t W, int32_t x0,
                                              int32_t y0, int32_t w, int32_t h,
                                              uint8_t *__restrict__ dst, int64_t dst_pitch) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t y = blockIdx.y;
  if (y >= h) return;
  const T *s = src + (int64_t)(y0 + y) * W + x0;
  T *d = reinterpret_cast<T *>(dst + (int64_t)y * dst_pitch);
  if constexpr (VEC) {
    constexpr int32_t E = 16 / sizeof(T);  // elements per 16-byte vector
    const int32_t nv = w / E;
    if (t < nv) {
      reinterpret_cast<uint4 *>(d)[t] = reinterpret_cast<const uint4 *>(s)[t];
    } else {
      const int32_t x = nv * E + (t - nv);
      if (x < w) d[x] = s[x];
    }
  } else if (t < w) {
    d[t] = s[t];
  }
}

// One workgroup walks a contiguous band of vectors of 8 counts and counts them
// into bins privatized in LDS (or straight into global memory for large bin
// counts), one atomic per run of equal values; LDS bins are flushed once per
// workgroup.
template <bool C16, bool LDS>
__global__ __launch_bounds__(256) void k_histogram(const void *__restrict__ count, uint32_t npix,
                                                   int32_t nbins,
                                                   unsigned long long *__restrict__ bins) {
  extern __shared__ uint32_t sh[];
  if constexpr (LDS) {
    for (int b = threadIdx.x; b <= nbins; b += blockDim.x) sh[b] = 0u;
    __syncthreads();
  }
  auto put = [&](uint32_t c, uint32_t k) {
    const int b = c < (uint32_t)nbins ? (int)c : nbins;
    if constexpr (LDS) atomicAdd(&sh[b], k);
    else atomicAdd(&bins[b], (unsigned long long)k);
  };
  // Neighbouring pixels of a composite mostly share their class: a run of
  // equal values among a thread's 8 pixels costs one atomic.
  auto put8 = [&](const uint32_t (&c)[8]) {
    uint32_t cur = c[0], run = 1;
#pragma unroll
    for (int k = 1; k < 8; ++k) {
      if (c[k] == cur) {
        ++run;
      } else {
        put(cur, run);
        cur = c[k];
        run = 1;
      }
    }
    put(cur, run);
  };
  // one vector of 8 counts: 16 bytes of u16 or 32 bytes of u32
  typedef uint4 vec_t[C16 ? 1 : 2];
  auto load = [&](uint32_t v, vec_t &x) {
    const uint4 *p = reinterpret_cast<const uint4 *>(count) + (C16 ? 1 : 2) * (size_t)v;
#pragma unroll
    for (int h = 0; h < (C16 ? 1 : 2); ++h) x[h] = p[h];
  };
  auto count8 = [&](const vec_t &x) {
    if constexpr (C16) {
      const uint32_t c[8] = {x[0].x & 0xffffu, x[0].x >> 16, x[0].y & 0xffffu, x[0].y >> 16,
                             x[0].z & 0xffffu, x[0].z >> 16, x[0].w & 0xffffu, x[0].w >> 16};
      put8(c);
    } else {
      const uint32_t c[8] = {x[0].x, x[0].y, x[0].z, x[0].w, x[1].x, x[1].y, x[1].z, x[1].w};
      put8(c);
    }
  };
  // Each workgroup takes one contiguous band of the composite: a band of a
  // smooth composite holds few of its classes, so the workgroup's flush
  // below touches few bins (with a grid stride every workgroup met every
  // class, and the flush's global atomics, all workgroups' at once, were a
  // visible part of the kernel).
  const uint32_t nv = npix / 8;
  const uint32_t stride = blockDim.x;
  const uint32_t per = (nv + gridDim.x - 1) / gridDim.x;
  const uint32_t v1 = min(nv, blockIdx.x * per + per);  // nv < 2^29: no overflow
  uint32_t v = blockIdx.x * per + threadIdx.x;
  // four steps at a time, their loads issued before any atomic, so that each
  // wave keeps several loads in flight
  for (; v + 3 * stride < v1; v += 4 * stride) {
    vec_t x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) load(v + u * stride, x[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) count8(x[u]);
  }
  for (; v < v1; v += stride) {
    vec_t x;
    load(v, x);
    count8(x);
  }
  // the last npix % 8 values
  if (blockIdx.x == 0 && threadIdx.x < npix - nv * 8) {
    const uint32_t i = nv * 8 + threadIdx.x;
    put(C16 ? static_cast<const uint16_t *>(count)[i] : static_cast<const uint32_t *>(count)[i], 1u);
  }
  if constexpr (LDS) {
    __syncthreads();
    for (int b = threadIdx.x; b <= nbins; b += blockDim.x)
      if (sh[b]) atomicAdd(&bins[b], (unsigned long long)sh[b]);
  }
}

}  // namespace

hipError_t launch_histogram(const void *count, bool count16, int64_t npix, int32_t nbins,
                            unsigned long long *bins, int cus, hipStream_t s) {
  if (npix <= 0) return hipSuccess;
  if (npix >= (int64_t(1) << 32) || nbins < 1) return hipErrorInvalidValue;
  const bool lds = nbins <= kLdsBins;
  const int64_t nv = npix / 8;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nv + 255) / 256, (int64_t)cus * 2));
  const size_t shm = lds ? sizeof(uint32_t) * (nbins + 1) : 0;
  if (count16) {
    if (lds) k_histogram<true, true><<<grid, 256, shm, s>>>(count, (uint32_t)npix, nbins, bins);
    else k_histogram<true, false><<<grid, 256, 0, s>>>(count, (uint32_t)npix, nbins, bins);
  } else {
    if (lds) k_histogram<false, true><<<grid, 256, shm, s>>>(count, (uint32_t)npix, nbins, bins);
    else k_histogram<false, false><<<grid, 256, 0, s>>>(count, (uint32_t)npix, nbins, bins);
  }
  return hipGetLastError();
}

hipError_t launch_fill(void *p, uint8_t value, int64_t bytes, hipStream_t s) {
  if (bytes <= 0) return hipSuccess;
  const uint32_t word = 0x01010101u * value;
  const int64_t nvec = bytes / 16;
  const int64_t blocks = nvec > 0 ? (nvec + 255) / 256 : 1;
  k_fill<<<(unsigned)blocks, 256, 0, s>>>(static_cast<uint8_t *>(p), word, nvec, bytes);
  return hipGetLastError();
}

hipError_t launch_pack_window(const void *src, int elem, int32_t W, int32_t x0, int32_t y0,
                              int32_t w, int32_t h, void *dst, int64_t dst_pitch,
                              hipStream_t s) {
  if (w <= 0 || h <= 0) return hipSuccess;
  if (elem != 1 && elem != 2 && elem != 4) return hipErrorInvalidValue;
  // 16-byte moves when every source row and every destination row of the
  // window starts on a 16-byte boundary
  const bool vec = (reinterpret_cast<uintptr_t>(src) & 15u) == 0 && ((int64_t)W * elem) % 16 == 0 &&
                   ((int64_t)x0 * elem) % 16 == 0 && (reinterpret_cast<uintptr_t>(dst) & 15u) == 0 &&
                   dst_pitch % 16 == 0;
  const int32_t E = 16 / elem;
  const int32_t per_row = vec ? w / E + w % E : w;  // threads per row
  // one grid row per window row, at most 65535 rows per launch
  for (int32_t r0 = 0; r0 < h; r0 += 65535) {
    const int32_t hr = std::min<int32_t>(65535, h - r0);
    dim3 grid((unsigned)((per_row + 255) / 256), (unsigned)hr);
    uint8_t *d = static_cast<uint8_t *>(dst) + (int64_t)r0 * dst_pitch;
#define CMP_PACK(T)                                                                                    \
  do {                                                                                                 \
    if (vec)                                                                                           \
      k_pack<T, true><<<grid, 256, 0, s>>>(static_cast<const T *>(src), W, x0, y0 + r0, w, hr, d, dst_pitch); \
    else                                                                                               \
      k_pack<T, false><<<grid, 256, 0, s>>>(static_cast<const T *>(src), W, x0, y0 + r0, w, hr, d, dst_pitch); \
  } while (0)
    switch (elem) {
      case 1: CMP_PACK(uint8_t); break;
      case 2: CMP_PACK(uint16_t); break;
      default: CMP_PACK(uint32_t); break;
    }
#undef CMP_PACK
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace cmp
