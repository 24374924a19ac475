// Compositing kernels for gfx950 (CDNA4).
//
// The accumulation step of the paper (Section 4, Figures 2 and 3) folds each
// input raster into the running composite.  Here one thread owns 16 adjacent
// pixels and walks all members of the launch: per member it issues one 16-byte
// load (a 64-lane wave reads 1 KiB of contiguous HBM), splits the 4 dwords
// into 16-bit lanes with v_perm_b32 (bytes 0,2 and bytes 1,3 of each dword),
// and updates packed 16-bit accumulators: count with min(x, 1), sum with x,
// max with a packed max.  That is 10 VALU operations per dword for all three
// outputs, about half of what the VALU can issue per dword at HBM rate, so
// the kernel stays bound by memory.  After a group of at most 256 members the
// lanes are widened to 32 bits, and at the end the composite is updated in
// place once (read-modify-write): HIP buffers may be read and written by one
// kernel, while the paper's image kernels needed two accumulators used in turn
// (image objects are read-only or write-only inside a kernel, Section 5.3).
// That ping-pong form is kept as an option (PP: read one accumulator, write the
// other) to measure the paper's kernel variants.  A pass over accumulators that
// were just cleared (SET) writes the new values without reading the old ones,
// so a composite built from scratch moves member bytes plus one write of the
// composite.  No matrix cores: nothing here is a contraction.

#include "lanes.h"

#include <algorithm>

namespace cmp {
namespace {

// The composite values of 16 pixels before this launch's update.
template <bool C16>
struct Old {
  uint4 c[C16 ? 2 : 4];
  uint4 s[4];
  uint4 m;
};

template <uint32_t OUTS, bool SUB, bool C16>
__device__ __forceinline__ void load_old(Old<C16> &o, uint32_t p, const void *__restrict__ count,
                                         const uint32_t *__restrict__ sum,
                                         const uint8_t *__restrict__ mx) {
  if constexpr (OUTS & kCount) {
    const uint4 *src = C16 ? reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(count) + p)
                           : reinterpret_cast<const uint4 *>(static_cast<const uint32_t *>(count) + p);
#pragma unroll
    for (int q = 0; q < (C16 ? 2 : 4); ++q) o.c[q] = src[q];
  }
  if constexpr (OUTS & kSum) {
    const uint4 *src = reinterpret_cast<const uint4 *>(sum + p);
#pragma unroll
    for (int q = 0; q < 4; ++q) o.s[q] = src[q];
  }
  if constexpr ((OUTS & kMax) && !SUB) o.m = *reinterpret_cast<const uint4 *>(mx + p);
}

// Writes old (+ or -) new for 16 pixels starting at pixel index p; max takes
// the bytewise maximum.  cnt, sm: per-pixel 32-bit contributions; mx8: the
// new maxima as 16 bytes.
template <uint32_t OUTS, bool SUB, bool C16>
__device__ __forceinline__ void store_new(const Old<C16> &o, const uint32_t *cnt,
                                          const uint32_t *sm, const uint32_t *mx8, uint32_t p,
                                          void *__restrict__ count, uint32_t *__restrict__ sum,
                                          uint8_t *__restrict__ mx) {
  if constexpr (OUTS & kCount) {
    if constexpr (C16) {
      uint4 *dst = reinterpret_cast<uint4 *>(static_cast<uint16_t *>(count) + p);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        uint32_t ow[4] = {o.c[q].x, o.c[q].y, o.c[q].z, o.c[q].w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t nw = cnt[8 * q + 2 * k] | (cnt[8 * q + 2 * k + 1] << 16);
          ow[k] = SUB ? psub(ow[k], nw) : padd(ow[k], nw);
        }
        dst[q] = make_uint4(ow[0], ow[1], ow[2], ow[3]);
      }
    } else {
      uint4 *dst = reinterpret_cast<uint4 *>(static_cast<uint32_t *>(count) + p);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint4 v = o.c[q];
        if (SUB) {
          v.x -= cnt[4 * q]; v.y -= cnt[4 * q + 1]; v.z -= cnt[4 * q + 2]; v.w -= cnt[4 * q + 3];
        } else {
          v.x += cnt[4 * q]; v.y += cnt[4 * q + 1]; v.z += cnt[4 * q + 2]; v.w += cnt[4 * q + 3];
        }
        dst[q] = v;
      }
    }
  }
  if constexpr (OUTS & kSum) {
    uint4 *dst = reinterpret_cast<uint4 *>(sum + p);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint4 v = o.s[q];
      if (SUB) {
        v.x -= sm[4 * q]; v.y -= sm[4 * q + 1]; v.z -= sm[4 * q + 2]; v.w -= sm[4 * q + 3];
      } else {
        v.x += sm[4 * q]; v.y += sm[4 * q + 1]; v.z += sm[4 * q + 2]; v.w += sm[4 * q + 3];
      }
      dst[q] = v;
    }
  }
  if constexpr ((OUTS & kMax) && !SUB) {
    uint4 v = o.m;
    v.x = bmax(v.x, mx8[0]); v.y = bmax(v.y, mx8[1]); v.z = bmax(v.z, mx8[2]); v.w = bmax(v.w, mx8[3]);
    *reinterpret_cast<uint4 *>(mx + p) = v;
  }
}

// Output position of 16-pixel vector v: linear (identity) or tiled.
// Pixel indices fit 32 bits: the library refuses rasters of 2^32 pixels or more.
struct LinearMap {
  __device__ __forceinline__ bool pixel(uint32_t v, uint32_t &p) const {
    p = v * 16u;
    return true;
  }
};
struct TiledMap {
  uint32_t W, H, tw, th, ntx;
  __device__ __forceinline__ bool pixel(uint32_t v, uint32_t &p) const {
    const uint32_t vpr = tw >> 4;                 // vectors per tile row
    const uint32_t per_tile = vpr * th;
    const uint32_t tile = v / per_tile;
    const uint32_t in = v - tile * per_tile;
    const uint32_t r = in / vpr, c = in - r * vpr;
    const uint32_t ty = tile / ntx, tx = tile - ty * ntx;
    const uint32_t y = ty * th + r, x = tx * tw + 16u * c;
    p = y * W + x;
    return y < H && x < W;
  }
};

template <uint32_t OUTS, bool SUB, bool C16, bool MULTI, class Map, bool PP, bool SET>
__global__ __launch_bounds__(256) void k_composite(const uint8_t *const *__restrict__ tab,
                                                   int n, uint32_t nvec, Map map,
                                                   void *__restrict__ count,
                                                   uint32_t *__restrict__ sum,
                                                   uint8_t *__restrict__ mx,
                                                   const void *__restrict__ count_in,
                                                   const uint32_t *__restrict__ sum_in,
                                                   const uint8_t *__restrict__ mx_in) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvec) return;
  uint32_t p;
  if (!map.pixel(v, p)) return;
  const uint32_t off = v * 16u;
  constexpr int UNROLL = (OUTS == kCount) ? 8 : 4;

  Acc<OUTS> a;
  a.zero();
  Old<C16> old;
  if constexpr (SET) {  // cleared accumulators: nothing to read
#pragma unroll
    for (int q = 0; q < (C16 ? 2 : 4); ++q) old.c[q] = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int q = 0; q < 4; ++q) old.s[q] = make_uint4(0u, 0u, 0u, 0u);
    old.m = make_uint4(0u, 0u, 0u, 0u);
  }
  uint32_t cnt[16], sm[16], mx8[4];
  if constexpr (MULTI) {
#pragma unroll
    for (int j = 0; j < 16; ++j) cnt[j] = sm[j] = 0u;
    for (int g0 = 0; g0 < n; g0 += kGroup) {
      const int g1 = min(n, g0 + kGroup);
      fold_members<UNROLL>(tab, g0, g1, off, a);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if constexpr (OUTS & kCount) cnt[j] += lane_px(a.c, j);
        if constexpr (OUTS & kSum) sm[j] += lane_px(a.s, j);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) a.c[k] = a.s[k] = 0u;
    }
    if constexpr (SET) {
    } else if constexpr (PP) {
      load_old<OUTS, SUB, C16>(old, p, count_in, sum_in, mx_in);
    } else {
      load_old<OUTS, SUB, C16>(old, p, count, sum, mx);
    }
  } else {
    // The old composite is requested before the last members are read, so
    // its latency overlaps them instead of trailing the wave (+1-2%).
    int i = 0;
    for (; i + UNROLL < n; i += UNROLL) {
      uint4 x[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) x[u] = ld16(tab[i + u], off);
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) a.fold(x[u]);
    }
    if constexpr (SET) {
    } else if constexpr (PP) {
      load_old<OUTS, SUB, C16>(old, p, count_in, sum_in, mx_in);
    } else {
      load_old<OUTS, SUB, C16>(old, p, count, sum, mx);
    }
    {  // the last 1..UNROLL members (n >= 1)
      uint4 x[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u)
        if (i + u < n) x[u] = ld16(tab[i + u], off);
#pragma unroll
      for (int u = 0; u < UNROLL; ++u)
        if (i + u < n) a.fold(x[u]);
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      cnt[j] = lane_px(a.c, j);
      sm[j] = lane_px(a.s, j);
    }
  }
  if constexpr (OUTS & kMax) {
#pragma unroll
    for (int k = 0; k < 4; ++k) mx8[k] = __builtin_amdgcn_perm(a.m[2 * k + 1], a.m[2 * k], 0x06020400u);
  }
  store_new<OUTS, SUB, C16>(old, cnt, sm, mx8, p, count, sum, mx);
}

// Pixels [p0, npix) that do not fill a 16-pixel vector: one thread per pixel.
template <uint32_t OUTS, bool SUB, bool C16, bool PP, bool SET>
__global__ __launch_bounds__(64) void k_composite_tail(const uint8_t *const *__restrict__ tab,
                                                       int n, int64_t p0, int64_t npix,
                                                       void *__restrict__ count,
                                                       uint32_t *__restrict__ sum,
                                                       uint8_t *__restrict__ mx,
                                                       const void *__restrict__ count_in,
                                                       const uint32_t *__restrict__ sum_in,
                                                       const uint8_t *__restrict__ mx_in) {
  const int64_t p = p0 + threadIdx.x;
  if (p >= npix) return;
  uint32_t c = 0, s = 0, m = 0;
  for (int i = 0; i < n; ++i) {
    const uint32_t x = tab[i][p];
    c += x != 0u;
    s += x;
    m = x > m ? x : m;
  }
  if constexpr (OUTS & kCount) {
    if constexpr (C16) {
      const uint16_t o = SET ? 0 : static_cast<const uint16_t *>(PP ? count_in : count)[p];
      static_cast<uint16_t *>(count)[p] = (uint16_t)(SUB ? o - c : o + c);
    } else {
      const uint32_t o = SET ? 0u : static_cast<const uint32_t *>(PP ? count_in : count)[p];
      static_cast<uint32_t *>(count)[p] = SUB ? o - c : o + c;
    }
  }
  if constexpr (OUTS & kSum) {
    const uint32_t o = SET ? 0u : (PP ? sum_in : sum)[p];
    sum[p] = SUB ? o - s : o + s;
  }
  if constexpr ((OUTS & kMax) && !SUB) {
    const uint32_t o = SET ? 0u : (PP ? mx_in : mx)[p];
    mx[p] = (uint8_t)(m > o ? m : o);
  }
}

template <uint32_t OUTS, bool SUB, bool C16, class Map>
hipError_t go(const uint8_t *const *tab, int n, int64_t nvec, const Map &map,
              const Outputs &o, hipStream_t s) {
  if (nvec <= 0) return hipSuccess;
  if (nvec >= (int64_t(1) << 28)) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((nvec + 255) / 256);
  const bool pp = o.count_in || o.sum_in || o.max_in;
#define CMP_GO(MULTI, PP, SET)                                                                   \
  k_composite<OUTS, SUB, C16, MULTI, Map, PP, SET><<<blocks, 256, 0, s>>>(                       \
      tab, n, (uint32_t)nvec, map, o.count, o.sum, o.max, o.count_in, o.sum_in, o.max_in)
  if (o.set) {
    // cleared accumulators are written, never read (and never subtracted from)
    if constexpr (SUB) return hipErrorInvalidValue;
    else if (n > kGroup) CMP_GO(true, false, true);
    else CMP_GO(false, false, true);
  } else if (n > kGroup) {
    if (pp) CMP_GO(true, true, false);
    else CMP_GO(true, false, false);
  } else {
    if (pp) CMP_GO(false, true, false);
    else CMP_GO(false, false, false);
  }
#undef CMP_GO
  return hipGetLastError();
}

template <uint32_t OUTS, bool SUB, bool C16>
hipError_t go_tail(const uint8_t *const *tab, int n, int64_t p0, int64_t npix,
                   const Outputs &o, hipStream_t s) {
  if (npix <= p0) return hipSuccess;
  if (o.set) {
    if constexpr (SUB) return hipErrorInvalidValue;
    else
      k_composite_tail<OUTS, SUB, C16, false, true><<<1, 64, 0, s>>>(tab, n, p0, npix, o.count, o.sum,
                                                                     o.max, o.count_in, o.sum_in, o.max_in);
  } else if (o.count_in || o.sum_in || o.max_in) {
    k_composite_tail<OUTS, SUB, C16, true, false><<<1, 64, 0, s>>>(tab, n, p0, npix, o.count, o.sum, o.max,
                                                                   o.count_in, o.sum_in, o.max_in);
  } else {
    k_composite_tail<OUTS, SUB, C16, false, false><<<1, 64, 0, s>>>(tab, n, p0, npix, o.count, o.sum,
                                                                    o.max, o.count_in, o.sum_in, o.max_in);
  }
  return hipGetLastError();
}

template <uint32_t O, bool S, bool C>
hipError_t run_linear(const uint8_t *const *tab, int n, int64_t npix, const Outputs &o,
                      hipStream_t s) {
  const int64_t nvec = npix / 16;
  hipError_t e = go<O, S, C>(tab, n, nvec, LinearMap{}, o, s);
  if (e != hipSuccess) return e;
  return go_tail<O, S, C>(tab, n, nvec * 16, npix, o, s);
}

template <uint32_t O, bool S, bool C>
hipError_t run_tiled(const uint8_t *const *tab, int n, int64_t nvec, const TiledMap &map,
                     const Outputs &o, hipStream_t s) {
  return go<O, S, C>(tab, n, nvec, map, o, s);
}

// Runtime (outs, sub, count16) -> template instance of FN<O, S, C>(ARGS).
#define CMP_DISPATCH(FN, outs, sub, c16, ...)                                   \
  do {                                                                          \
    switch (outs) {                                                             \
      CMP_DISPATCH_CASE(FN, 1, sub, c16, __VA_ARGS__)                           \
      CMP_DISPATCH_CASE(FN, 2, sub, c16, __VA_ARGS__)                           \
      CMP_DISPATCH_CASE(FN, 3, sub, c16, __VA_ARGS__)                           \
      CMP_DISPATCH_CASE(FN, 4, sub, c16, __VA_ARGS__)                           \
      CMP_DISPATCH_CASE(FN, 5, sub, c16, __VA_ARGS__)                           \
      CMP_DISPATCH_CASE(FN, 6, sub, c16, __VA_ARGS__)                           \
      CMP_DISPATCH_CASE(FN, 7, sub, c16, __VA_ARGS__)                           \
      default:                                                                  \
        return hipErrorInvalidValue;                                            \
    }                                                                           \
  } while (0)
#define CMP_DISPATCH_CASE(FN, O, sub, c16, ...)                                 \
  case O:                                                                       \
    if (sub)                                                                    \
      return c16 ? FN<O, true, true>(__VA_ARGS__) : FN<O, true, false>(__VA_ARGS__); \
    return c16 ? FN<O, false, true>(__VA_ARGS__) : FN<O, false, false>(__VA_ARGS__);

}  // namespace

hipError_t launch_composite_linear(const uint8_t *const *d_tab, int n, int64_t npix,
                                   const Outputs &o, uint32_t outs, bool sub, hipStream_t s) {
  if (n <= 0 || npix <= 0) return hipSuccess;
  CMP_DISPATCH(run_linear, outs, sub, o.count16, d_tab, n, npix, o, s);
}

hipError_t launch_composite_tiled(const uint8_t *const *d_tab, int n, const Tiling &t,
                                  const Outputs &o, uint32_t outs, bool sub, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (t.W % 16 || t.tw % 16) return hipErrorInvalidValue;
  const TiledMap map{(uint32_t)t.W, (uint32_t)t.H, (uint32_t)t.tw, (uint32_t)t.th, (uint32_t)t.ntx()};
  const int64_t nvec = t.plane() / 16;
  CMP_DISPATCH(run_tiled, outs, sub, o.count16, d_tab, n, nvec, map, o, s);
}

}  // namespace cmp
