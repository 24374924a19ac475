// Batched crop requests against a device-resident pool (composite_pool_*,
// composite_batch_*).
//
// A request = (pool ids, crop window) -> uint32 member count of the window.
// The host turns a batch into work items (request, band of whole crop rows of
// about tile_vecs 16-pixel vectors), ordered by decreasing cost, and uploads
// one descriptor arena.  One persistent launch of blocks_per_cu workgroups per
// compute unit then pulls items from an atomic counter until the queue is
// empty, so small and large requests share the whole chip in one launch; the
// launch (queue reset + kernel) is captured once into a hipGraph and replayed,
// its per-batch data living in the arena it reads.  The per-request mode runs
// one plain launch per request, in order, as the baseline.
//
// The shared mode reads each pool raster's bytes once for all the requests
// that want them: a workgroup owns a tile of 1024 pixels of one raster row,
// finds the requests whose windows cover it (up to S per pass), marks in LDS
// which of them hold each pool member, and streams every marked member's
// tile once, adding its nonzero pixels to an LDS accumulator per covering
// request that holds it.  The accumulators then go to those requests'
// outputs.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/composite.h"
#include "lanes.h"
#include "pool.h"

namespace {

struct ReqDesc {
  uint32_t *out;
  int64_t pitch;      // elements
  int32_t ids_off;    // into the arena's id array
  int32_t n;
  int32_t x0, y0, w, h;
  int32_t nvr;        // 16-pixel vectors per crop row
  int32_t pad;
};
struct Item {
  int32_t req, row0, nrows, pad;
};
struct Header {
  int32_t nitems, nreq;
  int64_t reqs_off, items_off, ids_off;  // byte offsets in the arena
  int64_t bits_off;                      // matrix mode: M of each request block
  int64_t pad[3];
};
static_assert(sizeof(Header) == 64, "arena header is 64 bytes");

// Output pointers read from the arena are generic; as global-space pointers
// their stores are global (not flat) stores, which count only against the
// vector-memory counter.
typedef __attribute__((address_space(1))) uint32_t gu32_t;
typedef unsigned int u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));  // 4-byte aligned
__device__ __forceinline__ gu32_t *as_global(uint32_t *p) { return (gu32_t *)p; }

// Counts of one 16-pixel vector of a request: pixels (y, x .. x+15) of the
// pool rasters ids[0..n), written to out[0..valid).
template <bool NT>
__device__ __forceinline__ void crop_vector(const uint8_t *__restrict__ base, int64_t stride,
                                            const int32_t *__restrict__ ids, int n, uint32_t off,
                                            gu32_t *__restrict__ out, int valid) {
  constexpr int U = 8;
  uint32_t cnt[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) cnt[j] = 0u;
  for (int g0 = 0; g0 < n; g0 += cmp::kGroup) {
    const int g1 = min(n, g0 + cmp::kGroup);
    cmp::Acc<cmp::kCount> a;
    a.zero();
    int i = g0;
    for (; i + U <= g1; i += U) {
      uint4 x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = cmp::ld16_t<NT>(base + (int64_t)ids[i + u] * stride, off);
#pragma unroll
      for (int u = 0; u < U; ++u) a.fold(x[u]);
    }
    for (; i < g1; ++i) a.fold(cmp::ld16_t<NT>(base + (int64_t)ids[i] * stride, off));
#pragma unroll
    for (int j = 0; j < 16; ++j) cnt[j] += cmp::lane_px(a.c, j);
  }
  if (valid == 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      u32x4a4 v;
      v.x = cnt[4 * q];
      v.y = cnt[4 * q + 1];
      v.z = cnt[4 * q + 2];
      v.w = cnt[4 * q + 3];
      *(__attribute__((address_space(1))) u32x4a4 *)(out + 4 * q) = v;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (j < valid) out[j] = cnt[j];
  }
}

template <bool NT>
__global__ __launch_bounds__(256) void k_batch(const uint8_t *__restrict__ base, int64_t stride,
                                               int32_t W, const char *__restrict__ arena,
                                               uint32_t *__restrict__ queue) {
  const Header *hd = reinterpret_cast<const Header *>(arena);
  const int nitems = hd->nitems;
  const ReqDesc *reqs = reinterpret_cast<const ReqDesc *>(arena + hd->reqs_off);
  const Item *items = reinterpret_cast<const Item *>(arena + hd->items_off);
  const int32_t *ids_all = reinterpret_cast<const int32_t *>(arena + hd->ids_off);
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();  // s_item is rewritten only after every thread read it
    if (it >= nitems) break;  // the queue counter only grows: every wave exits
    const Item I = items[it];
    const ReqDesc R = reqs[I.req];
    const int32_t *ids = ids_all + R.ids_off;
    const int total = I.nrows * R.nvr;
    for (int v = threadIdx.x; v < total; v += blockDim.x) {
      const int row = v / R.nvr, j = v - row * R.nvr;
      const uint32_t off = (uint32_t)(R.y0 + I.row0 + row) * (uint32_t)W + (uint32_t)(R.x0 + 16 * j);
      gu32_t *out = as_global(R.out) + (int64_t)(I.row0 + row) * R.pitch + 16 * j;
      crop_vector<NT>(base, stride, ids, R.n, off, out, min(16, R.w - 16 * j));
    }
  }
}

// ---------------------------------------------------------------- shared mode

constexpr int kShTile = 1024;   // pixels per tile
constexpr int kShMaxSlots = 32; // requests per pass (bits of a member mask)
constexpr int kShUnroll = 8;    // member loads per group (two groups in flight)
// Members streamed between flushes of the 8-bit accumulators (each byte lane
// then holds at most this many, < 256); a multiple of two groups.
constexpr int kShFlush = 240;
static_assert(kShFlush % (2 * kShUnroll) == 0 && kShFlush < 256, "flush interval");
constexpr int kShPad = 3 * kShUnroll;  // list entries the prefetch may read past the end

typedef unsigned int u32u __attribute__((aligned(1)));
typedef const __attribute__((address_space(1))) u32u gu32u;
typedef unsigned int u32x2u __attribute__((ext_vector_type(2), aligned(1)));
typedef const __attribute__((address_space(1))) u32x2u gu32x2u;

// Nonzero flags of the 4 bytes of w, one per byte (0 or 1): bit 7 of
// (b & 0x7f) + 0x7f is set iff the low 7 bits are nonzero, and b's own bit 7
// covers the rest; no byte carries into the next.
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t w) {
  const uint32_t t = ((w & 0x7f7f7f7fu) + 0x7f7f7f7fu) | w;
  return (t >> 7) & 0x01010101u;
}

// PX pixels of one raster per thread (4 or 8 bytes, any alignment), and their
// nonzero flags as 8-bit lanes of one LDS accumulator word.
template <int PX> struct ShPx;
template <> struct ShPx<4> {
  typedef uint32_t Acc;
  template <bool NT> __device__ static uint32_t load(const uint8_t *p) {
    if constexpr (NT) return __builtin_nontemporal_load((gu32u *)p);
    else return *(gu32u *)p;
  }
  __device__ static Acc flags(uint32_t w) { return nonzero_bytes(w); }
};
template <> struct ShPx<8> {
  typedef unsigned long long Acc;
  template <bool NT> __device__ static unsigned long long load(const uint8_t *p) {
    u32x2u v;
    if constexpr (NT) v = __builtin_nontemporal_load((gu32x2u *)p);
    else v = *(gu32x2u *)p;
    return ((unsigned long long)v.y << 32) | v.x;
  }
  __device__ static Acc flags(unsigned long long w) {
    return ((unsigned long long)nonzero_bytes((uint32_t)(w >> 32)) << 32) | nonzero_bytes((uint32_t)w);
  }
};

// LDS of k_shared: acc8[S][TPB] accumulator words (PX 8-bit counts per thread
// and request), bits[count + kShPad] member masks (compacted in place into the
// masks of the listed members), ids[count + kShPad] listed member ids.
__host__ __device__ constexpr int64_t sh_bits_words(int64_t count) { return (count + kShPad + 3) / 4 * 4; }
__host__ __device__ constexpr int64_t sh_ids_halves(int64_t count) { return (count + kShPad + 7) / 8 * 8; }

// The 8-bit counts are flushed into 16-bit counters in registers every
// kShFlush members.  Requests must not repeat an id (a member's mask holds one
// bit per request), the pool must hold at most 65536 rasters, and n <= 65535
// per request keeps the 16-bit counters from overflowing.
template <bool NT, int TPB, int PX>
__global__ __launch_bounds__(TPB) void k_shared(const uint8_t *__restrict__ base, int64_t stride,
                                                int32_t W, int32_t H, int32_t count, int32_t S,
                                                const char *__restrict__ arena,
                                                uint32_t *__restrict__ queue) {
  static_assert(TPB * PX == kShTile, "a tile is kShTile pixels");
  typedef ShPx<PX> P;
  typedef typename P::Acc Acc;
  constexpr int NW = PX / 4;  // dwords per thread
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Acc *acc8 = reinterpret_cast<Acc *>(lds_raw);
  uint32_t *bits = reinterpret_cast<uint32_t *>(acc8 + (size_t)S * TPB);
  uint16_t *ids = reinterpret_cast<uint16_t *>(bits + sh_bits_words(count));
  __shared__ int s_item, s_ns, s_rnext, s_nlist;
  __shared__ int s_slot[kShMaxSlots];
  __shared__ int s_off[kShMaxSlots + 1];  // prefix sums of the slots' id counts

  const Header *hd = reinterpret_cast<const Header *>(arena);
  const int nreq = hd->nreq;
  const ReqDesc *reqs = reinterpret_cast<const ReqDesc *>(arena + hd->reqs_off);
  const int32_t *ids_all = reinterpret_cast<const int32_t *>(arena + hd->ids_off);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int segs = (W + kShTile - 1) / kShTile;
  const int ntiles = H * segs;

  for (;;) {
    if (tid == 0) s_item = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int tile = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (tile >= ntiles) break;  // the queue counter only grows: every wave exits
    const int y = tile / segs;
    const int xt = (tile - y * segs) * kShTile;
    const int tw = min(kShTile, W - xt);
    const int x = xt + PX * tid;
    const bool live = x < W;
    // lanes past the row end read the row start instead; their counts are
    // never written out
    const uint8_t *px = base + (uint32_t)y * (uint32_t)W + (live ? (uint32_t)x : 0u);
    int r_next = 0;
    while (r_next < nreq) {
      // the next (up to S) requests whose windows cover this tile
      if (wave == 0) {
        int ns = 0, r = r_next;
        while (r < nreq) {
          bool cov = false;
          if (r + lane < nreq) {
            const ReqDesc &R = reqs[r + lane];
            cov = y >= R.y0 && y < R.y0 + R.h && R.x0 < xt + tw && R.x0 + R.w > xt;
          }
          unsigned long long m = __ballot(cov);
          while (m != 0 && ns < S) {
            const int l = __builtin_ctzll(m);
            m &= m - 1;
            if (lane == 0) s_slot[ns] = r + l;
            ++ns;
          }
          if (m != 0) {  // slots full with covering requests left in this chunk
            r += __builtin_ctzll(m);
            break;
          }
          r += 64;
          if (ns == S) break;
        }
        if (lane == 0) {
          s_ns = ns;
          s_rnext = min(r, nreq);
          int o = 0;
          for (int j = 0; j < ns; ++j) {
            s_off[j] = o;
            o += reqs[s_slot[j]].n;
          }
          s_off[ns] = o;
        }
      }
      __syncthreads();
      const int ns = s_ns;
      r_next = s_rnext;
      if (ns == 0) break;
      for (int m = tid; m < count; m += TPB) bits[m] = 0u;
      for (int j = 0; j < ns; ++j) acc8[j * TPB + tid] = 0;
      __syncthreads();
      // mark the members of each slot's request: the (slot, id) pairs are
      // spread over the threads, four loads in flight per thread
      {
        const int total = s_off[ns];
        int j = 0;
        for (int p0 = tid; p0 < total; p0 += 4 * TPB) {
          int id[4], sj[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int p = p0 + u * TPB;
            while (j + 1 < ns && s_off[j + 1] <= p) ++j;
            sj[u] = j;
            id[u] = p < total ? ids_all[reqs[s_slot[j]].ids_off + (p - s_off[j])] : -1;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (id[u] >= 0) atomicOr(&bits[id[u]], 1u << sj[u]);
        }
      }
      __syncthreads();
      // compact the marked members in id order (wave 0): their ids, and their
      // masks moved down in place (an entry moves to a position no later than
      // its own, after the wave has read it); then the zero padding
      if (wave == 0) {
        int nl = 0;
        for (int c0 = 0; c0 < count; c0 += 64) {
          const uint32_t v = c0 + lane < count ? bits[c0 + lane] : 0u;
          const unsigned long long m = __ballot(v != 0u);
          const int before = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          if (v) {
            ids[nl + before] = (uint16_t)(c0 + lane);
            bits[nl + before] = v;
          }
          nl += __builtin_popcountll(m);
        }
        if (lane < kShPad) {
          ids[nl + lane] = 0;
          bits[nl + lane] = 0u;
        }
        if (lane == 0) s_nlist = nl;
      }
      __syncthreads();
      const int nl = s_nlist;
      // Stream the listed members' tiles: groups of kShUnroll (id, mask)
      // pairs read from LDS at once; the next group's loads are in flight
      // while this one is added.  Padding entries have id 0 and an empty mask.
      typedef decltype(P::template load<NT>(px)) Word;
      Word wa[kShUnroll], wb[kShUnroll];
      uint32_t ba[kShUnroll], bb[kShUnroll];
      auto fetch = [&](int i, Word(&w)[kShUnroll], uint32_t(&b)[kShUnroll]) {
        const uint4 q = *reinterpret_cast<const uint4 *>(ids + i);
        const uint4 m0 = *reinterpret_cast<const uint4 *>(bits + i);
        const uint4 m1 = *reinterpret_cast<const uint4 *>(bits + i + 4);
        const uint32_t qw[4] = {q.x, q.y, q.z, q.w};
        b[0] = m0.x; b[1] = m0.y; b[2] = m0.z; b[3] = m0.w;
        b[4] = m1.x; b[5] = m1.y; b[6] = m1.z; b[7] = m1.w;
#pragma unroll
        for (int u = 0; u < kShUnroll; ++u) {
          const uint32_t id = (qw[u >> 1] >> (16 * (u & 1))) & 0xffffu;
          w[u] = P::template load<NT>(px + (int64_t)id * stride);
        }
      };
      auto add = [&](const Word(&w)[kShUnroll], const uint32_t(&b)[kShUnroll]) {
#pragma unroll
        for (int u = 0; u < kShUnroll; ++u) {
          const Acc nz = P::flags(w[u]);
          uint32_t m = __builtin_amdgcn_readfirstlane(b[u]);
          while (m) {
            const int j = __builtin_ctz(m);
            m &= m - 1;
            atomicAdd(&acc8[j * TPB + tid], nz);
          }
        }
      };
      // 16-bit counters: per dword of pixels, lanes of pixels 0,2 and 1,3
      uint32_t c02[kShMaxSlots][NW], c13[kShMaxSlots][NW];
#pragma unroll
      for (int j = 0; j < kShMaxSlots; ++j)
#pragma unroll
        for (int k = 0; k < NW; ++k) c02[j][k] = c13[j][k] = 0u;
      // widen this thread's 8-bit counts (only this thread touches its
      // accumulator words: no barrier)
      auto flush = [&]() {
#pragma unroll
        for (int j = 0; j < kShMaxSlots; ++j) {
          if (j < ns) {
            const Acc v = acc8[j * TPB + tid];
            acc8[j * TPB + tid] = 0;
#pragma unroll
            for (int k = 0; k < NW; ++k) {
              const uint32_t d = (uint32_t)((unsigned long long)v >> (32 * k));
              c02[j][k] = cmp::padd(c02[j][k], cmp::lanes_lo(d));
              c13[j][k] = cmp::padd(c13[j][k], cmp::lanes_hi(d));
            }
          }
        }
      };
      fetch(0, wa, ba);
      for (int i = 0, next_flush = kShFlush; i < nl; i += 2 * kShUnroll) {
        fetch(i + kShUnroll, wb, bb);
        add(wa, ba);
        fetch(i + 2 * kShUnroll, wa, ba);
        add(wb, bb);
        if (i + 2 * kShUnroll >= next_flush) {
          flush();
          next_flush += kShFlush;
        }
      }
      flush();
      // the covering requests' pixels of this tile
#pragma unroll
      for (int j = 0; j < kShMaxSlots; ++j) {
        if (j >= ns) continue;
        const ReqDesc &R = reqs[s_slot[j]];
        if (y < R.y0 || y >= R.y0 + R.h) continue;
        const int64_t row = (int64_t)(y - R.y0) * R.pitch - R.x0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
          const uint32_t c[4] = {c02[j][k] & 0xffffu, c13[j][k] & 0xffffu, c02[j][k] >> 16,
                                 c13[j][k] >> 16};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int xk = x + 4 * k + q;
            if (xk < W && xk >= R.x0 && xk < R.x0 + R.w) as_global(R.out)[row + xk] = c[q];
          }
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- matrix mode
//
// The counts of a batch are a product of 0/1 matrices: over the pixels p of a
// tile, the pool members k and the requests r,
//   count[p][r] = sum_k F[p][k] * M[k][r],
// F[p][k] = [raster k is nonzero at p], M[k][r] = [k is one of r's ids].  A
// workgroup owns 128 pixels of one raster row per wave, and blocks of 64
// requests at a time: the counts of a wave's pixels for all 64 requests are
// 128 x 64 int32 accumulators of int8 matrix-core products (8 x 4 blocks of
// 16 x 16, in registers), so every (member, tile) is read once however many
// of the tile's covering requests hold it.  Members of the pool are taken in
// chunks of 32 consecutive ids; a chunk is streamed when one of the tile's
// covering requests holds one of its members, and only those members are
// read (the others load one shared cache line whose bytes meet zeros in M).
//
// Operands of one 16x16x32 int8 product, per lane l (row or column l % 16,
// k-group l / 16 of 8 consecutive k):
//   A: 8 bytes, the flags of members 8*(l/16) .. +7 of the chunk at one
//      pixel (0x80 for nonzero, i.e. -128, else 0);
//   B: 8 bytes, 1 where that member belongs to request l % 16 of the group;
//   D: 4 int32, rows 4*(l/16) .. +3, column l % 16;
// so D = -128 * count.  The flags come from 8-byte loads of 8 pixels of 8
// members, transposed in registers (an 8 x 8 byte transpose by byte permutes).
// M lives in LDS as one byte per (chunk, k-group, request): bit i = member
// 32*chunk + 8*kgroup + i, laid out [chunk][kgroup][request % 16][request / 16].
// The product's 64 columns are the tile's covering requests packed in order,
// and only the groups of 16 columns that hold one are multiplied.

constexpr int kMxReqs = 64;        // requests per block (4 groups of 16 columns)
constexpr int kMxMaxCount = 8192;  // pool rasters (M of a block: 256 B per chunk of 32)

__host__ __device__ constexpr int64_t mx_chunks(int64_t count) { return (count + 31) / 32; }
// LDS of k_matrix: M of one request block, the union byte of each (chunk,
// k-group), the list of chunks to stream.
__host__ __device__ constexpr int64_t mx_lds_bytes(int64_t count) {
  return mx_chunks(count) * (256 + 4) + (mx_chunks(count) * 2 + 15) / 16 * 16;
}

typedef int mx_i32x4 __attribute__((ext_vector_type(4)));

// 0x80 in every byte of w that is nonzero, 0 elsewhere (see nonzero_bytes).
__device__ __forceinline__ uint32_t nonzero_sign(uint32_t w) {
  return (((w & 0x7f7f7f7fu) + 0x7f7f7f7fu) | w) & 0x80808080u;
}

// 4x4 byte transpose: u[c] = (w0[c], w1[c], w2[c], w3[c]).
__device__ __forceinline__ void transpose4(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                           uint32_t &u0, uint32_t &u1, uint32_t &u2, uint32_t &u3) {
  const uint32_t a = __builtin_amdgcn_perm(w1, w0, 0x05010400u);  // w0[0] w1[0] w0[1] w1[1]
  const uint32_t b = __builtin_amdgcn_perm(w1, w0, 0x07030602u);  // w0[2] w1[2] w0[3] w1[3]
  const uint32_t c = __builtin_amdgcn_perm(w3, w2, 0x05010400u);
  const uint32_t d = __builtin_amdgcn_perm(w3, w2, 0x07030602u);
  u0 = __builtin_amdgcn_perm(c, a, 0x05040100u);
  u1 = __builtin_amdgcn_perm(c, a, 0x07060302u);
  u2 = __builtin_amdgcn_perm(d, b, 0x05040100u);
  u3 = __builtin_amdgcn_perm(d, b, 0x07060302u);
}

// The 8 bits of x as 8 bytes of 0 or 1 (bit i -> byte i): multiplying a
// nibble by 2^0 + 2^7 + 2^14 + 2^21 puts bit i at 8i with no two partial
// products meeting.
__device__ __forceinline__ long spread_bits(uint32_t x) {
  const uint32_t lo = ((x & 0xfu) * 0x204081u) & 0x01010101u;
  const uint32_t hi = (((x >> 4) & 0xfu) * 0x204081u) & 0x01010101u;
  return (long)(((unsigned long)hi << 32) | lo);
}

// Requests must not repeat an id (M is a set), the pool must hold at most
// kMxMaxCount rasters, and 31 * stride + W + 8 < 2^32 (per-lane 32-bit
// offsets from a chunk's first raster).
template <bool NT, int WAVES>
__global__ __launch_bounds__(WAVES * 64, 8 / WAVES) void k_matrix(const uint8_t *__restrict__ base,
                                                          int64_t stride, int32_t W, int32_t H,
                                                          int32_t count,
                                                          const char *__restrict__ arena,
                                                          uint32_t *__restrict__ queue) {
  constexpr int TPB = WAVES * 64, T = WAVES * 128;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int nc = (int)mx_chunks(count);
  uint32_t *memb = reinterpret_cast<uint32_t *>(lds_raw);  // [nc][4][16] dwords
  uint32_t *ub = memb + nc * 64;                            // [nc]: union byte per k-group
  uint16_t *list = reinterpret_cast<uint16_t *>(ub + nc);   // chunks to stream
  __shared__ int s_item, s_nl;
  __shared__ unsigned long long s_cov;
  __shared__ uint32_t s_cmask[16];
  __shared__ int8_t s_slot[kMxReqs];  // covering requests in order (block-local index)

  const Header *hd = reinterpret_cast<const Header *>(arena);
  const int nreq = hd->nreq;
  const ReqDesc *reqs = reinterpret_cast<const ReqDesc *>(arena + hd->reqs_off);
  const uint4 *bits_all = reinterpret_cast<const uint4 *>(arena + hd->bits_off);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row16 = lane & 15, kg = lane >> 4;
  const int segs = (W + T - 1) / T;
  const int ntiles = H * segs;
  const int nitems = ((nreq + kMxReqs - 1) / kMxReqs) * ntiles;
  int cur = -1;

  for (;;) {
    if (tid == 0) s_item = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= nitems) break;  // the queue counter only grows: every wave exits
    const int rb = item / ntiles, tile = item - rb * ntiles;
    if (rb != cur) {  // M of this request block into LDS
      const uint4 *src = bits_all + (int64_t)rb * nc * 16;
      uint4 *dst = reinterpret_cast<uint4 *>(memb);
      for (int q = tid; q < nc * 16; q += TPB) dst[q] = src[q];
      cur = rb;
    }
    const int y = tile / segs;
    const int xt = (tile - y * segs) * T;
    const int tw = min(T, W - xt);
    if (wave == 0) {  // the block's requests whose windows cover the tile
      const int r = rb * kMxReqs + lane;
      bool c = false;
      if (r < nreq) {
        const ReqDesc &R = reqs[r];
        c = y >= R.y0 && y < R.y0 + R.h && R.x0 < xt + tw && R.x0 + R.w > xt;
      }
      const unsigned long long cov = __ballot(c);
      if (lane < 16) {  // byte g of s_cmask[n]: request 16g + n covers
        uint32_t mk = 0;
#pragma unroll
        for (int g = 0; g < 4; ++g)
          if ((cov >> (16 * g + lane)) & 1ull) mk |= 0xffu << (8 * g);
        s_cmask[lane] = mk;
      }
      // product columns: the covering requests packed in order, so that only
      // ceil(covering / 16) groups of 16 columns are multiplied
      if (c)
        s_slot[__builtin_amdgcn_mbcnt_hi((uint32_t)(cov >> 32),
                                         __builtin_amdgcn_mbcnt_lo((uint32_t)cov, 0u))] = (int8_t)lane;
      if (lane == 0) s_cov = cov;
    }
    __syncthreads();
    const unsigned long long cov = s_cov;
    if (cov == 0ull) continue;
    // members any covering request holds, per (chunk, k-group) byte
    for (int q = tid; q < nc * 4; q += TPB) {
      const uint4 *e = reinterpret_cast<const uint4 *>(memb) + q * 4;
      uint32_t u = 0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const uint4 d = e[v];
        u |= (d.x & s_cmask[4 * v]) | (d.y & s_cmask[4 * v + 1]) | (d.z & s_cmask[4 * v + 2]) |
             (d.w & s_cmask[4 * v + 3]);
      }
      u |= u >> 16;
      u |= u >> 8;
      reinterpret_cast<uint8_t *>(ub)[q] = (uint8_t)u;
    }
    __syncthreads();
    if (wave == 0) {  // chunks with a member to stream, in id order
      int nl = 0;
      for (int c0 = 0; c0 < nc; c0 += 64) {
        const uint32_t v = c0 + lane < nc ? ub[c0 + lane] : 0u;
        const unsigned long long mm = __ballot(v != 0u);
        const int before = __builtin_amdgcn_mbcnt_hi((uint32_t)(mm >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mm, 0u));
        if (v) list[nl + before] = (uint16_t)(c0 + lane);
        nl += __builtin_popcountll(mm);
      }
      if (lane == 0) s_nl = nl;
    }
    __syncthreads();
    const int nl = s_nl;
    const int xw = xt + 128 * wave;
    if (xw >= W) continue;  // wave-uniform; no barrier until the next item
    // A role: pixels xw + 8*row16 .. +7 of members 8*kg .. +7 of each chunk.
    // Lanes past the row end read the row's last byte onwards instead (at
    // most 7 bytes past the row; the pool has 16 bytes of slack).
    const uint32_t loff = xw + 8 * row16 < W ? 8u * row16 : (uint32_t)(W - 1 - xw);
    // byte offsets from the chunk's first raster (32-bit: 31 * stride + W + 8 < 2^32)
    uint32_t off[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) off[i] = (uint32_t)(8 * kg + i) * (uint32_t)stride + loff;
    const uint8_t *rowb = base + (uint32_t)y * (uint32_t)W + xw;  // wave-uniform
    const uint8_t *ub8 = reinterpret_cast<const uint8_t *>(ub);
    const uint8_t *memb8 = reinterpret_cast<const uint8_t *>(memb);
    // B and D roles: column row16 of group g is slot 16g + row16; its
    // request's byte in a (chunk, k-group) row of M is 4 * (r % 16) + r / 16
    const int ncov = __builtin_popcountll(cov);
    const int ng = (ncov + 15) >> 4;
    int rq[4], boff[4];
    uint32_t vmask[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int sl = 16 * g + row16;
      rq[g] = sl < ncov ? (int)s_slot[sl] : -1;
      boff[g] = rq[g] < 0 ? 0 : 4 * (rq[g] & 15) + (rq[g] >> 4);
      vmask[g] = rq[g] < 0 ? 0u : 0xffu;
    }

    mx_i32x4 acc[8][4];
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int g = 0; g < 4; ++g) acc[j][g] = mx_i32x4{0, 0, 0, 0};

    // member loads of list entry li (past the end: one cached line, unused)
    auto fetch = [&](int li, uint32_t (&d)[16], int &chunk) {
      const bool in = li < nl;  // branch-free, so the loads stay ahead of the math
      const int cl = __builtin_amdgcn_readfirstlane((int)list[min(li, nc - 1)]);
      const int c = in ? cl : 0;
      const uint32_t uu = ub8[4 * c + kg];
      const uint32_t u = in ? uu : 0u;
      const uint8_t *cb = rowb + (int64_t)c * 32 * stride;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint32_t o = (u >> i) & 1u ? off[i] : loff;
        u32x2u v;
        if constexpr (NT) v = __builtin_nontemporal_load((gu32x2u *)(cb + o));
        else v = *(gu32x2u *)(cb + o);
        d[2 * i] = v.x;
        d[2 * i + 1] = v.y;
      }
      chunk = in ? c : -1;
    };
    auto mma = [&](const uint32_t (&d)[16], int c) {
      // B role: the four slots' bytes of M, read first so that the
      // conversion below hides their latency
      const uint8_t *mrow = memb8 + max(c, 0) * 256 + kg * 64;
      uint32_t xb[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) xb[g] = mrow[boff[g]];
      uint32_t f[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) f[k] = nonzero_sign(d[k]);
      // f[2i + h]: member i, pixels 4h .. 4h+3 -> a[j]: pixel j, members 0..7
      uint32_t lo[8], hi[8];
      transpose4(f[0], f[2], f[4], f[6], lo[0], lo[1], lo[2], lo[3]);
      transpose4(f[8], f[10], f[12], f[14], hi[0], hi[1], hi[2], hi[3]);
      transpose4(f[1], f[3], f[5], f[7], lo[4], lo[5], lo[6], lo[7]);
      transpose4(f[9], f[11], f[13], f[15], hi[4], hi[5], hi[6], hi[7]);
      long a[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) a[j] = (long)(((unsigned long)hi[j] << 32) | lo[j]);
      // zero for an empty slot and past the list's end, so those products
      // add nothing; one register pair per group, so the products of all
      // groups in use issue back to back
      const uint32_t live = c >= 0 ? 0xffu : 0u;  // wave-uniform
      long b[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        b[g] = spread_bits(xb[g] & live & vmask[g]);
        asm volatile("" ::"v"(b[g]));  // built here, not sunk into the branches below
      }
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        if (g < ng) {
#pragma unroll
          for (int j = 0; j < 8; ++j)
            acc[j][g] = __builtin_amdgcn_mfma_i32_16x16x32_i8(a[j], b[g], acc[j][g], 0, 0, 0);
        }
      }
    };
    uint32_t da[16], db[16], dc[16];
    int ca = 0, cb2 = 0, cc = 0;
    // Three chunk buffers, two chunks' loads in flight while one is
    // converted and multiplied; the scheduling barriers keep each chunk's
    // loads issued ahead of the math.  The previous tile's output stores are
    // retired first: with stores and loads both outstanding, every wait below
    // would have to be a full one.
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
    fetch(0, da, ca);
    fetch(1, db, cb2);
    int li = 0;
    for (; li + 2 < nl; li += 3) {
      fetch(li + 2, dc, cc);
      __builtin_amdgcn_sched_barrier(0);
      mma(da, ca);
      __builtin_amdgcn_sched_barrier(0);
      fetch(li + 3, da, ca);
      __builtin_amdgcn_sched_barrier(0);
      mma(db, cb2);
      __builtin_amdgcn_sched_barrier(0);
      fetch(li + 4, db, cb2);
      __builtin_amdgcn_sched_barrier(0);
      mma(dc, cc);
      __builtin_amdgcn_sched_barrier(0);
    }
    // the last one or two chunks (products of entries past the end use a
    // zero B and add nothing)
    if (li < nl) {
      mma(da, ca);
      mma(db, cb2);
    }
    // D role: lane (row16 = request column n, kg = row group): pixels
    // xw + 32*kg + 8i + j in register i of block j
    const int p0 = xw + 32 * kg;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      if (rq[g] < 0) continue;
      const ReqDesc &R = reqs[rb * kMxReqs + rq[g]];
      gu32_t *o = as_global(R.out) + (int64_t)(y - R.y0) * R.pitch - R.x0;
      if (p0 >= R.x0 && p0 + 32 <= R.x0 + R.w) {
        // the whole run inside the window: eight 16-byte stores
#pragma unroll
        for (int q = 0; q < 32; q += 4) {
          u32x4a4 v;
          v.x = (uint32_t)(-acc[(q + 0) & 7][g][(q + 0) >> 3]) >> 7;
          v.y = (uint32_t)(-acc[(q + 1) & 7][g][(q + 1) >> 3]) >> 7;
          v.z = (uint32_t)(-acc[(q + 2) & 7][g][(q + 2) >> 3]) >> 7;
          v.w = (uint32_t)(-acc[(q + 3) & 7][g][(q + 3) >> 3]) >> 7;
          *(__attribute__((address_space(1))) u32x4a4 *)(o + p0 + q) = v;
        }
      } else {
        const int lo_x = max(p0, R.x0), hi_x = min(p0 + 32, R.x0 + R.w);
#pragma unroll
        for (int q = 0; q < 32; ++q) {
          const int p = p0 + q;
          if (p >= lo_x && p < hi_x) o[p] = (uint32_t)(-acc[q & 7][g][q >> 3]) >> 7;
        }
      }
    }
  }
}

template <bool NT>
__global__ __launch_bounds__(256) void k_crop(const uint8_t *__restrict__ base, int64_t stride,
                                              int32_t W, ReqDesc R,
                                              const int32_t *__restrict__ ids) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= R.h * R.nvr) return;
  const int row = v / R.nvr, j = v - row * R.nvr;
  const uint32_t off = (uint32_t)(R.y0 + row) * (uint32_t)W + (uint32_t)(R.x0 + 16 * j);
  crop_vector<NT>(base, stride, ids, R.n, off, as_global(R.out) + (int64_t)row * R.pitch + 16 * j,
              min(16, R.w - 16 * j));
}

int64_t align64(int64_t x) { return (x + 63) / 64 * 64; }

}  // namespace



namespace {

void drop_graphs(cmp_pool *p) {
  for (auto &kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  p->graphs.clear();
}

#define POOL_TRY(call)          \
  do {                          \
    if ((call) != hipSuccess) { \
      p->poisoned = true;       \
      return CMP_EDEVICE;       \
    }                           \
  } while (0)

int ensure_arena(cmp_pool *p, int64_t bytes) {
  if (bytes <= p->arena_cap) return CMP_OK;
  if (hipStreamSynchronize(p->s) != hipSuccess) return CMP_EDEVICE;
  drop_graphs(p);
  (void)hipFree(p->d_arena);
  if (p->h_arena) (void)hipHostFree(p->h_arena);
  p->d_arena = nullptr;
  p->h_arena = nullptr;
  p->arena_cap = 0;
  const int64_t cap = std::max<int64_t>(bytes, 1 << 20);
  if (hipMalloc((void **)&p->d_arena, cap) != hipSuccess) return CMP_ENOMEM;
  if (hipHostMalloc((void **)&p->h_arena, cap, hipHostMallocDefault) != hipSuccess) return CMP_ENOMEM;
  p->arena_cap = cap;
  return CMP_OK;
}

// Threads per workgroup and pixels per thread of k_shared (a tile is 1024).
constexpr int kShTpb = 128, kShPx = 8;

// LDS bytes of k_shared with S slots over a pool of `count` rasters.
int64_t shared_lds_bytes(int64_t count, int S) {
  return (int64_t)S * kShTpb * kShPx + sh_bits_words(count) * 4 + sh_ids_halves(count) * 2;
}

// Slots per pass the shared mode can use on this pool (0: not usable).
int shared_slots(const cmp_pool *p) {
  if (p->count > 65536) return 0;
  const int64_t room = (int64_t)p->max_lds - p->static_lds_shared - shared_lds_bytes(p->count, 0);
  const int64_t S = std::min<int64_t>(kShMaxSlots, room / (kShTpb * kShPx));
  return S >= 4 ? (int)S : 0;
}

hipError_t launch_shared(cmp_pool *p, int grid, bool nt, int S) {
  hipError_t e = cmp::launch_fill(p->d_queue, 0, 4, p->s);
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)shared_lds_bytes(p->count, S);
  if (nt)
    k_shared<true, kShTpb, kShPx><<<grid, kShTpb, lds, p->s>>>(
        p->base, p->stride, p->W, p->H, (int32_t)p->count, S, p->d_arena, p->d_queue);
  else
    k_shared<false, kShTpb, kShPx><<<grid, kShTpb, lds, p->s>>>(
        p->base, p->stride, p->W, p->H, (int32_t)p->count, S, p->d_arena, p->d_queue);
  return hipGetLastError();
}

// Waves per workgroup of k_matrix (a tile is 128 pixels per wave).
constexpr int kMxWaves = 4;

// Whether k_matrix can run on this pool (request sets are checked per batch).
bool matrix_pool_ok(const cmp_pool *p) {
  return p->count <= kMxMaxCount && 31 * p->stride + p->W + 8 < (int64_t(1) << 32) &&
         p->max_lds_matrix >= mx_lds_bytes(p->count);
}

hipError_t launch_matrix(cmp_pool *p, int grid, bool nt) {
  hipError_t e = cmp::launch_fill(p->d_queue, 0, 4, p->s);
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)mx_lds_bytes(p->count);
  if (nt)
    k_matrix<true, kMxWaves><<<grid, kMxWaves * 64, lds, p->s>>>(
        p->base, p->stride, p->W, p->H, (int32_t)p->count, p->d_arena, p->d_queue);
  else
    k_matrix<false, kMxWaves><<<grid, kMxWaves * 64, lds, p->s>>>(
        p->base, p->stride, p->W, p->H, (int32_t)p->count, p->d_arena, p->d_queue);
  return hipGetLastError();
}

hipError_t launch_persistent(cmp_pool *p, int grid, bool nt) {
  hipError_t e = cmp::launch_fill(p->d_queue, 0, 4, p->s);
  if (e != hipSuccess) return e;
  if (nt)
    k_batch<true><<<grid, 256, 0, p->s>>>(p->base, p->stride, p->W, p->d_arena, p->d_queue);
  else
    k_batch<false><<<grid, 256, 0, p->s>>>(p->base, p->stride, p->W, p->d_arena, p->d_queue);
  return hipGetLastError();
}

}  // namespace

extern "C" {

void composite_default_tune(cmp_tune *t) {
  if (!t) return;
  std::memset(t, 0, sizeof(*t));
  // measured on 64 requests over a pool of 2048 masks of 2048x2048: matrix
  // mode with non-temporal loads (1.73 ms; two workgroups per compute unit
  // run at once); the shared fallback is best there with the same load hint,
  // 24 requests per pass and 4 workgroups per compute unit (2.74 ms).  The
  // persistent fallback (repeated ids) prefers cached loads and 256-vector
  // items, 2 per compute unit (4.86 ms against 6.26 ms with these values);
  // the autotuner finds that
  t->mode = CMP_BATCH_MATRIX;
  t->tile_vecs = 1024;
  t->blocks_per_cu = 4;
  t->use_graph = 1;
  t->order = CMP_ORDER_ROWS;
  t->stream_loads = 1;
  t->slots = 24;
}

// The larger static LDS of two instances of a kernel, in bytes.
static hipError_t static_lds(const void *f1, const void *f2, int *bytes) {
  hipFuncAttributes a{}, b{};
  hipError_t e = hipFuncGetAttributes(&a, f1);
  if (e == hipSuccess) e = hipFuncGetAttributes(&b, f2);
  if (e == hipSuccess) *bytes = (int)std::max(a.sharedSizeBytes, b.sharedSizeBytes);
  return e;
}

int composite_pool_create(cmp_pool **out, const uint8_t *dev_base, int64_t count, int32_t W,
                          int32_t H, int64_t stride_bytes, int64_t pool_bytes, int32_t device) {
  if (!out) return CMP_EINVAL;
  *out = nullptr;
  if (!dev_base || count < 1 || W < 1 || H < 1) return CMP_EINVAL;
  const int64_t plane = (int64_t)W * H;
  if (plane > (int64_t(1) << 32) - 16 || stride_bytes < plane) return CMP_EINVAL;
  if ((count - 1) > (INT64_MAX - plane - 16) / stride_bytes) return CMP_EINVAL;
  if ((count - 1) * stride_bytes + plane + 16 > pool_bytes) return CMP_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return CMP_EDEVICE;
  if (device < 0 || device >= ndev) return CMP_EINVAL;
  cmp_pool *p = new (std::nothrow) cmp_pool();
  if (!p) return CMP_ENOMEM;
  p->dev = device;
  p->base = dev_base;
  p->count = count;
  p->W = W;
  p->H = H;
  p->stride = stride_bytes;
  p->bytes = pool_bytes;
  int rc = CMP_EDEVICE;
  do {
    if (hipSetDevice(device) != hipSuccess) break;
    if (hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
      break;
    if (hipDeviceGetAttribute(&p->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess)
      break;
    // the dynamic LDS a mode may ask for is what a workgroup may use less the
    // kernels' static LDS, as the compiler laid it out
    int st_mx = 0, st_sh = 0;
    if (static_lds((const void *)k_matrix<true, kMxWaves>, (const void *)k_matrix<false, kMxWaves>,
                   &st_mx) != hipSuccess ||
        static_lds((const void *)k_shared<true, kShTpb, kShPx>,
                   (const void *)k_shared<false, kShTpb, kShPx>, &st_sh) != hipSuccess)
      break;
    p->max_lds_matrix = p->max_lds - st_mx;
    p->static_lds_shared = st_sh;
    if (const int S = shared_slots(p)) {
      // allow k_shared its dynamic LDS (beyond the default per-launch limit)
      const int lds = (int)shared_lds_bytes(p->count, S);
      if (hipFuncSetAttribute((const void *)k_shared<true, kShTpb, kShPx>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess ||
          hipFuncSetAttribute((const void *)k_shared<false, kShTpb, kShPx>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
        p->max_lds = 0;  // shared mode unavailable; batches fall back to persistent
    }
    if (p->count <= kMxMaxCount) {
      const int lds = (int)mx_lds_bytes(p->count);
      if (lds <= p->max_lds_matrix &&
          (hipFuncSetAttribute((const void *)k_matrix<true, kMxWaves>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess ||
           hipFuncSetAttribute((const void *)k_matrix<false, kMxWaves>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess))
        p->max_lds_matrix = 0;  // matrix mode unavailable
    }
    if (hipStreamCreateWithFlags(&p->s, hipStreamNonBlocking) != hipSuccess) break;
    if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess) break;
    rc = CMP_ENOMEM;
    if (hipMalloc((void **)&p->d_queue, 64) != hipSuccess) break;
    rc = CMP_OK;
  } while (false);
  if (rc != CMP_OK) {
    composite_pool_free(p);
    return rc;
  }
  *out = p;
  return CMP_OK;
}

void composite_pool_free(cmp_pool *p) {
  if (!p) return;
  (void)hipSetDevice(p->dev);
  if (p->s) (void)hipStreamSynchronize(p->s);
  drop_graphs(p);
  (void)hipFree(p->d_arena);
  if (p->h_arena) (void)hipHostFree(p->h_arena);
  (void)hipFree(p->d_queue);
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
  if (p->s) (void)hipStreamDestroy(p->s);
  delete p;
}

int composite_batch_run(cmp_pool *p, const cmp_request *reqs, int32_t nreq, const cmp_tune *tune) {
  if (!p) return CMP_EINVAL;
  if (p->poisoned) return CMP_EDEVICE;
  if (nreq < 0 || (nreq > 0 && !reqs)) return CMP_EINVAL;
  cmp_tune t;
  composite_default_tune(&t);
  if (tune) t = *tune;
  if (t.mode != CMP_BATCH_PERSISTENT && t.mode != CMP_BATCH_PER_REQUEST && t.mode != CMP_BATCH_SHARED &&
      t.mode != CMP_BATCH_MATRIX)
    return CMP_EINVAL;
  if (t.mode != CMP_BATCH_PER_REQUEST &&
      (t.tile_vecs < 64 || t.tile_vecs > 65536 || t.blocks_per_cu < 1 || t.blocks_per_cu > 16 ||
       (t.use_graph != 0 && t.use_graph != 1) ||
       (t.order != CMP_ORDER_COST && t.order != CMP_ORDER_ROWS)))
    return CMP_EINVAL;
  if (t.stream_loads != 0 && t.stream_loads != 1) return CMP_EINVAL;
  if (t.slots != 0 && (t.slots < 4 || t.slots > kShMaxSlots)) return CMP_EINVAL;
  for (int r : t.reserved)
    if (r) return CMP_EINVAL;
  // validate every request before anything is enqueued
  int64_t total_ids = 0;
  for (int32_t r = 0; r < nreq; ++r) {
    const cmp_request &q = reqs[r];
    if (q.n < 0 || q.n > 65535 || (q.n > 0 && !q.ids)) return CMP_EINVAL;
    if (q.w < 1 || q.h < 1 || q.x0 < 0 || q.y0 < 0 || (int64_t)q.x0 + q.w > p->W ||
        (int64_t)q.y0 + q.h > p->H)
      return CMP_EINVAL;
    if (!q.dev_count || q.out_pitch < q.w) return CMP_EINVAL;
    for (int32_t i = 0; i < q.n; ++i)
      if (q.ids[i] < 0 || q.ids[i] >= p->count) return CMP_EINVAL;
    total_ids += q.n;
  }
  if (nreq == 0) {
    p->last_ms = 0.0;
    p->last_items = 0;
    p->last_mode = t.mode;
    return CMP_OK;
  }
  // the shared and matrix modes need distinct ids per request (sets); the
  // matrix mode also a pool it can address, and falls back to the shared
  // mode; the shared mode needs room in LDS and falls back to the persistent
  // mode with the same parameters
  bool sets = false;
  if (t.mode == CMP_BATCH_SHARED || t.mode == CMP_BATCH_MATRIX) {
    // repeated ids: one bit per pool raster, set and cleared per request
    sets = true;
    std::vector<uint64_t> seen((size_t)(p->count + 63) / 64, 0);
    for (int32_t r = 0; r < nreq && sets; ++r) {
      const cmp_request &q = reqs[r];
      int32_t i = 0;
      for (; i < q.n; ++i) {
        uint64_t &w = seen[q.ids[i] >> 6];
        const uint64_t b = uint64_t(1) << (q.ids[i] & 63);
        if (w & b) break;
        w |= b;
      }
      if (i < q.n) sets = false;
      for (int32_t k = 0; k < i; ++k) seen[q.ids[k] >> 6] = 0;
    }
  }
  const int64_t mx_segs = (p->W + kMxWaves * 128 - 1) / (kMxWaves * 128);
  const int64_t mx_blocks = (nreq + kMxReqs - 1) / kMxReqs;
  const int64_t mx_items = mx_blocks * p->H * mx_segs;
  if (t.mode == CMP_BATCH_MATRIX &&
      !(sets && matrix_pool_ok(p) && mx_items + (int64_t)p->cus * 2 < INT32_MAX))
    t.mode = CMP_BATCH_SHARED;
  int S = 0;
  if (t.mode == CMP_BATCH_SHARED) {
    S = sets ? shared_slots(p) : 0;
    if (S && t.slots) S = std::min(S, t.slots);
    if (!S) t.mode = CMP_BATCH_PERSISTENT;
  }
  // work items: bands of whole rows of about tile_vecs vectors
  std::vector<ReqDesc> rd(nreq);
  std::vector<Item> items;
  std::vector<double> cost;
  int64_t ids_off = 0;
  for (int32_t r = 0; r < nreq; ++r) {
    const cmp_request &q = reqs[r];
    ReqDesc &d = rd[r];
    d.out = q.dev_count;
    d.pitch = q.out_pitch;
    d.ids_off = (int32_t)ids_off;
    d.n = q.n;
    d.x0 = q.x0;
    d.y0 = q.y0;
    d.w = q.w;
    d.h = q.h;
    d.nvr = (q.w + 15) / 16;
    d.pad = 0;
    ids_off += q.n;
    if (t.mode == CMP_BATCH_PERSISTENT) {
      const int rows = std::max(1, t.tile_vecs / d.nvr);
      for (int r0 = 0; r0 < q.h; r0 += rows) {
        const int nr = std::min(rows, q.h - r0);
        items.push_back(Item{r, r0, nr, 0});
        // cost order: largest first; row order: by the first raster row read
        cost.push_back(t.order == CMP_ORDER_COST ? (double)(q.n + 1) * nr * d.nvr
                                                 : -(double)(q.y0 + r0));
      }
    }
  }
  if (ids_off > INT32_MAX) return CMP_EINVAL;
  if (t.mode == CMP_BATCH_PERSISTENT) {
    // costliest items first, so the queue ends with small ones; or top to
    // bottom through the raster, so that concurrent items of different
    // requests read the same rows of shared members while they are cached
    std::vector<int> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<Item> sorted(items.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = items[order[i]];
    items.swap(sorted);
  }
  Header hd{};
  hd.nitems = (int32_t)items.size();
  hd.nreq = nreq;
  hd.reqs_off = 64;
  hd.items_off = align64(hd.reqs_off + (int64_t)sizeof(ReqDesc) * nreq);
  hd.ids_off = align64(hd.items_off + (int64_t)sizeof(Item) * items.size());
  hd.bits_off = (hd.ids_off + 4 * total_ids + 255) / 256 * 256;
  const int64_t mx_nc = mx_chunks(p->count);
  const int64_t bits_bytes = t.mode == CMP_BATCH_MATRIX ? mx_blocks * mx_nc * 256 : 0;
  const int64_t bytes = hd.bits_off + bits_bytes;

  if (hipSetDevice(p->dev) != hipSuccess) {
    p->poisoned = true;
    return CMP_EDEVICE;
  }
  int rc = ensure_arena(p, bytes);
  if (rc != CMP_OK) return rc;
  // the previous batch finished (runs are synchronous): the host arena is free
  std::memcpy(p->h_arena, &hd, sizeof(hd));
  std::memcpy(p->h_arena + hd.reqs_off, rd.data(), sizeof(ReqDesc) * nreq);
  if (!items.empty()) std::memcpy(p->h_arena + hd.items_off, items.data(), sizeof(Item) * items.size());
  int32_t *ids = reinterpret_cast<int32_t *>(p->h_arena + hd.ids_off);
  for (int32_t r = 0; r < nreq; ++r)
    if (reqs[r].n) std::memcpy(ids + rd[r].ids_off, reqs[r].ids, 4 * (size_t)reqs[r].n);
  if (bits_bytes) {
    // M of each block of 64 requests: byte [chunk][k-group][r % 16][(r % 64) / 16],
    // bit i = member 32 * chunk + 8 * k-group + i
    uint8_t *bits = reinterpret_cast<uint8_t *>(p->h_arena + hd.bits_off);
    std::memset(bits, 0, (size_t)bits_bytes);
    for (int32_t r = 0; r < nreq; ++r) {
      uint8_t *blk = bits + (int64_t)(r / kMxReqs) * mx_nc * 256 + ((r % 16) * 4 + (r % kMxReqs) / 16);
      for (int32_t i = 0; i < reqs[r].n; ++i) {
        const int32_t id = reqs[r].ids[i];
        blk[(id >> 5) * 256 + ((id >> 3) & 3) * 64] |= (uint8_t)(1u << (id & 7));
      }
    }
  }
  POOL_TRY(hipMemcpyAsync(p->d_arena, p->h_arena, bytes, hipMemcpyHostToDevice, p->s));
  POOL_TRY(hipEventRecord(p->ev0, p->s));
  if (t.mode != CMP_BATCH_PER_REQUEST) {
    const int kind = t.mode == CMP_BATCH_SHARED ? 1 : t.mode == CMP_BATCH_MATRIX ? 2 : 0;
    // k_matrix fits two workgroups per compute unit at once (registers)
    const int grid = p->cus * (kind == 2 ? std::min(t.blocks_per_cu, 2) : t.blocks_per_cu);
    auto launch = [&]() {
      return kind == 1   ? launch_shared(p, grid, t.stream_loads != 0, S)
             : kind == 2 ? launch_matrix(p, grid, t.stream_loads != 0)
                         : launch_persistent(p, grid, t.stream_loads != 0);
    };
    if (t.use_graph) {
      // graphs by mode, grid, load kind and (shared mode) slots per pass
      const int key = ((grid * 2 + t.stream_loads) * 4 + kind) * 64 + S;
      auto it = p->graphs.find(key);
      if (it == p->graphs.end()) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        POOL_TRY(hipStreamBeginCapture(p->s, hipStreamCaptureModeThreadLocal));
        const hipError_t le = launch();
        const hipError_t ce = hipStreamEndCapture(p->s, &g);
        if (le != hipSuccess || ce != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          p->poisoned = true;
          return CMP_EDEVICE;
        }
        const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
          p->poisoned = true;
          return CMP_EDEVICE;
        }
        it = p->graphs.emplace(key, ge).first;
      }
      POOL_TRY(hipGraphLaunch(it->second, p->s));
    } else {
      POOL_TRY(launch());
    }
  } else {
    const int32_t *d_ids = reinterpret_cast<const int32_t *>(p->d_arena + hd.ids_off);
    for (int32_t r = 0; r < nreq; ++r) {
      const int64_t nv = (int64_t)rd[r].h * rd[r].nvr;
      if (t.stream_loads)
        k_crop<true><<<(unsigned)((nv + 255) / 256), 256, 0, p->s>>>(p->base, p->stride, p->W, rd[r],
                                                                     d_ids + rd[r].ids_off);
      else
        k_crop<false><<<(unsigned)((nv + 255) / 256), 256, 0, p->s>>>(p->base, p->stride, p->W, rd[r],
                                                                      d_ids + rd[r].ids_off);
      POOL_TRY(hipGetLastError());
    }
  }
  POOL_TRY(hipEventRecord(p->ev1, p->s));
  POOL_TRY(hipEventSynchronize(p->ev1));
  float ms = 0.f;
  POOL_TRY(hipEventElapsedTime(&ms, p->ev0, p->ev1));
  p->last_ms = ms;
  p->last_items = t.mode == CMP_BATCH_PERSISTENT ? (int64_t)items.size()
                  : t.mode == CMP_BATCH_SHARED ? (int64_t)p->H * ((p->W + kShTile - 1) / kShTile)
                  : t.mode == CMP_BATCH_MATRIX ? mx_items
                                               : nreq;
  p->last_mode = t.mode;
  return CMP_OK;
}

int composite_batch_last(const cmp_pool *p, double *ms, int64_t *items, int32_t *mode) {
  if (!p || !ms || !items) return CMP_EINVAL;
  *ms = p->last_ms;
  *items = p->last_items;
  if (mode) *mode = p->last_mode;
  return CMP_OK;
}

}  // extern "C"
