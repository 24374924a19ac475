// Linear -> tiled transform of uint8 rasters for gfx950: the counterpart of
// the paper's buffer-to-image conversion (Section 4, third implementation
// method; its rate is measured in Section 5.2), whose tiled result the
// compositing kernels read in the tiled layout.
//
// Staged through LDS.  A workgroup takes R rows of a 1024-byte-wide block of
// one raster: rows r0 .. r0 + R - 1 of the tiles tx0 .. tx0 + 1024 / tw - 1 of
// tile row ty.  Each thread first issues all of its loads (whole 1 KiB row
// segments per wave, up to 8 16-byte vectors per thread in flight), then
// stores them to LDS; after one barrier each tile's R rows are written as one
// contiguous run (R * tw bytes: rows of a tile are consecutive in the tiled
// layout).  Both the reads and the writes are long runs of HBM.  Bytes outside
// the raster (right and bottom edge tiles) are written as zero.

#include "kernels.h"
#include "lanes.h"

#include <algorithm>

namespace cmp {
namespace {

constexpr uint32_t kBlockW = 1024;            // bytes of a row per workgroup
constexpr uint32_t kPitch = kBlockW + 16;     // LDS row pitch: rows start on different banks
constexpr uint32_t kMaxRows = 32;             // rows per workgroup at most
constexpr uint32_t kThreads = 256;
constexpr uint32_t kPerThread = kMaxRows * (kBlockW / 16) / kThreads;  // 8 vectors

struct Geom {
  uint32_t W, H, tw, th, ntx;
  uint32_t vpr_log;  // log2(tw / 16): vectors per tile row
  uint32_t R;        // rows per workgroup (<= th, <= kMaxRows)
  uint32_t nsb;      // row groups per tile row: ceil(th / R)
  uint32_t ncb;      // 1024-byte column blocks: ceil(ntx * tw / 1024)
};

// 16 bytes of row-major raster s at (x, y), zero past its right and bottom
// edges.  A vector that crosses the right edge is loaded whole when its 16
// bytes lie inside the raster (they run into the next row) and the bytes past
// the edge are cleared; only at the raster's very end, where a whole load
// would leave the raster, it is read byte by byte, all 15 loads issued at
// once.
__device__ __forceinline__ uint4 load_vec(const uint8_t *__restrict__ s, const Geom &g, uint32_t x,
                                          uint32_t y) {
  if (y >= g.H || x >= g.W) return make_uint4(0u, 0u, 0u, 0u);
  const uint32_t off = y * g.W + x;  // < W * H < 2^32
  if (x + 16u <= g.W) return ld16(s, off);
  const uint32_t nb = g.W - x;  // bytes of the vector inside the row: 1 .. 15
  if ((uint64_t)off + 16u <= (uint64_t)g.W * g.H) {
    const uint4 v = ld16(s, off);
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (uint32_t d = 0; d < 4; ++d) {
      const uint32_t keep = nb >= 4 * d + 4 ? 4u : (nb > 4 * d ? nb - 4 * d : 0u);  // bytes kept
      w[d] &= keep == 4u ? 0xffffffffu : (1u << (8 * keep)) - 1u;
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
  }
  uint32_t b[15];
#pragma unroll
  for (uint32_t k = 0; k < 15; ++k) b[k] = k < nb ? (uint32_t)s[off + k] : 0u;
  uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (uint32_t k = 0; k < 15; ++k) w[k >> 2] |= b[k] << (8 * (k & 3));
  return make_uint4(w[0], w[1], w[2], w[3]);
}

__global__ __launch_bounds__(kThreads) void k_repack(const uint8_t *__restrict__ src,
                                                     int64_t src_stride, uint8_t *__restrict__ dst,
                                                     int64_t dst_stride, Geom g) {
  __shared__ uint4 lds[kMaxRows * kPitch / 16];
  uint8_t *l8 = reinterpret_cast<uint8_t *>(lds);
  const uint32_t b = blockIdx.x;
  const uint32_t cb = b % g.ncb, t2 = b / g.ncb;
  const uint32_t sb = t2 % g.nsb, ty = t2 / g.nsb;
  const uint32_t r0 = sb * g.R;
  const uint32_t rows = min(g.R, g.th - r0);
  const uint32_t y0 = ty * g.th + r0, x0 = cb * kBlockW;
  const uint8_t *s = src + (int64_t)blockIdx.y * src_stride;
  const uint32_t nin = rows * (kBlockW / 16);  // vectors in: rows x 64

  // all loads first, then the LDS stores: every load of a thread is in flight
  // at once instead of one full HBM latency per vector
  uint4 val[kPerThread];
#pragma unroll
  for (uint32_t u = 0; u < kPerThread; ++u) {
    const uint32_t v = threadIdx.x + u * kThreads;
    val[u] = v < nin ? load_vec(s, g, x0 + 16u * (v & 63u), y0 + (v >> 6)) : make_uint4(0u, 0u, 0u, 0u);
  }
#pragma unroll
  for (uint32_t u = 0; u < kPerThread; ++u) {
    const uint32_t v = threadIdx.x + u * kThreads;
    if (v < nin) *reinterpret_cast<uint4 *>(l8 + (v >> 6) * kPitch + 16u * (v & 63u)) = val[u];
  }
  __syncthreads();

  // each tile's rows r0 .. r0 + rows - 1 out, contiguous in the tiled layout
  const uint32_t K = kBlockW / g.tw;
  const uint32_t tx0 = cb * K;
  const uint32_t ktiles = min(K, g.ntx - tx0);
  const uint32_t per_tile = rows << g.vpr_log;  // vectors of one tile's part
  const uint32_t nout = ktiles * per_tile;
  const uint32_t vmask = (1u << g.vpr_log) - 1u;
  const int64_t tile_bytes = (int64_t)g.tw * g.th;
  uint8_t *d = dst + (int64_t)blockIdx.y * dst_stride + ((int64_t)ty * g.ntx + tx0) * tile_bytes +
               (int64_t)r0 * g.tw;
#pragma unroll
  for (uint32_t u = 0; u < kPerThread; ++u) {
    const uint32_t v = threadIdx.x + u * kThreads;
    if (v < nout) {
      const uint32_t k = v / per_tile, in = v - k * per_tile;
      const uint32_t r = in >> g.vpr_log, c = in & vmask;
      const uint4 x = *reinterpret_cast<const uint4 *>(l8 + r * kPitch + k * g.tw + 16u * c);
      *reinterpret_cast<uint4 *>(d + k * tile_bytes + 16u * in) = x;
    }
  }
}

}  // namespace

hipError_t launch_repack_tiled(const uint8_t *src, int64_t src_stride, uint8_t *dst,
                               int64_t dst_stride, int n, const Tiling &t, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (t.tw < 16 || t.tw > (int)kBlockW || kBlockW % t.tw || t.tw % 16 || t.th < 1 || n > 65535)
    return hipErrorInvalidValue;
  if ((int64_t)t.W * t.H >= (int64_t(1) << 32) || t.plane() / 16 >= (int64_t(1) << 28))
    return hipErrorInvalidValue;
  Geom g;
  g.W = (uint32_t)t.W;
  g.H = (uint32_t)t.H;
  g.tw = (uint32_t)t.tw;
  g.th = (uint32_t)t.th;
  g.ntx = (uint32_t)t.ntx();
  g.vpr_log = 0;
  while ((16u << g.vpr_log) < g.tw) ++g.vpr_log;
  g.R = std::min<uint32_t>(g.th, kMaxRows);
  g.nsb = (g.th + g.R - 1) / g.R;
  g.ncb = (uint32_t)(((int64_t)g.ntx * g.tw + kBlockW - 1) / kBlockW);
  // every vector in and out of a workgroup has a slot: R rows of 64 vectors,
  // and at most K tiles of R rows of tw / 16 vectors (K * tw = 1024)
  static_assert(kPerThread * kThreads == kMaxRows * (kBlockW / 16), "load slots");
  const int64_t blocks = (int64_t)t.nty() * g.nsb * g.ncb;
  if (blocks >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  dim3 grid((unsigned)blocks, (unsigned)n);
  k_repack<<<grid, kThreads, 0, s>>>(src, src_stride, dst, dst_stride, g);
  return hipGetLastError();
}

}  // namespace cmp
