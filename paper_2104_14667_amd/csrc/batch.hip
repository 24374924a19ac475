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
  int64_t pad[4];
};
static_assert(sizeof(Header) == 64, "arena header is 64 bytes");

// Counts of one 16-pixel vector of a request: pixels (y, x .. x+15) of the
// pool rasters ids[0..n), written to out[0..valid).
template <bool NT>
__device__ __forceinline__ void crop_vector(const uint8_t *__restrict__ base, int64_t stride,
                                            const int32_t *__restrict__ ids, int n, uint32_t off,
                                            uint32_t *__restrict__ out, int valid) {
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
      const uint4 v = make_uint4(cnt[4 * q], cnt[4 * q + 1], cnt[4 * q + 2], cnt[4 * q + 3]);
      __builtin_memcpy(out + 4 * q, &v, 16);
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
      uint32_t *out = R.out + (int64_t)(I.row0 + row) * R.pitch + 16 * j;
      crop_vector<NT>(base, stride, ids, R.n, off, out, min(16, R.w - 16 * j));
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
  crop_vector<NT>(base, stride, ids, R.n, off, R.out + (int64_t)row * R.pitch + 16 * j,
              min(16, R.w - 16 * j));
}

int64_t align64(int64_t x) { return (x + 63) / 64 * 64; }

}  // namespace



namespace {

void drop_graphs(cmp_pool *p) {
  for (auto &kv : p->graphs) hipGraphExecDestroy(kv.second);
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
  hipFree(p->d_arena);
  if (p->h_arena) hipHostFree(p->h_arena);
  p->d_arena = nullptr;
  p->h_arena = nullptr;
  p->arena_cap = 0;
  const int64_t cap = std::max<int64_t>(bytes, 1 << 20);
  if (hipMalloc((void **)&p->d_arena, cap) != hipSuccess) return CMP_ENOMEM;
  if (hipHostMalloc((void **)&p->h_arena, cap, hipHostMallocDefault) != hipSuccess) return CMP_ENOMEM;
  p->arena_cap = cap;
  return CMP_OK;
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
  t->mode = CMP_BATCH_PERSISTENT;
  t->tile_vecs = 1024;
  t->blocks_per_cu = 8;
  t->use_graph = 1;
  t->order = CMP_ORDER_ROWS;
  t->stream_loads = 0;
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
  hipSetDevice(p->dev);
  if (p->s) hipStreamSynchronize(p->s);
  drop_graphs(p);
  hipFree(p->d_arena);
  if (p->h_arena) hipHostFree(p->h_arena);
  hipFree(p->d_queue);
  if (p->ev0) hipEventDestroy(p->ev0);
  if (p->ev1) hipEventDestroy(p->ev1);
  if (p->s) hipStreamDestroy(p->s);
  delete p;
}

int composite_batch_run(cmp_pool *p, const cmp_request *reqs, int32_t nreq, const cmp_tune *tune) {
  if (!p) return CMP_EINVAL;
  if (p->poisoned) return CMP_EDEVICE;
  if (nreq < 0 || (nreq > 0 && !reqs)) return CMP_EINVAL;
  cmp_tune t;
  composite_default_tune(&t);
  if (tune) t = *tune;
  if (t.mode != CMP_BATCH_PERSISTENT && t.mode != CMP_BATCH_PER_REQUEST) return CMP_EINVAL;
  if (t.mode == CMP_BATCH_PERSISTENT &&
      (t.tile_vecs < 64 || t.tile_vecs > 65536 || t.blocks_per_cu < 1 || t.blocks_per_cu > 16 ||
       (t.use_graph != 0 && t.use_graph != 1) ||
       (t.order != CMP_ORDER_COST && t.order != CMP_ORDER_ROWS)))
    return CMP_EINVAL;
  if (t.stream_loads != 0 && t.stream_loads != 1) return CMP_EINVAL;
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
    return CMP_OK;
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
  const int64_t bytes = hd.ids_off + 4 * total_ids;

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
  POOL_TRY(hipMemcpyAsync(p->d_arena, p->h_arena, bytes, hipMemcpyHostToDevice, p->s));
  POOL_TRY(hipEventRecord(p->ev0, p->s));
  if (t.mode == CMP_BATCH_PERSISTENT) {
    const int grid = p->cus * t.blocks_per_cu;
    if (t.use_graph) {
      const int key = grid * 2 + t.stream_loads;
      auto it = p->graphs.find(key);
      if (it == p->graphs.end()) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        POOL_TRY(hipStreamBeginCapture(p->s, hipStreamCaptureModeThreadLocal));
        const hipError_t le = launch_persistent(p, grid, t.stream_loads != 0);
        const hipError_t ce = hipStreamEndCapture(p->s, &g);
        if (le != hipSuccess || ce != hipSuccess) {
          if (g) hipGraphDestroy(g);
          p->poisoned = true;
          return CMP_EDEVICE;
        }
        const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (ie != hipSuccess) {
          p->poisoned = true;
          return CMP_EDEVICE;
        }
        it = p->graphs.emplace(key, ge).first;
      }
      POOL_TRY(hipGraphLaunch(it->second, p->s));
    } else {
      POOL_TRY(launch_persistent(p, grid, t.stream_loads != 0));
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
  p->last_items = t.mode == CMP_BATCH_PERSISTENT ? (int64_t)items.size() : nreq;
  return CMP_OK;
}

int composite_batch_last(const cmp_pool *p, double *ms, int64_t *items) {
  if (!p || !ms || !items) return CMP_EINVAL;
  *ms = p->last_ms;
  *items = p->last_items;
  return CMP_OK;
}

}  // extern "C"
