// Compositing context: device composite, staging ring, streams, events and
// the member registry behind the C ABI in include/composite.h.
//
// The streamed path is the paper's dual-buffer algorithm (Section 4, Figure 3,
// "2b final" of the third implementation method): permanent receiving buffers
// on the device are filled from host memory by the copy engine while the
// previous chunk is composited, ordered by events (Section 4, last paragraph;
// Section 7.1):
//   copy stream:    [wait slot_free[k % nbuf]]; H2D chunk k; record copied[k % nbuf]
//   compute stream: wait copied[k % nbuf]; [repack to tiles]; composite;
//                   record slot_free[k % nbuf]
// Ordering is by events only: no host synchronisation inside the loop.  As an
// option (host_paced) the copy stream's wait on slot_free is replaced by a host
// wait on the same event, which happens when the kernel has long finished and
// the previous chunk is still uploading.  nbuf = 1 gives the single-buffer
// control (Figure 2): every upload waits for the kernel that read the previous
// one.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/composite.h"
#include "kernels.h"
#include "verify.h"

namespace {

constexpr int64_t kMaxPixels = (int64_t(1) << 32) - 16;  // 32-bit pixel indices
constexpr int64_t kSumGuard = 16843009;  // floor((2^32 - 1) / 255): members whose sum fits u32

struct Timed {
  hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace

struct cmp_ctx {
  int dev = 0;
  int32_t W = 0, H = 0;
  int64_t npix = 0;
  uint32_t outs = 0;
  int count_bits = 32;
  cmp_opts o{};
  bool poisoned = false;

  hipStream_t copy_s = nullptr, comp_s = nullptr;
  hipStream_t copy_s2 = nullptr;  // slot 1's uploads with copy_streams = 2
  bool own_copy = false, own_comp = false;

  void *d_count = nullptr;
  uint32_t *d_sum = nullptr;
  uint8_t *d_max = nullptr;
  // Outputs whose accumulators are logically zero but not written yet (after
  // init, clear, or the start of a max rebuild): the next add writes them
  // without reading (a set pass); anything else that needs their memory
  // fills them first (materialize).
  uint32_t zero_pending = 0;
  // With pingpong: the other accumulator of each output; a pass reads the
  // current one (above), writes this one, and the two are swapped.
  void *d_count_alt = nullptr;
  uint32_t *d_sum_alt = nullptr;
  uint8_t *d_max_alt = nullptr;

  // Staging ring (allocated on the first streamed call).
  int64_t stage_stride = 0;          // bytes between members in a slot
  int64_t tiled_stride = 0;          // bytes between members in a tiled slot
  uint8_t *d_stage[2] = {nullptr, nullptr};
  uint8_t *d_tiled[2] = {nullptr, nullptr};
  const uint8_t **d_slot_tab[2] = {nullptr, nullptr};  // member pointers of each slot
  hipEvent_t ev_copied[2] = {nullptr, nullptr};
  hipEvent_t ev_free[2] = {nullptr, nullptr};
  hipEvent_t ev_host_done = nullptr;  // last upload done: host maps reusable

  // Pointer tables for device-resident members: two pinned halves, each with
  // the event that marks its last upload done.
  const uint8_t **h_tab[2] = {nullptr, nullptr};
  const uint8_t **d_tab[2] = {nullptr, nullptr};
  int64_t tab_cap = 0;
  int tab_half = 0;
  int tab_last = -1;        // half holding the last uploaded table, or -1
  int64_t tab_last_n = 0;
  hipEvent_t ev_tab[2] = {nullptr, nullptr};

  // Pinned bounce buffers for uploads from pageable host memory, and pinned
  // staging for reads into pageable host memory (the library never relies on
  // the runtime's own handling of pageable memory).
  uint8_t *h_bounce[2] = {nullptr, nullptr};
  hipEvent_t ev_bounce[2] = {nullptr, nullptr};
  uint8_t *h_read[2] = {nullptr, nullptr};
  int64_t read_cap = 0;
  hipEvent_t ev_read[2] = {nullptr, nullptr};

  // Registry: members with multiplicity (anonymous ones under id -1) and,
  // with retain_members, their device pointers.
  int64_t members = 0;
  int64_t host_members = 0;  // members that came through composite_add
  std::unordered_map<int64_t, std::vector<const uint8_t *>> held;
  // With verify_members: the fingerprints of the members held under each id,
  // and device/pinned buffers that receive the fingerprints of one call.
  std::unordered_map<int64_t, std::vector<uint64_t>> fps;
  unsigned long long *d_fp = nullptr;
  unsigned long long *h_fp = nullptr;
  int64_t fp_cap = 0;

  // Histogram counters on the device and their pinned host copy (grown on
  // demand, together).
  unsigned long long *d_hist = nullptr;
  unsigned long long *h_hist = nullptr;
  int64_t hist_cap = 0;

  // Profiling of compositing kernels.
  std::vector<Timed> timed;
  size_t timed_used = 0;
  double timed_ms = 0.0;
  int64_t timed_launches = 0;
};

namespace {

#define CMP_TRY(call)                          \
  do {                                         \
    if ((call) != hipSuccess) {                \
      ctx->poisoned = true;                    \
      return CMP_EDEVICE;                      \
    }                                          \
  } while (0)

int elem_bytes(const cmp_ctx *ctx, uint32_t which) {
  if (which == CMP_COUNT) return ctx->count_bits / 8;
  if (which == CMP_SUM) return 4;
  if (which == CMP_MAX) return 1;
  return 0;
}

hipError_t set_device(const cmp_ctx *ctx) { return hipSetDevice(ctx->dev); }

// Device memory of the context: through the caller's allocator hooks when
// given (cmp_opts.dev_alloc / dev_free), else hipMalloc / hipFree.  Memory is
// freed only once the context's streams no longer use it.
bool dalloc(cmp_ctx *ctx, void **p, size_t bytes) {
  *p = nullptr;
  if (ctx->o.dev_alloc) *p = ctx->o.dev_alloc(bytes, ctx->o.alloc_ctx);
  else if (hipMalloc(p, bytes) != hipSuccess) *p = nullptr;
  return *p != nullptr;
}
void dfree(cmp_ctx *ctx, void *p) {
  if (!p) return;
  if (ctx->o.dev_free) ctx->o.dev_free(p, ctx->o.alloc_ctx);
  else (void)hipFree(p);
}

// Range guard: refuse any add that could overflow a stored value.
bool fits(const cmp_ctx *ctx, int64_t add) {
  const int64_t total = ctx->members + add;
  if ((ctx->outs & CMP_COUNT) && total > ((int64_t(1) << ctx->count_bits) - 1)) return false;
  if ((ctx->outs & CMP_SUM) && total > kSumGuard) return false;
  return total <= (int64_t(1) << 40);
}

void free_all(cmp_ctx *ctx) {
  (void)hipSetDevice(ctx->dev);
  if (ctx->comp_s) (void)hipStreamSynchronize(ctx->comp_s);
  if (ctx->copy_s) (void)hipStreamSynchronize(ctx->copy_s);
  if (ctx->copy_s2) (void)hipStreamSynchronize(ctx->copy_s2);
  dfree(ctx, ctx->d_count);
  dfree(ctx, ctx->d_sum);
  dfree(ctx, ctx->d_max);
  dfree(ctx, ctx->d_count_alt);
  dfree(ctx, ctx->d_sum_alt);
  dfree(ctx, ctx->d_max_alt);
  for (int i = 0; i < 2; ++i) {
    dfree(ctx, ctx->d_stage[i]);
    dfree(ctx, ctx->d_tiled[i]);
    dfree(ctx, ctx->d_slot_tab[i]);
    dfree(ctx, ctx->d_tab[i]);
    if (ctx->h_tab[i]) (void)hipHostFree(ctx->h_tab[i]);
    if (ctx->h_bounce[i]) (void)hipHostFree(ctx->h_bounce[i]);
    if (ctx->h_read[i]) (void)hipHostFree(ctx->h_read[i]);
    if (ctx->ev_bounce[i]) (void)hipEventDestroy(ctx->ev_bounce[i]);
    if (ctx->ev_read[i]) (void)hipEventDestroy(ctx->ev_read[i]);
    if (ctx->ev_copied[i]) (void)hipEventDestroy(ctx->ev_copied[i]);
    if (ctx->ev_free[i]) (void)hipEventDestroy(ctx->ev_free[i]);
    if (ctx->ev_tab[i]) (void)hipEventDestroy(ctx->ev_tab[i]);
  }
  if (ctx->ev_host_done) (void)hipEventDestroy(ctx->ev_host_done);
  dfree(ctx, ctx->d_hist);
  if (ctx->h_hist) (void)hipHostFree(ctx->h_hist);
  dfree(ctx, ctx->d_fp);
  if (ctx->h_fp) (void)hipHostFree(ctx->h_fp);
  for (auto &t : ctx->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  if (ctx->own_copy && ctx->copy_s) (void)hipStreamDestroy(ctx->copy_s);
  if (ctx->copy_s2) (void)hipStreamDestroy(ctx->copy_s2);
  if (ctx->own_comp && ctx->comp_s) (void)hipStreamDestroy(ctx->comp_s);
}

// Writes the zeros of the pending outputs among `which` (on the compute stream).
hipError_t materialize(cmp_ctx *ctx, uint32_t which) {
  const uint32_t w = ctx->zero_pending & which;
  hipError_t e = hipSuccess;
  if ((w & CMP_COUNT) && e == hipSuccess)
    e = cmp::launch_fill(ctx->d_count, 0, ctx->npix * (ctx->count_bits / 8), ctx->comp_s);
  if ((w & CMP_SUM) && e == hipSuccess) e = cmp::launch_fill(ctx->d_sum, 0, ctx->npix * 4, ctx->comp_s);
  if ((w & CMP_MAX) && e == hipSuccess) e = cmp::launch_fill(ctx->d_max, 0, ctx->npix, ctx->comp_s);
  if (e == hipSuccess) ctx->zero_pending &= ~w;
  return e;
}

// Brackets a compositing launch with events when profiling.
hipError_t timed_begin(cmp_ctx *ctx, Timed **t) {
  *t = nullptr;
  if (!ctx->o.profile) return hipSuccess;
  if (ctx->timed_used == ctx->timed.size()) {
    Timed n;
    hipError_t e = hipEventCreate(&n.a);
    if (e == hipSuccess) e = hipEventCreate(&n.b);
    if (e != hipSuccess) return e;
    ctx->timed.push_back(n);
  }
  *t = &ctx->timed[ctx->timed_used++];
  return hipEventRecord((*t)->a, ctx->comp_s);
}
hipError_t timed_end(cmp_ctx *ctx, Timed *t) {
  return t ? hipEventRecord(t->b, ctx->comp_s) : hipSuccess;
}
hipError_t harvest_timing(cmp_ctx *ctx) {
  for (size_t i = 0; i < ctx->timed_used; ++i) {
    hipError_t e = hipEventSynchronize(ctx->timed[i].b);
    if (e != hipSuccess) return e;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, ctx->timed[i].a, ctx->timed[i].b);
    if (e != hipSuccess) return e;
    ctx->timed_ms += ms;
    ctx->timed_launches += 1;
  }
  ctx->timed_used = 0;
  return hipSuccess;
}

// One compositing launch over n members (device table d_tab; tiled: the
// members are in the tiled layout).  In place, or with pingpong from the
// current accumulators into the other ones, which then become current.
hipError_t composite_pass(cmp_ctx *ctx, const uint8_t *const *d_tab, int n, bool sub,
                          uint32_t outs, bool tiled) {
  if (sub) outs &= ~(uint32_t)CMP_MAX;  // max has no inverse: never subtracted
  cmp::Outputs o;
  o.count16 = ctx->count_bits == 16;
  // an add over outputs that are all still zero writes them without reading
  // them (a set pass); any other mix writes the pending zeros first
  const uint32_t pend = ctx->zero_pending & outs;
  if (pend && !sub && pend == outs) {
    o.set = true;
  } else if (pend) {
    const hipError_t e = materialize(ctx, pend);
    if (e != hipSuccess) return e;
  }
  const bool pp = ctx->o.pingpong != 0;
  if (outs & CMP_COUNT) {
    o.count = pp ? ctx->d_count_alt : ctx->d_count;
    if (pp) o.count_in = ctx->d_count;
  }
  if (outs & CMP_SUM) {
    o.sum = pp ? ctx->d_sum_alt : ctx->d_sum;
    if (pp) o.sum_in = ctx->d_sum;
  }
  if (outs & CMP_MAX) {
    o.max = pp ? ctx->d_max_alt : ctx->d_max;
    if (pp) o.max_in = ctx->d_max;
  }
  Timed *t = nullptr;
  hipError_t e = timed_begin(ctx, &t);
  if (e != hipSuccess) return e;
  if (tiled) {
    cmp::Tiling tl{ctx->W, ctx->H, ctx->o.tile_w, ctx->o.tile_h};
    e = cmp::launch_composite_tiled(d_tab, n, tl, o, outs, sub, ctx->comp_s);
  } else {
    e = cmp::launch_composite_linear(d_tab, n, ctx->npix, o, outs, sub, ctx->comp_s);
  }
  if (e != hipSuccess) return e;
  ctx->zero_pending &= ~outs;
  if (pp) {
    if (outs & CMP_COUNT) std::swap(ctx->d_count, ctx->d_count_alt);
    if (outs & CMP_SUM) std::swap(ctx->d_sum, ctx->d_sum_alt);
    if (outs & CMP_MAX) std::swap(ctx->d_max, ctx->d_max_alt);
  }
  return timed_end(ctx, t);
}

// Bytes of one member raster as the device kernels read it: W*H, or the
// padded tiled plane in a CMP_TILED context (device rasters are tiled there).
int64_t member_bytes(const cmp_ctx *ctx) {
  if (ctx->o.layout != CMP_TILED) return ctx->npix;
  return cmp::Tiling{ctx->W, ctx->H, ctx->o.tile_w, ctx->o.tile_h}.plane();
}

void drop_staging(cmp_ctx *ctx) {
  for (int i = 0; i < 2; ++i) {
    dfree(ctx, ctx->d_stage[i]);
    dfree(ctx, ctx->d_tiled[i]);
    dfree(ctx, ctx->d_slot_tab[i]);
    ctx->d_stage[i] = ctx->d_tiled[i] = nullptr;
    ctx->d_slot_tab[i] = nullptr;
  }
}

int alloc_staging(cmp_ctx *ctx);

// Allocates the staging ring on first use; on failure nothing is kept.
int ensure_staging(cmp_ctx *ctx) {
  if (ctx->d_stage[0]) return CMP_OK;
  const int rc = alloc_staging(ctx);
  if (rc != CMP_OK) drop_staging(ctx);
  return rc;
}

int alloc_staging(cmp_ctx *ctx) {
  const int d = ctx->o.chunk_depth;
  ctx->stage_stride = (ctx->npix + 255) / 256 * 256;
  const bool tiled = ctx->o.layout == CMP_TILED;
  if (tiled) {
    cmp::Tiling tl{ctx->W, ctx->H, ctx->o.tile_w, ctx->o.tile_h};
    ctx->tiled_stride = (tl.plane() + 255) / 256 * 256;
  }
  for (int sidx = 0; sidx < ctx->o.nbuf; ++sidx) {
    if (!dalloc(ctx, (void **)&ctx->d_stage[sidx], ctx->stage_stride * d)) return CMP_ENOMEM;
    if (tiled && !dalloc(ctx, (void **)&ctx->d_tiled[sidx], ctx->tiled_stride * d)) return CMP_ENOMEM;
    if (!dalloc(ctx, (void **)&ctx->d_slot_tab[sidx], sizeof(void *) * d)) return CMP_ENOMEM;
    std::vector<const uint8_t *> tab(d);
    uint8_t *base = tiled ? ctx->d_tiled[sidx] : ctx->d_stage[sidx];
    const int64_t stride = tiled ? ctx->tiled_stride : ctx->stage_stride;
    for (int j = 0; j < d; ++j) tab[j] = base + j * stride;
    if (hipMemcpy(ctx->d_slot_tab[sidx], tab.data(), sizeof(void *) * d, hipMemcpyHostToDevice) != hipSuccess)
      return CMP_EDEVICE;
  }
  return CMP_OK;
}

// Uploads a device pointer table through the pinned double buffer and returns
// its device address (valid for work enqueued on the compute stream next).  A
// table equal to the last one uploaded is not uploaded again: its device copy
// is only overwritten by a later upload, which goes to the other half and is
// ordered on the compute stream after every kernel that reads this one.
int upload_table(cmp_ctx *ctx, const uint8_t *const *ptrs, int64_t n, const uint8_t ***d_out) {
  if (ctx->tab_last >= 0 && n == ctx->tab_last_n &&
      std::memcmp(ctx->h_tab[ctx->tab_last], ptrs, n * sizeof(void *)) == 0) {
    *d_out = ctx->d_tab[ctx->tab_last];
    return CMP_OK;
  }
  if (n > ctx->tab_cap) {
    ctx->tab_last = -1;
    for (int i = 0; i < 2; ++i) {
      if (ctx->ev_tab[i] && hipEventSynchronize(ctx->ev_tab[i]) != hipSuccess) return CMP_EDEVICE;
      if (ctx->h_tab[i]) (void)hipHostFree(ctx->h_tab[i]);
      dfree(ctx, ctx->d_tab[i]);
      ctx->h_tab[i] = nullptr;
      ctx->d_tab[i] = nullptr;
    }
    // the compute stream may still read the old device tables
    if (hipStreamSynchronize(ctx->comp_s) != hipSuccess) return CMP_EDEVICE;
    int64_t cap = std::max<int64_t>(n, 4096);
    for (int i = 0; i < 2; ++i) {
      if (hipHostMalloc((void **)&ctx->h_tab[i], cap * sizeof(void *), hipHostMallocDefault) != hipSuccess)
        return CMP_ENOMEM;
      if (!dalloc(ctx, (void **)&ctx->d_tab[i], cap * sizeof(void *))) return CMP_ENOMEM;
    }
    ctx->tab_cap = cap;
  }
  const int h = ctx->tab_half;
  ctx->tab_half ^= 1;
  // the pinned half may still be the source of an upload two calls ago
  if (hipEventSynchronize(ctx->ev_tab[h]) != hipSuccess) return CMP_EDEVICE;
  std::memcpy(ctx->h_tab[h], ptrs, n * sizeof(void *));
  if (hipMemcpyAsync(ctx->d_tab[h], ctx->h_tab[h], n * sizeof(void *), hipMemcpyHostToDevice,
                     ctx->comp_s) != hipSuccess)
    return CMP_EDEVICE;
  if (hipEventRecord(ctx->ev_tab[h], ctx->comp_s) != hipSuccess) return CMP_EDEVICE;
  ctx->tab_last = h;
  ctx->tab_last_n = n;
  *d_out = ctx->d_tab[h];
  return CMP_OK;
}

int ensure_bounce(cmp_ctx *ctx) {
  if (ctx->h_bounce[0]) return CMP_OK;
  const int64_t bytes = ctx->stage_stride * ctx->o.chunk_depth;
  for (int i = 0; i < ctx->o.nbuf; ++i) {
    if (hipHostMalloc((void **)&ctx->h_bounce[i], bytes, hipHostMallocDefault) != hipSuccess) {
      for (int j = 0; j < 2; ++j) {
        if (ctx->h_bounce[j]) (void)hipHostFree(ctx->h_bounce[j]);
        ctx->h_bounce[j] = nullptr;
      }
      return CMP_ENOMEM;
    }
  }
  return CMP_OK;
}

// Streams n host rasters through the staging slots with op add or sub on the
// outputs `outs` (none: upload only).  With fp non-null, fp[i] += the
// fingerprint of raster i, taken from the staging slot.
int stream_members(cmp_ctx *ctx, const uint8_t *const *maps, int32_t n, bool sub, uint32_t outs,
                   unsigned long long *fp = nullptr) {
  int rc = ensure_staging(ctx);
  if (rc != CMP_OK) return rc;
  const int d = ctx->o.chunk_depth;
  const int nb = ctx->o.nbuf;
  const bool tiled = ctx->o.layout == CMP_TILED;
  const int64_t plane = ctx->npix;
  const bool pinned = ctx->o.pageable_host == 0;
  if (!pinned) {
    // Pageable sources are first copied by the host into pinned bounce
    // buffers (one per slot), then uploaded by the copy engine.
    rc = ensure_bounce(ctx);
    if (rc != CMP_OK) return rc;
  }
  for (int32_t k0 = 0, k = 0; k0 < n; k0 += d, ++k) {
    const int slot = k % nb;
    const int cnt = std::min<int32_t>(d, n - k0);
    // the slot's uploads: on the copy stream, or slot 1's on a stream of its own
    hipStream_t cs = (slot == 1 && ctx->copy_s2) ? ctx->copy_s2 : ctx->copy_s;
    if (ctx->o.host_paced) {
      // the slot's last reader (chunk k - nbuf) is a short kernel that ran
      // while chunk k - 1 was uploading; that upload is still in flight
      CMP_TRY(hipEventSynchronize(ctx->ev_free[slot]));
    } else {
      CMP_TRY(hipStreamWaitEvent(cs, ctx->ev_free[slot], 0));
    }
    if (pinned) {
      // Runs of host rasters that are contiguous, and staged contiguously, go
      // as one copy.
      int j = 0;
      while (j < cnt) {
        int r = j + 1;
        if (ctx->stage_stride == plane)
          while (r < cnt && maps[k0 + r] == maps[k0 + r - 1] + plane) ++r;
        CMP_TRY(hipMemcpyAsync(ctx->d_stage[slot] + j * ctx->stage_stride, maps[k0 + j],
                               (size_t)(plane * (r - j)), hipMemcpyHostToDevice, cs));
        j = r;
      }
    } else {
      // the bounce buffer of this slot may still feed its previous upload
      CMP_TRY(hipEventSynchronize(ctx->ev_bounce[slot]));
      for (int j = 0; j < cnt; ++j)
        std::memcpy(ctx->h_bounce[slot] + j * ctx->stage_stride, maps[k0 + j], (size_t)plane);
      CMP_TRY(hipMemcpyAsync(ctx->d_stage[slot], ctx->h_bounce[slot],
                             (size_t)((cnt - 1) * ctx->stage_stride + plane), hipMemcpyHostToDevice,
                             cs));
      CMP_TRY(hipEventRecord(ctx->ev_bounce[slot], cs));
    }
    CMP_TRY(hipEventRecord(ctx->ev_copied[slot], cs));
    CMP_TRY(hipStreamWaitEvent(ctx->comp_s, ctx->ev_copied[slot], 0));
    if (fp && !tiled)
      CMP_TRY(cmp::launch_fingerprint(nullptr, ctx->d_stage[slot], ctx->stage_stride, cnt, plane,
                                      fp + k0, ctx->comp_s));
    if (tiled && outs == 0) {
      // fingerprints only: of the tiled copy, as for device rasters here
      cmp::Tiling tl{ctx->W, ctx->H, ctx->o.tile_w, ctx->o.tile_h};
      CMP_TRY(cmp::launch_repack_tiled(ctx->d_stage[slot], ctx->stage_stride, ctx->d_tiled[slot],
                                       ctx->tiled_stride, cnt, tl, ctx->comp_s));
      CMP_TRY(hipEventRecord(ctx->ev_free[slot], ctx->comp_s));
      CMP_TRY(cmp::launch_fingerprint(nullptr, ctx->d_tiled[slot], ctx->tiled_stride, cnt,
                                      tl.plane(), fp + k0, ctx->comp_s));
    } else if (outs == 0) {
      CMP_TRY(hipEventRecord(ctx->ev_free[slot], ctx->comp_s));
    } else if (tiled) {
      // The receiving buffer is free again once it is repacked (the paper's
      // decoupled transfer and transform); the tiled copy is only read by the
      // kernel that follows on the same stream.
      cmp::Tiling tl{ctx->W, ctx->H, ctx->o.tile_w, ctx->o.tile_h};
      Timed *t = nullptr;
      CMP_TRY(timed_begin(ctx, &t));
      CMP_TRY(cmp::launch_repack_tiled(ctx->d_stage[slot], ctx->stage_stride, ctx->d_tiled[slot],
                                       ctx->tiled_stride, cnt, tl, ctx->comp_s));
      CMP_TRY(timed_end(ctx, t));
      if (ctx->o.debug_poison)
        CMP_TRY(cmp::launch_fill(ctx->d_stage[slot], 0xA5, ctx->stage_stride * d, ctx->comp_s));
      CMP_TRY(hipEventRecord(ctx->ev_free[slot], ctx->comp_s));
      if (fp)  // of the tiled copy, as for device rasters in a tiled context
        CMP_TRY(cmp::launch_fingerprint(nullptr, ctx->d_tiled[slot], ctx->tiled_stride, cnt,
                                        tl.plane(), fp + k0, ctx->comp_s));
      CMP_TRY(composite_pass(ctx, ctx->d_slot_tab[slot], cnt, sub, outs, true));
    } else {
      CMP_TRY(composite_pass(ctx, ctx->d_slot_tab[slot], cnt, sub, outs, false));
      if (ctx->o.debug_poison)
        CMP_TRY(cmp::launch_fill(ctx->d_stage[slot], 0xA5, ctx->stage_stride * d, ctx->comp_s));
      CMP_TRY(hipEventRecord(ctx->ev_free[slot], ctx->comp_s));
    }
  }
  CMP_TRY(hipEventRecord(ctx->ev_host_done, ctx->copy_s));
  CMP_TRY(hipEventSynchronize(ctx->ev_host_done));
  if (ctx->copy_s2) CMP_TRY(hipStreamSynchronize(ctx->copy_s2));
  return CMP_OK;
}

// Zeroed device buffer for the fingerprints of n rasters, on the compute stream.
int begin_fingerprints(cmp_ctx *ctx, int64_t n) {
  if (n > ctx->fp_cap) {
    if (hipStreamSynchronize(ctx->comp_s) != hipSuccess) return CMP_EDEVICE;
    dfree(ctx, ctx->d_fp);
    if (ctx->h_fp) (void)hipHostFree(ctx->h_fp);
    ctx->d_fp = nullptr;
    ctx->h_fp = nullptr;
    ctx->fp_cap = 0;
    const int64_t cap = std::max<int64_t>(n, 1024);
    if (!dalloc(ctx, (void **)&ctx->d_fp, cap * 8)) return CMP_ENOMEM;
    if (hipHostMalloc((void **)&ctx->h_fp, cap * 8, hipHostMallocDefault) != hipSuccess) return CMP_ENOMEM;
    ctx->fp_cap = cap;
  }
  if (cmp::launch_fill(ctx->d_fp, 0, n * 8, ctx->comp_s) != hipSuccess) return CMP_EDEVICE;
  return CMP_OK;
}

// Waits for the fingerprints of n rasters and copies them to the host.
int end_fingerprints(cmp_ctx *ctx, int64_t n, std::vector<uint64_t> *out) {
  if (hipMemcpyAsync(ctx->h_fp, ctx->d_fp, n * 8, hipMemcpyDeviceToHost, ctx->comp_s) != hipSuccess ||
      hipStreamSynchronize(ctx->comp_s) != hipSuccess)
    return CMP_EDEVICE;
  out->assign(ctx->h_fp, ctx->h_fp + n);
  return CMP_OK;
}

// Fingerprints of n rasters (device pointers, or host rasters uploaded
// through the staging slots without touching the composite).
int fingerprints(cmp_ctx *ctx, const uint8_t *const *maps, int32_t n, bool on_device,
                 std::vector<uint64_t> *out) {
  int rc = begin_fingerprints(ctx, n);
  if (rc != CMP_OK) return rc;
  if (on_device) {
    const uint8_t **d_tab = nullptr;
    rc = upload_table(ctx, maps, n, &d_tab);
    if (rc != CMP_OK) return rc;
    if (cmp::launch_fingerprint(d_tab, nullptr, 0, n, member_bytes(ctx), ctx->d_fp, ctx->comp_s) !=
        hipSuccess)
      return CMP_EDEVICE;
  } else {
    rc = stream_members(ctx, maps, n, false, 0, ctx->d_fp);
    if (rc != CMP_OK) return rc;
  }
  return end_fingerprints(ctx, n, out);
}

int check_ids_removable(const cmp_ctx *ctx, const int64_t *ids, int32_t n) {
  std::unordered_map<int64_t, int64_t> need;
  for (int32_t i = 0; i < n; ++i) need[ids[i]] += 1;
  for (auto &kv : need) {
    auto it = ctx->held.find(kv.first);
    if (it == ctx->held.end() || (int64_t)it->second.size() < kv.second) return CMP_ENOTMEMBER;
  }
  return CMP_OK;
}

}  // namespace

extern "C" {

void composite_default_opts(cmp_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->nbuf = 2;
  o->chunk_depth = 8;
  o->layout = CMP_LINEAR;
  o->tile_w = 64;
  o->tile_h = 64;
  o->device = 0;
  o->host_paced = 0;
}

int composite_init(cmp_ctx **out, int32_t W, int32_t H, uint32_t outputs, int32_t count_bits,
                   const cmp_opts *opts) {
  if (!out) return CMP_EINVAL;
  *out = nullptr;
  if (W < 1 || H < 1 || (int64_t)W * H > kMaxPixels) return CMP_EINVAL;
  if (outputs == 0 || (outputs & ~7u)) return CMP_EINVAL;
  if ((outputs & CMP_COUNT) && count_bits != 16 && count_bits != 32) return CMP_EINVAL;
  cmp_opts o;
  composite_default_opts(&o);
  if (opts) o = *opts;
  if (o.nbuf < 1 || o.nbuf > 2) return CMP_EINVAL;
  if (o.chunk_depth < 1 || o.chunk_depth > cmp::kGroup) return CMP_EINVAL;
  if (o.layout != CMP_LINEAR && o.layout != CMP_TILED) return CMP_EINVAL;
  if (o.host_paced != 0 && o.host_paced != 1) return CMP_EINVAL;
  if (o.pageable_host != 0 && o.pageable_host != 1) return CMP_EINVAL;
  if (o.verify_members != 0 && o.verify_members != 1) return CMP_EINVAL;
  if (o.pingpong != 0 && o.pingpong != 1) return CMP_EINVAL;
  if (o.copy_streams < 0 || o.copy_streams > 2 || (o.copy_streams == 2 && o.nbuf != 2))
    return CMP_EINVAL;
  if ((o.dev_alloc == nullptr) != (o.dev_free == nullptr)) return CMP_EINVAL;
  if (o.layout == CMP_TILED) {
    if (o.tile_w != 16 && o.tile_w != 32 && o.tile_w != 64 && o.tile_w != 128) return CMP_EINVAL;
    if (o.tile_h < 1 || o.tile_h > 256) return CMP_EINVAL;
    if (W % 16) return CMP_EUNSUPPORTED;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return CMP_EDEVICE;
  if (o.device < 0 || o.device >= ndev) return CMP_EINVAL;

  cmp_ctx *ctx = new (std::nothrow) cmp_ctx();
  if (!ctx) return CMP_ENOMEM;
  ctx->dev = o.device;
  ctx->W = W;
  ctx->H = H;
  ctx->npix = (int64_t)W * H;
  ctx->outs = outputs;
  ctx->count_bits = (outputs & CMP_COUNT) ? count_bits : 32;
  ctx->o = o;
  int rc = CMP_EDEVICE;
  do {
    if (hipSetDevice(ctx->dev) != hipSuccess) break;
    if (o.copy_stream) {
      ctx->copy_s = (hipStream_t)o.copy_stream;
    } else {
      if (hipStreamCreateWithFlags(&ctx->copy_s, hipStreamNonBlocking) != hipSuccess) break;
      ctx->own_copy = true;
    }
    if (o.copy_streams == 2 &&
        hipStreamCreateWithFlags(&ctx->copy_s2, hipStreamNonBlocking) != hipSuccess)
      break;
    if (o.compute_stream) {
      ctx->comp_s = (hipStream_t)o.compute_stream;
    } else {
      if (hipStreamCreateWithFlags(&ctx->comp_s, hipStreamNonBlocking) != hipSuccess) break;
      ctx->own_comp = true;
    }
    bool ok = true;
    for (int i = 0; i < 2 && ok; ++i) {
      ok = hipEventCreateWithFlags(&ctx->ev_copied[i], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&ctx->ev_free[i], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&ctx->ev_tab[i], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&ctx->ev_bounce[i], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&ctx->ev_read[i], hipEventDisableTiming) == hipSuccess;
      // every event starts recorded, so the first wait on it is satisfied
      ok = ok && hipEventRecord(ctx->ev_free[i], ctx->comp_s) == hipSuccess &&
           hipEventRecord(ctx->ev_copied[i], ctx->copy_s) == hipSuccess &&
           hipEventRecord(ctx->ev_tab[i], ctx->comp_s) == hipSuccess &&
           hipEventRecord(ctx->ev_bounce[i], ctx->copy_s) == hipSuccess &&
           hipEventRecord(ctx->ev_read[i], ctx->comp_s) == hipSuccess;
    }
    if (!ok || hipEventCreateWithFlags(&ctx->ev_host_done, hipEventDisableTiming) != hipSuccess) break;
    rc = CMP_ENOMEM;
    const bool pp = o.pingpong != 0;
    if (outputs & CMP_COUNT) {
      if (!dalloc(ctx, &ctx->d_count, ctx->npix * (ctx->count_bits / 8) + 64)) break;
      if (pp && !dalloc(ctx, &ctx->d_count_alt, ctx->npix * (ctx->count_bits / 8) + 64)) break;
    }
    if (outputs & CMP_SUM) {
      if (!dalloc(ctx, (void **)&ctx->d_sum, ctx->npix * 4 + 64)) break;
      if (pp && !dalloc(ctx, (void **)&ctx->d_sum_alt, ctx->npix * 4 + 64)) break;
    }
    if (outputs & CMP_MAX) {
      if (!dalloc(ctx, (void **)&ctx->d_max, ctx->npix + 64)) break;
      if (pp && !dalloc(ctx, (void **)&ctx->d_max_alt, ctx->npix + 64)) break;
    }
    // the accumulators start logically cleared: the first add writes them
    ctx->zero_pending = outputs;
    rc = CMP_OK;
  } while (false);
  if (rc != CMP_OK) {
    free_all(ctx);
    delete ctx;
    return rc;
  }
  *out = ctx;
  return CMP_OK;
}

int composite_clear(cmp_ctx *ctx) {
  if (!ctx) return CMP_EINVAL;
  if (ctx->poisoned) return CMP_EDEVICE;
  CMP_TRY(set_device(ctx));
  // the clear must not overtake uploads still feeding the compute stream
  CMP_TRY(hipStreamSynchronize(ctx->copy_s));
  // nothing is written now: the next add writes the accumulators without
  // reading them, and a read before any add writes the zeros first
  ctx->zero_pending = ctx->outs;
  ctx->members = 0;
  ctx->host_members = 0;
  ctx->held.clear();
  ctx->fps.clear();
  return CMP_OK;
}

int composite_add(cmp_ctx *ctx, const uint8_t *const *host_maps, const int64_t *ids, int32_t n) {
  if (!ctx) return CMP_EINVAL;
  if (ctx->poisoned) return CMP_EDEVICE;
  if (n < 0 || (n > 0 && !host_maps)) return CMP_EINVAL;
  for (int32_t i = 0; i < n; ++i)
    if (!host_maps[i]) return CMP_EINVAL;
  if (n == 0) return CMP_OK;
  if (!fits(ctx, n)) return CMP_ERANGE;
  CMP_TRY(set_device(ctx));
  int rc = ensure_staging(ctx);
  if (rc != CMP_OK) return rc;
  const bool verify = ctx->o.verify_members != 0;
  if (verify) {
    rc = begin_fingerprints(ctx, n);
    if (rc != CMP_OK) return rc;
  }
  rc = stream_members(ctx, host_maps, n, false, ctx->outs, verify ? ctx->d_fp : nullptr);
  std::vector<uint64_t> fp;
  if (rc == CMP_OK && verify) rc = end_fingerprints(ctx, n, &fp);
  if (rc != CMP_OK) {
    ctx->poisoned = true;
    return rc == CMP_ENOMEM ? CMP_ENOMEM : CMP_EDEVICE;
  }
  ctx->members += n;
  ctx->host_members += n;
  for (int32_t i = 0; i < n; ++i) ctx->held[ids ? ids[i] : -1].push_back(nullptr);
  if (verify)
    for (int32_t i = 0; i < n; ++i) ctx->fps[ids ? ids[i] : -1].push_back(fp[i]);
  return CMP_OK;
}

int composite_add_device(cmp_ctx *ctx, const uint8_t *const *dev_maps, const int64_t *ids,
                         int32_t n) {
  if (!ctx) return CMP_EINVAL;
  if (ctx->poisoned) return CMP_EDEVICE;
  if (n < 0 || (n > 0 && !dev_maps)) return CMP_EINVAL;
  for (int32_t i = 0; i < n; ++i)
    if (!dev_maps[i]) return CMP_EINVAL;
  if (n == 0) return CMP_OK;
  if (!fits(ctx, n)) return CMP_ERANGE;
  CMP_TRY(set_device(ctx));
  const uint8_t **d_tab = nullptr;
  int rc = upload_table(ctx, dev_maps, n, &d_tab);
  if (rc != CMP_OK) {
    ctx->poisoned = true;
    return rc;
  }
  CMP_TRY(composite_pass(ctx, d_tab, n, false, ctx->outs, ctx->o.layout == CMP_TILED));
  std::vector<uint64_t> fp;
  if (ctx->o.verify_members) {
    rc = begin_fingerprints(ctx, n);
    if (rc == CMP_OK && cmp::launch_fingerprint(d_tab, nullptr, 0, n, member_bytes(ctx), ctx->d_fp,
                                                ctx->comp_s) != hipSuccess)
      rc = CMP_EDEVICE;
    if (rc == CMP_OK) rc = end_fingerprints(ctx, n, &fp);
    if (rc != CMP_OK) {
      ctx->poisoned = true;
      return rc;
    }
  }
  ctx->members += n;
  for (int32_t i = 0; i < n; ++i)
    ctx->held[ids ? ids[i] : -1].push_back(ctx->o.retain_members ? dev_maps[i] : nullptr);
  if (ctx->o.verify_members)
    for (int32_t i = 0; i < n; ++i) ctx->fps[ids ? ids[i] : -1].push_back(fp[i]);
  return CMP_OK;
}

int composite_remove(cmp_ctx *ctx, const uint8_t *const *maps, const int64_t *ids, int32_t n,
                     int32_t maps_on_device) {
  if (!ctx) return CMP_EINVAL;
  if (ctx->poisoned) return CMP_EDEVICE;
  if (n < 0) return CMP_EINVAL;
  if (n == 0) return CMP_OK;
  if (maps_on_device != 0 && maps_on_device != 1) return CMP_EINVAL;
  if (n > ctx->members) return ids ? CMP_ENOTMEMBER : CMP_EINVAL;
  std::vector<const uint8_t *> rm(n);
  if (ids) {
    int rc = check_ids_removable(ctx, ids, n);
    if (rc != CMP_OK) return rc;
  } else {
    auto it = ctx->held.find(-1);
    if (it == ctx->held.end() || (int64_t)it->second.size() < n) return CMP_ENOTMEMBER;
  }
  if (maps) {
    for (int32_t i = 0; i < n; ++i) {
      if (!maps[i]) return CMP_EINVAL;
      rm[i] = maps[i];
    }
  } else {
    // use the retained device rasters of the ids being removed
    if (!ids || !ctx->o.retain_members) return CMP_EINVAL;
    std::unordered_map<int64_t, size_t> used;
    for (int32_t i = 0; i < n; ++i) {
      auto &v = ctx->held.at(ids[i]);
      const uint8_t *p = v[used[ids[i]]++];
      if (!p) return CMP_EINVAL;  // that copy came from host memory
      rm[i] = p;
    }
    maps_on_device = 1;
  }
  const bool need_max = (ctx->outs & CMP_MAX) != 0;
  if (need_max && (!ctx->o.retain_members || ctx->host_members > 0)) return CMP_EUNSUPPORTED;

  CMP_TRY(set_device(ctx));
  // With verify_members every raster must carry a fingerprint held under its
  // id; the check reads the rasters once before anything is changed.
  auto fps = ctx->fps;
  if (ctx->o.verify_members) {
    std::vector<uint64_t> fp;
    int rc = fingerprints(ctx, rm.data(), n, maps_on_device != 0, &fp);
    if (rc != CMP_OK) {
      ctx->poisoned = true;
      return rc;
    }
    for (int32_t i = 0; i < n; ++i) {
      auto &v = fps[ids ? ids[i] : -1];
      auto it = std::find(v.begin(), v.end(), fp[i]);
      if (it == v.end()) return CMP_EINVAL;
      v.erase(it);
    }
    for (auto it = fps.begin(); it != fps.end();) {
      if (it->second.empty()) it = fps.erase(it);
      else ++it;
    }
  }

  // Registry after the removal (committed only on success).
  auto held = ctx->held;
  for (int32_t i = 0; i < n; ++i) {
    auto &v = held[ids ? ids[i] : -1];
    // drop the copy with this raster if the registry knows it, else any copy
    auto it = std::find(v.begin(), v.end(), rm[i]);
    if (it == v.end()) it = v.begin();
    v.erase(it);
  }
  std::vector<const uint8_t *> keep;
  if (need_max) {
    for (auto &kv : held)
      for (auto *p : kv.second) keep.push_back(p);
  }

  const uint32_t sub_outs = ctx->outs & (CMP_COUNT | CMP_SUM);
  if (sub_outs) {
    int rc;
    if (maps_on_device) {
      const uint8_t **d_tab = nullptr;
      rc = upload_table(ctx, rm.data(), n, &d_tab);
      if (rc == CMP_OK &&
          composite_pass(ctx, d_tab, n, true, sub_outs, ctx->o.layout == CMP_TILED) != hipSuccess)
        rc = CMP_EDEVICE;
    } else {
      rc = ensure_staging(ctx);
      if (rc != CMP_OK) return rc;
      rc = stream_members(ctx, rm.data(), n, true, sub_outs);
    }
    if (rc != CMP_OK) {
      ctx->poisoned = true;
      return rc;
    }
  }
  if (need_max) {
    // max has no inverse: rebuild it from the members that remain, the first
    // pass writing it from scratch (it is zero if none remain)
    ctx->zero_pending |= CMP_MAX;
    for (size_t k0 = 0; k0 < keep.size(); k0 += 65536) {
      const int cnt = (int)std::min<size_t>(65536, keep.size() - k0);
      const uint8_t **d_tab = nullptr;
      int rc = upload_table(ctx, keep.data() + k0, cnt, &d_tab);
      if (rc != CMP_OK) {
        ctx->poisoned = true;
        return rc;
      }
      CMP_TRY(composite_pass(ctx, d_tab, cnt, false, CMP_MAX, ctx->o.layout == CMP_TILED));
    }
  }
  for (auto it = held.begin(); it != held.end();) {
    if (it->second.empty()) it = held.erase(it);
    else ++it;
  }
  ctx->held.swap(held);
  ctx->fps.swap(fps);
  ctx->members -= n;
  return CMP_OK;
}

int composite_read(cmp_ctx *ctx, uint32_t which, int32_t x0, int32_t y0, int32_t w, int32_t h,
                   void *dst, int64_t dst_pitch_bytes, int32_t dst_kind) {
  if (!ctx) return CMP_EINVAL;
  if (ctx->poisoned) return CMP_EDEVICE;
  if (which != CMP_COUNT && which != CMP_SUM && which != CMP_MAX) return CMP_EINVAL;
  if (!(ctx->outs & which)) return CMP_EINVAL;
  if (x0 < 0 || y0 < 0 || w < 0 || h < 0 || (int64_t)x0 + w > ctx->W || (int64_t)y0 + h > ctx->H)
    return CMP_EINVAL;
  if (dst_kind != CMP_DST_HOST && dst_kind != CMP_DST_DEVICE && dst_kind != CMP_DST_PINNED)
    return CMP_EINVAL;
  const int eb = elem_bytes(ctx, which);
  if (w == 0 || h == 0) return CMP_OK;
  if (!dst || dst_pitch_bytes < (int64_t)w * eb) return CMP_EINVAL;
  const void *src = which == CMP_COUNT ? ctx->d_count
                    : which == CMP_SUM ? (const void *)ctx->d_sum
                                       : (const void *)ctx->d_max;
  CMP_TRY(set_device(ctx));
  CMP_TRY(hipStreamSynchronize(ctx->copy_s));
  CMP_TRY(materialize(ctx, which));
  if (dst_kind == CMP_DST_DEVICE) {
    CMP_TRY(cmp::launch_pack_window(src, eb, ctx->W, x0, y0, w, h, dst, dst_pitch_bytes, ctx->comp_s));
    CMP_TRY(hipStreamSynchronize(ctx->comp_s));
    return CMP_OK;
  }
  const uint8_t *s8 = static_cast<const uint8_t *>(src) + ((int64_t)y0 * ctx->W + x0) * eb;
  const size_t spitch = (size_t)ctx->W * eb, row = (size_t)w * eb;
  if (dst_kind == CMP_DST_PINNED) {
    CMP_TRY(hipMemcpy2DAsync(dst, (size_t)dst_pitch_bytes, s8, spitch, row, (size_t)h,
                             hipMemcpyDeviceToHost, ctx->comp_s));
    CMP_TRY(hipStreamSynchronize(ctx->comp_s));
    return CMP_OK;
  }
  // Pageable destination: bands of rows go through two pinned buffers; the
  // copy engine fills one while the host empties the other.
  const int64_t want = std::max<int64_t>(16 << 20, (int64_t)row);
  if (ctx->read_cap < want) {
    for (int i = 0; i < 2; ++i) {
      CMP_TRY(hipEventSynchronize(ctx->ev_read[i]));
      if (ctx->h_read[i]) (void)hipHostFree(ctx->h_read[i]);
      ctx->h_read[i] = nullptr;
    }
    ctx->read_cap = 0;
    for (int i = 0; i < 2; ++i)
      if (hipHostMalloc((void **)&ctx->h_read[i], want, hipHostMallocDefault) != hipSuccess)
        return CMP_ENOMEM;
    ctx->read_cap = want;
  }
  const int64_t band = std::max<int64_t>(1, ctx->read_cap / (int64_t)row);
  auto drain = [&](int slot, int64_t r0, int64_t rows) -> bool {
    if (hipEventSynchronize(ctx->ev_read[slot]) != hipSuccess) return false;
    uint8_t *d8 = static_cast<uint8_t *>(dst);
    for (int64_t r = 0; r < rows; ++r)
      std::memcpy(d8 + (r0 + r) * dst_pitch_bytes, ctx->h_read[slot] + r * row, row);
    return true;
  };
  int64_t prev_r0 = -1, prev_rows = 0;
  int prev_slot = 0;
  for (int64_t r0 = 0, b = 0; r0 < h; r0 += band, ++b) {
    const int slot = (int)(b & 1);
    const int64_t rows = std::min<int64_t>(band, h - r0);
    CMP_TRY(hipMemcpy2DAsync(ctx->h_read[slot], row, s8 + r0 * spitch, spitch, row, (size_t)rows,
                             hipMemcpyDeviceToHost, ctx->comp_s));
    CMP_TRY(hipEventRecord(ctx->ev_read[slot], ctx->comp_s));
    if (prev_r0 >= 0 && !drain(prev_slot, prev_r0, prev_rows)) {
      ctx->poisoned = true;
      return CMP_EDEVICE;
    }
    prev_r0 = r0;
    prev_rows = rows;
    prev_slot = slot;
  }
  if (prev_r0 >= 0 && !drain(prev_slot, prev_r0, prev_rows)) {
    ctx->poisoned = true;
    return CMP_EDEVICE;
  }
  return CMP_OK;
}

int composite_sync(cmp_ctx *ctx) {
  if (!ctx) return CMP_EINVAL;
  if (ctx->poisoned) return CMP_EDEVICE;
  CMP_TRY(set_device(ctx));
  CMP_TRY(hipStreamSynchronize(ctx->copy_s));
  CMP_TRY(hipStreamSynchronize(ctx->comp_s));
  CMP_TRY(harvest_timing(ctx));
  return CMP_OK;
}

int composite_members(const cmp_ctx *ctx, int64_t *n_out) {
  if (!ctx || !n_out) return CMP_EINVAL;
  *n_out = ctx->members;
  return CMP_OK;
}

int composite_device_buffer(cmp_ctx *ctx, uint32_t which, void **dev_ptr) {
  if (!ctx || !dev_ptr) return CMP_EINVAL;
  if (which != CMP_COUNT && which != CMP_SUM && which != CMP_MAX) return CMP_EINVAL;
  if (!(ctx->outs & which)) return CMP_EINVAL;
  if (ctx->poisoned) return CMP_EDEVICE;
  // the caller reads the memory itself: pending zeros are written first
  CMP_TRY(set_device(ctx));
  CMP_TRY(materialize(ctx, which));
  *dev_ptr = which == CMP_COUNT ? ctx->d_count
             : which == CMP_SUM ? (void *)ctx->d_sum
                                : (void *)ctx->d_max;
  return CMP_OK;
}

int composite_kernel_stats(cmp_ctx *ctx, int64_t *launches, double *total_ms, int32_t reset) {
  if (!ctx || !launches || !total_ms) return CMP_EINVAL;
  if (ctx->poisoned) return CMP_EDEVICE;
  CMP_TRY(set_device(ctx));
  CMP_TRY(harvest_timing(ctx));
  *launches = ctx->timed_launches;
  *total_ms = ctx->timed_ms;
  if (reset) {
    ctx->timed_launches = 0;
    ctx->timed_ms = 0.0;
  }
  return CMP_OK;
}

int composite_histogram(cmp_ctx *ctx, int64_t *bins, int32_t nbins, int64_t *overflow) {
  if (!ctx || !bins || !overflow) return CMP_EINVAL;
  if (ctx->poisoned) return CMP_EDEVICE;
  if (!(ctx->outs & CMP_COUNT) || nbins < 1 || nbins > (1 << 24)) return CMP_EINVAL;
  CMP_TRY(set_device(ctx));
  CMP_TRY(hipStreamSynchronize(ctx->copy_s));
  if (ctx->hist_cap < nbins + 1) {
    CMP_TRY(hipStreamSynchronize(ctx->comp_s));
    dfree(ctx, ctx->d_hist);
    if (ctx->h_hist) (void)hipHostFree(ctx->h_hist);
    ctx->d_hist = nullptr;
    ctx->h_hist = nullptr;
    ctx->hist_cap = 0;
    if (!dalloc(ctx, (void **)&ctx->d_hist, sizeof(unsigned long long) * (nbins + 1)))
      return CMP_ENOMEM;
    // the bins come back through page-locked memory of the context, never
    // through the runtime's handling of pageable memory
    if (hipHostMalloc((void **)&ctx->h_hist, sizeof(unsigned long long) * (nbins + 1),
                      hipHostMallocDefault) != hipSuccess)
      return CMP_ENOMEM;
    ctx->hist_cap = nbins + 1;
  }
  CMP_TRY(materialize(ctx, CMP_COUNT));
  unsigned long long *d_bins = ctx->d_hist;
  int cus = 256;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->dev);
  if (e == hipSuccess) e = cmp::launch_fill(d_bins, 0, sizeof(unsigned long long) * (nbins + 1), ctx->comp_s);
  if (e == hipSuccess)
    e = cmp::launch_histogram(ctx->d_count, ctx->count_bits == 16, ctx->npix, nbins, d_bins, cus,
                              ctx->comp_s);
  const unsigned long long *h = ctx->h_hist;
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->h_hist, d_bins, sizeof(unsigned long long) * (nbins + 1),
                       hipMemcpyDeviceToHost, ctx->comp_s);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->comp_s);
  if (e != hipSuccess) {
    ctx->poisoned = true;
    return CMP_EDEVICE;
  }
  for (int32_t k = 0; k < nbins; ++k) bins[k] = (int64_t)h[k];
  *overflow = (int64_t)h[nbins];
  return CMP_OK;
}

int64_t composite_tiled_bytes(int32_t W, int32_t H, int32_t tile_w, int32_t tile_h) {
  if (W < 1 || H < 1 || tile_w < 1 || tile_h < 1) return -1;
  cmp::Tiling tl{W, H, tile_w, tile_h};
  return tl.plane();
}

int composite_repack_tiled(const uint8_t *src, int64_t src_stride, uint8_t *dst, int64_t dst_stride,
                           int32_t n, int32_t W, int32_t H, int32_t tile_w, int32_t tile_h,
                           void *stream) {
  if (!src || !dst || n < 0 || n > 65535 || W < 1 || H < 1) return CMP_EINVAL;
  if (tile_w != 16 && tile_w != 32 && tile_w != 64 && tile_w != 128) return CMP_EINVAL;
  if (tile_h < 1 || tile_h > 256) return CMP_EINVAL;
  const int64_t plane = (int64_t)W * H;
  cmp::Tiling tl{W, H, tile_w, tile_h};
  if (plane > (int64_t(1) << 32) - 16 || src_stride < plane || dst_stride < tl.plane()) return CMP_EINVAL;
  if (n == 0) return CMP_OK;
  if (cmp::launch_repack_tiled(src, src_stride, dst, dst_stride, n, tl, (hipStream_t)stream) != hipSuccess)
    return CMP_EDEVICE;
  return CMP_OK;
}

const char *composite_strerror(int status) {
  switch (status) {
    case CMP_OK: return "ok";
    case CMP_EINVAL: return "invalid argument";
    case CMP_ENOMEM: return "out of memory";
    case CMP_ERANGE: return "composite value could overflow its stored width";
    case CMP_ENOTMEMBER: return "not a member of the working set";
    case CMP_EUNSUPPORTED: return "unsupported in this configuration";
    case CMP_EDEVICE: return "GPU unavailable or HIP failure";
    case CMP_EBUSY: return "busy";
    case CMP_ETIMEDOUT: return "timed out";
    case CMP_ECANCELED: return "not attempted: an earlier failure ended the call";
    default: return "unknown status";
  }
}

void composite_free(cmp_ctx *ctx) {
  if (!ctx) return;
  free_all(ctx);
  delete ctx;
}

}  // extern "C"
