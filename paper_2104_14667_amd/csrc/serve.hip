// Served sessions (composite_server_*, composite_session_*): continuous
// batching of interactive add/remove requests against per-session
// device-resident count composites.
//
// Threads:
//   submitters (any)  validate a request against the session's projected
//                     working set and append it to the queue;
//   worker            forms a step from the queue (the oldest request of each
//                     session, at most max_batch), makes the step's sessions
//                     resident and launches the update kernel on the compute
//                     stream, with the step's descriptors in its kernel
//                     arguments (small steps) or uploaded ahead of it; the
//                     kernel writes the viewports into the callers' page-
//                     locked memory.  Unless a full step's worth of requests
//                     already waits, the rows holding viewports are launched
//                     first and the rest second, so that the requests are
//                     complete before the rest of the update is;
//   completer         waits for each step's viewport launch in order and
//                     completes its requests (timestamps, waiters).
// At most two steps are in flight; their descriptors, staging and events
// alternate between two halves.  With overlap = 0 the worker waits for each
// step to complete before forming the next (the unbatched FIFO baseline uses
// max_batch = 1 and overlap = 0).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <mutex>
#include <new>
#include <thread>
#include <type_traits>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/composite.h"
#include "lanes.h"
#include "pool.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

enum : int32_t { kModeAdd = 0, kModeSub = 1, kModeSet = 2 };

struct SReq {
  void *comp;         // session composite (device): uint16 or uint32 counts
  void *view;         // the caller's page-locked viewport (device address): vh rows of vw
                      // counts of the composite's width, vpitch counts apart
  int32_t mode, ids_off, n;  // kMode*: composite += / -= / = count of ids
  int32_t vx0, vy0, vw, vh;
  int32_t vb0, vb1;          // the row blocks holding the viewport: [vb0, vb1)
  int32_t it_view, it_rest;  // this request's first item among the viewport items / the others
  int32_t vpitch;
};
static_assert(sizeof(SReq) == 64, "request descriptor is 64 bytes");

// A step's descriptors: in device memory (an uploaded arena), or, for a step
// of at most kArgReqs requests and kArgIds ids, in the launch's own kernel
// arguments, which need no upload.
struct ArenaStep {
  const SReq *reqs;
  const int32_t *ids;
  __device__ const SReq &req(int k) const { return reqs[k]; }
  __device__ int32_t id(int i) const { return ids[i]; }
};
template <int NR, int NI>
struct ArgStepT {
  static constexpr int kReqs = NR, kIds = NI;
  SReq reqs[NR];
  int32_t ids[NI];
  __device__ const SReq &req(int k) const { return reqs[k]; }
  __device__ int32_t id(int i) const { return ids[i]; }
};
// the one-request steps of interactive serving (0.4 KiB of arguments), and
// steps of up to 8 requests (2.6 KiB)
typedef ArgStepT<2, 64> ArgStep1;
typedef ArgStepT<8, 512> ArgStep;
constexpr int kArgReqs = ArgStep::kReqs, kArgIds = ArgStep::kIds;
static_assert(sizeof(ArgStep) <= 4096, "kernel arguments stay within 4 KiB");

// Work items.  A session composite is nb blocks of `rows` rows.  A request's
// viewport items are groups of `group` blocks from vb0 on over [vb0, vb1),
// the blocks holding its viewport (the last group may be shorter): fewer,
// larger workgroups for the launch that writes the viewports over PCIe, so
// that the other rows' launch finds room beside it.  Its other items are the
// single blocks outside [vb0, vb1).  A step's items are all blocks of all its
// requests (phase 0, request-major), only the viewport items (phase 1), only
// the others (phase 2), each request's in order, or the nview items of phase
// 1 followed by those of phase 2 (phase 3: one launch that writes the
// viewports first).  The request of an item in phases 1 and 2 is found by a
// binary search over the requests' first items (the last request whose first
// item is at most it; a request with no items in the phase shares its first
// item with the next one and is passed over).  Out: request k, first block b
// and blocks nblk.
enum : int32_t { kPhaseAll = 0, kPhaseView = 1, kPhaseRest = 2, kPhaseViewFirst = 3 };

template <class D>
__device__ __forceinline__ void item_of(const D &d, int nreq, int nb, int group, int nview, int phase,
                                        int it, int &k, int &b, int &nblk) {
  nblk = 1;
  if (phase == kPhaseViewFirst) {
    if (it < nview) {
      phase = kPhaseView;
    } else {
      phase = kPhaseRest;
      it -= nview;
    }
  }
  if (phase == kPhaseAll) {
    k = it / nb;
    b = it - k * nb;
    return;
  }
  int lo = 0, hi = nreq - 1;  // invariant: first(lo) <= it
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int f = phase == kPhaseView ? d.req(mid).it_view : d.req(mid).it_rest;
    if (f <= it) lo = mid;
    else hi = mid - 1;
  }
  k = lo;
  const SReq &R = d.req(k);
  if (phase == kPhaseView) {
    b = R.vb0 + group * (it - R.it_view);
    nblk = min(group, R.vb1 - b);
  } else {
    const int j = it - R.it_rest;
    b = j < R.vb0 ? j : j + (R.vb1 - R.vb0);
  }
}

// Row segment [0, n) of a viewport from LDS (element l0 on) to the caller's
// host memory: 16-byte stores from the first 16-byte boundary of the
// destination on, single counts before it and after the last whole vector, so
// that the writes cross PCIe as whole lines whatever the viewport's position.
template <class T>
__device__ __forceinline__ void put_row(T *__restrict__ drow, const T *__restrict__ lds, int l0, int n) {
  constexpr int E = 16 / sizeof(T);  // counts per 16-byte store
  const int mis = (int)((reinterpret_cast<uintptr_t>(drow) & 15u) / sizeof(T));
  const int h = min(n, (E - mis) % E);  // counts before the first boundary
  const int nvec = (n - h) / E;
  typedef __attribute__((address_space(1))) T gT;
  gT *g = (gT *)drow;
  for (int i = threadIdx.x; i < h; i += blockDim.x) g[i] = lds[l0 + i];
  for (int i = threadIdx.x; i < nvec; i += blockDim.x) {
    uint32_t w[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if constexpr (sizeof(T) == 2)
        w[m] = (uint32_t)lds[l0 + h + E * i + 2 * m] | ((uint32_t)lds[l0 + h + E * i + 2 * m + 1] << 16);
      else
        w[m] = lds[l0 + h + E * i + m];
    }
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    *(__attribute__((address_space(1))) v4u *)(g + h + E * i) = v4u{w[0], w[1], w[2], w[3]};
  }
  for (int i = h + E * nvec + (int)threadIdx.x; i < n; i += blockDim.x) g[i] = lds[l0 + i];
}

// One work item: rows [b * rows, b * rows + rows) of a session composite, in
// chunks of 256 vectors of 16 pixels.  Each thread updates 16 pixels (count
// +/- the nonzero members, or count set to that of the whole working set when
// the composite is rebuilt).  A chunk holding viewport rows also stages its
// new counts in LDS, and the workgroup writes the viewport's part of them to
// the caller's page-locked memory (in the composite's width: uint16 or
// uint32), visible to the host once the launch has completed.  C16: the
// session composites are uint16 (the server refuses a request that would take
// a session past 65535 members, so no lane carries into its neighbour).
template <bool C16, class D>
__global__ __launch_bounds__(256) void k_serve(const uint8_t *__restrict__ base, int64_t stride,
                                               int32_t W, int32_t H, int32_t rows, int32_t nb,
                                               int32_t nreq, int32_t group, int32_t phase,
                                               int32_t nitems, int32_t nview, uint32_t *__restrict__ queue,
                                               const D d) {
  const int nvr = W >> 4;
  constexpr int NQ = C16 ? 2 : 4;  // 16-byte words of composite per 16 pixels
  typedef typename std::conditional<C16, uint16_t, uint32_t>::type T;
  __shared__ int s_item;
  __shared__ uint4 s_px[256 * NQ];  // a chunk's new counts, pixel-major
  T *px = reinterpret_cast<T *>(s_px);
  for (int pass = 0;; ++pass) {
    int it;
    if (queue) {
      // persistent grid: items from the queue
      if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
      __syncthreads();
      it = __builtin_amdgcn_readfirstlane(s_item);
      __syncthreads();
    } else {
      // one item per workgroup: no queue, no barrier
      it = pass == 0 ? (int)blockIdx.x : nitems;
    }
    if (it >= nitems) break;  // the queue counter only grows: every wave exits
    int k, b, nblk;
    item_of(d, nreq, nb, group, nview, phase, it, k, b, nblk);
    const SReq &R = d.req(k);
    const int row0 = b * rows;
    const int nrows = min(nblk * rows, H - row0);
    const int total = nrows * nvr;
    // chunks of blockDim vectors: every thread takes every chunk, so the
    // barriers of a chunk holding viewport rows are reached by all
    for (int v0 = 0; v0 < total; v0 += blockDim.x) {
      const int cend = min(total, v0 + (int)blockDim.x);
      // item rows r_lo .. r_hi hold this chunk; va .. vb of them are viewport rows
      const int r_lo = v0 / nvr, r_hi = (cend - 1) / nvr;
      const int va = max(r_lo, R.vy0 - row0), vb = min(r_hi, R.vy0 + R.vh - 1 - row0);
      const int v = v0 + (int)threadIdx.x;
      if (v < total) {
      const int row = v / nvr, j = v - row * nvr;
      const int y = row0 + row, x = 16 * j;
      const uint32_t off = (uint32_t)y * (uint32_t)W + (uint32_t)x;
      // global-space pointers (the descriptors' are generic): global, not
      // flat, loads and stores
      typedef unsigned int v4u __attribute__((ext_vector_type(4)));
      __attribute__((address_space(1))) v4u *c =
          C16 ? (__attribute__((address_space(1))) v4u *)(static_cast<uint16_t *>(R.comp) + off)
              : (__attribute__((address_space(1))) v4u *)(static_cast<uint32_t *>(R.comp) + off);
      // the old composite is requested first, so that its latency overlaps
      // the member loads instead of trailing them
      v4u o[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) o[q] = v4u{0u, 0u, 0u, 0u};
      if (R.mode != kModeSet) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) o[q] = c[q];
      }
      uint32_t cnt[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) cnt[q] = 0u;
      const int ids0 = R.ids_off, n = R.n;
      for (int g0 = 0; g0 < n; g0 += cmp::kGroup) {
        const int g1 = min(n, g0 + cmp::kGroup);
        cmp::Acc<cmp::kCount> a;
        a.zero();
        int i = g0;
        for (; i + 16 <= g1; i += 16) {
          uint4 xs[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) xs[u] = cmp::ld16(base + (int64_t)d.id(ids0 + i + u) * stride, off);
#pragma unroll
          for (int u = 0; u < 16; ++u) a.fold(xs[u]);
        }
        for (; i + 4 <= g1; i += 4) {
          uint4 xs[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) xs[u] = cmp::ld16(base + (int64_t)d.id(ids0 + i + u) * stride, off);
#pragma unroll
          for (int u = 0; u < 4; ++u) a.fold(xs[u]);
        }
        for (; i < g1; ++i) a.fold(cmp::ld16(base + (int64_t)d.id(ids0 + i) * stride, off));
#pragma unroll
        for (int q = 0; q < 16; ++q) cnt[q] += cmp::lane_px(a.c, q);
      }
      uint32_t nv[16];
      if constexpr (C16) {
        // pixels 2m and 2m+1 share dword m of the composite (low half first)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          uint32_t w[4] = {o[q].x, o[q].y, o[q].z, o[q].w};
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const uint32_t dd = cnt[8 * q + 2 * m] | (cnt[8 * q + 2 * m + 1] << 16);
            w[m] = R.mode == kModeSub ? cmp::psub(w[m], dd) : cmp::padd(w[m], dd);
            nv[8 * q + 2 * m] = w[m] & 0xffffu;
            nv[8 * q + 2 * m + 1] = w[m] >> 16;
          }
          c[q] = v4u{w[0], w[1], w[2], w[3]};
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const v4u dd = {cnt[4 * q], cnt[4 * q + 1], cnt[4 * q + 2], cnt[4 * q + 3]};
          if (R.mode == kModeSub) o[q] -= dd;
          else o[q] += dd;
          c[q] = o[q];
          nv[4 * q] = o[q].x; nv[4 * q + 1] = o[q].y; nv[4 * q + 2] = o[q].z; nv[4 * q + 3] = o[q].w;
        }
      }
      if (va <= vb) {
        // this chunk holds viewport rows: its new counts to LDS
        uint32_t pk[4 * NQ];
        if constexpr (C16) {
#pragma unroll
          for (int m = 0; m < 8; ++m) pk[m] = nv[2 * m] | (nv[2 * m + 1] << 16);
        } else {
#pragma unroll
          for (int m = 0; m < 16; ++m) pk[m] = nv[m];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          s_px[NQ * threadIdx.x + q] = make_uint4(pk[4 * q], pk[4 * q + 1], pk[4 * q + 2], pk[4 * q + 3]);
      }
      }  // v < total
      if (va <= vb) {
        __syncthreads();
        for (int r = va; r <= vb; ++r) {
          // pixels of item row r in this chunk (item-local, row-major), and
          // their part inside the viewport
          const int p0 = max(16 * v0, r * W), p1 = min(16 * cend, r * W + W);
          const int xa = max(p0 - r * W, R.vx0), xb = min(p1 - r * W, R.vx0 + R.vw);
          if (xa < xb) {
            T *drow = static_cast<T *>(R.view) + (int64_t)(row0 + r - R.vy0) * R.vpitch + (xa - R.vx0);
            put_row<T>(drow, px, r * W + xa - 16 * v0, xb - xa);
          }
        }
        // LDS is free for the next chunk; after the last one nothing waits
        // for the host writes to drain (the launch's end does)
        if (v0 + (int)blockDim.x < total) __syncthreads();
      }
    }
  }
}

// Mean members per request above which an automatic step runs persistent,
// and the most work items it launches one workgroup each (a larger step runs
// persistent too, well inside the launch's grid limits).
constexpr int64_t kServeHeavy = 64;
// Row blocks per work item of the launch that writes the viewports, unless
// the options set it.  On the served workload (one 1024x1024 viewport of a
// 4096x4096 session per step) 1, 2, 4, 8 and 16 gave p50 0.090, 0.095,
// 0.098, 0.12 and 0.17 ms for 0.088, 0.086, 0.079, 0.084 and 0.12 ms of
// device time per request: larger groups leave the other rows' launch more
// room and lengthen the viewport launch.  Latency first.
constexpr int kServeViewGroup = 1;
constexpr size_t kServeMaxGrid = size_t(1) << 22;

struct Request {
  uint64_t ticket;
  int64_t sid;
  int32_t op;
  std::vector<int32_t> ids;
  int32_t vx0, vy0, vw, vh;
  void *dst;    // vh rows of vw counts (uint16 or uint32: the composite's width)
  void *dview;  // dst's device address
  int64_t pitch;
  int64_t t_submit;
};

struct Session {
  bool open = false;
  int slot = -1;            // resident slot or -1
  bool has_data = false;    // false: all zero (new); true: data in slot, spill, or dropped
  bool dropped = false;     // evicted without a copy: rebuilt from `applied` when next used
  uint8_t *spill = nullptr;  // pinned host copy while spilled
  std::unordered_map<int32_t, int64_t> projected;  // working set after queued requests
  std::unordered_map<int32_t, int64_t> applied;    // working set after launched requests
  int64_t projected_n = 0;
  int64_t applied_n = 0;
  int64_t inflight = 0;     // requests submitted and not completed
  // Eviction priority (GreedyDual): the floor at the last use plus the cost
  // of bringing the composite back; ties go to the least recently used.
  double gd_h = 0.0;
  uint64_t last_use = 0;
};

struct Done {
  int64_t t_submit, t_done;
};

struct Step {
  std::vector<uint64_t> tickets;
  std::vector<int64_t> sids;
  int half;
  uint64_t index;
  int64_t t_formed, t_enq;  // requests taken from the queue; last enqueue done
  bool split;               // viewport launch, and a rest launch on the second stream
};

}  // namespace

struct cmp_server {
  cmp_pool *pool = nullptr;
  cmp_server_opts o{};
  int dev = 0;
  int32_t W = 0, H = 0;
  int64_t comp_bytes = 0;         // one session composite: W*H*count_bits/8
  int64_t admit_limit = 0;        // sessions admitted at most (HBM budget)
  hipStream_t comp = nullptr;
  hipStream_t rest = nullptr;  // a split step's launch of the rows outside its viewports
  size_t view_lds = 0;         // dynamic LDS of a viewport launch's workgroup (unused: a cap)
  uint8_t *slab = nullptr;
  std::vector<int64_t> slot_owner;  // session id per slot, or -1
  uint32_t *d_queue = nullptr;
  // per half: descriptor arena (pinned + device), viewport staging, events
  char *h_arena[2] = {nullptr, nullptr};
  char *d_arena[2] = {nullptr, nullptr};
  int64_t arena_cap = 0;
  hipEvent_t ev_ref = nullptr;                    // recorded at creation: the time origin
  double busy_until = 0.0;                        // ms after ev_ref: end of the last step's span
  hipEvent_t ev_k0[2] = {nullptr, nullptr};      // a step's start (compute stream)
  hipEvent_t ev_rest[2] = {nullptr, nullptr};    // a split step's rest launch has ended
  hipEvent_t ev_pre[2] = {nullptr, nullptr};     // compute stream before a viewport launch
  hipEvent_t ev_view[2] = {nullptr, nullptr};  // the step's viewports are in host memory

  std::mutex mu;
  std::condition_variable cv_queue, cv_done, cv_steps;
  std::deque<Request> queue;
  std::unordered_map<int64_t, Session> sessions;
  int64_t next_sid = 1;
  int64_t open_sessions = 0;
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, Done> done;
  std::unordered_set<uint64_t> pending;
  std::deque<Step> steps;        // launched, not completed (for the completer)
  uint64_t steps_launched = 0, steps_completed = 0;
  uint64_t use_clock = 0;
  double gd_floor = 0.0;         // priority of the last evicted session
  bool stop = false;
  bool paused = false;
  bool worker_done = false;
  int failed = CMP_OK;           // sticky device failure
  cmp_server_stats st{};
  std::thread worker, completer;
};

namespace {

void fail(cmp_server *s, int rc) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->failed == CMP_OK) s->failed = rc;
  s->cv_done.notify_all();
  s->cv_steps.notify_all();
}

// Makes `sid` resident.  Called by the worker with the server lock held.
// *rebuild is set when the slot holds no valid composite and the step's
// kernel must write the composite of the session's whole working set.
// A residency copy, enqueued on the compute stream once the step knows what
// it must wait for.
struct SlotCopy {
  void *dst;
  const void *src;
  hipMemcpyKind kind;
};

hipError_t make_resident(cmp_server *s, Session &ss, int64_t sid,
                         const std::unordered_set<int64_t> &in_step, bool *rebuild,
                         std::vector<SlotCopy> &copies) {
  *rebuild = false;
  if (ss.slot >= 0) return hipSuccess;
  int slot = -1;
  for (size_t i = 0; i < s->slot_owner.size(); ++i)
    if (s->slot_owner[i] < 0) {
      slot = (int)i;
      break;
    }
  if (slot < 0) {
    // evict the resident session outside this step with the lowest priority
    int64_t victim = -1;
    double low = 0.0;
    uint64_t oldest = 0;
    for (size_t i = 0; i < s->slot_owner.size(); ++i) {
      const int64_t v = s->slot_owner[i];
      if (in_step.count(v)) continue;
      const Session &c = s->sessions[v];
      if (victim < 0 || c.gd_h < low || (c.gd_h == low && c.last_use < oldest)) {
        low = c.gd_h;
        oldest = c.last_use;
        victim = v;
        slot = (int)i;
      }
    }
    if (victim < 0) return hipErrorOutOfMemory;  // cannot happen: slots >= max_batch
    Session &vs = s->sessions[victim];
    s->gd_floor = vs.gd_h;
    if (vs.applied_n <= s->o.remat_max_members) {
      // recounting its members from the resident pool costs less than moving
      // the composite out and back over PCIe: drop it
      vs.dropped = true;
      s->st.drops += 1;
    } else {
      if (!vs.spill) {
        hipError_t e = hipHostMalloc((void **)&vs.spill, s->comp_bytes, hipHostMallocDefault);
        if (e != hipSuccess) return e;
      }
      // ordered after every kernel that wrote the slot (compute stream)
      copies.push_back({vs.spill, s->slab + (int64_t)slot * s->comp_bytes, hipMemcpyDeviceToHost});
      vs.dropped = false;
      s->st.spills += 1;
    }
    vs.slot = -1;
    s->slot_owner[slot] = -1;
  }
  uint8_t *dst = s->slab + (int64_t)slot * s->comp_bytes;
  if (ss.has_data && !ss.dropped) {
    copies.push_back({dst, ss.spill, hipMemcpyHostToDevice});
    s->st.restores += 1;
  } else {
    // new (all zero) or dropped: the step writes the whole composite
    *rebuild = true;
    if (ss.has_data) s->st.rebuilds += 1;
  }
  ss.dropped = false;
  ss.slot = slot;
  ss.has_data = true;
  s->slot_owner[slot] = sid;
  return hipSuccess;
}

void worker_body(cmp_server *s);

void worker_loop(cmp_server *s) {
  if (hipSetDevice(s->dev) != hipSuccess) fail(s, CMP_EDEVICE);
  else worker_body(s);
  std::lock_guard<std::mutex> lk(s->mu);
  s->worker_done = true;
  s->cv_steps.notify_all();
  s->cv_done.notify_all();
}

void worker_body(cmp_server *s) {
  bool prev_split = false;  // the previous step launched rows on the rest stream
  std::vector<void *> prev_comps;  // the composites that step updates (sorted)
  for (;;) {
    std::vector<Request> step;
    uint64_t index;
    bool backlog = false;  // a full step's worth of requests still waiting
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // a paused server forms no step (free stops it anyway, after draining)
      s->cv_queue.wait(lk, [&] { return s->stop || (!s->queue.empty() && !s->paused); });
      if (s->queue.empty() && s->stop) return;
      if (s->failed != CMP_OK) return;
      index = s->steps_launched;
      // both halves busy, or (no overlap) the previous step still running
      const uint64_t need = s->o.overlap ? (index >= 2 ? index - 1 : 0) : index;
      s->cv_steps.wait(lk, [&] { return s->steps_completed >= need || s->failed != CMP_OK; });
      if (s->failed != CMP_OK) return;
      std::unordered_set<int64_t> taken;
      for (auto it = s->queue.begin(); it != s->queue.end() && (int)step.size() < s->o.max_batch;) {
        if (taken.insert(it->sid).second) {
          step.push_back(std::move(*it));
          it = s->queue.erase(it);
        } else {
          ++it;
        }
      }
      backlog = s->queue.size() >= (size_t)s->o.max_batch;
    }
    const int64_t t_formed = now_ns();
    const int half = (int)(index & 1), prev = half ^ 1;
    hipError_t e = hipSuccess;
    std::vector<SlotCopy> scopies;  // residency copies of this step, in order
    std::unordered_set<int64_t> in_step;
    for (auto &r : step) in_step.insert(r.sid);
    // residency and descriptors (slots are touched by this thread only)
    std::vector<SReq> rd(step.size());
    std::vector<std::vector<int32_t>> rebuilt(step.size());  // ids of rebuilt composites
    const int rows = std::max(1, s->o.tile_vecs / (s->W / 16));  // rows per work item
    const int nb = (s->H + rows - 1) / rows;                     // row blocks per session
    const int group = s->o.view_group > 0 ? s->o.view_group : kServeViewGroup;
    int64_t nview = 0, nrest = 0;  // viewport items (groups of blocks), other items (blocks)
    int64_t nids = 0;
    // Residency changes hold the lock: sessions may be opened and closed
    // concurrently, and a close releases the slot of an idle session.
    std::unique_lock<std::mutex> lk(s->mu);
    for (size_t k = 0; k < step.size() && e == hipSuccess; ++k) {
      Request &r = step[k];
      Session *ss = &s->sessions[r.sid];
      // (make_resident collects its spill and restore copies; they are
      // enqueued on the compute stream below)
      bool rebuild = false;
      e = make_resident(s, *ss, r.sid, in_step, &rebuild, scopies);
      if (e != hipSuccess) break;
      // the working set the composite holds once this request has run
      for (int32_t id : r.ids) {
        if (r.op == CMP_OP_REMOVE) {
          if (--ss->applied[id] == 0) ss->applied.erase(id);
          ss->applied_n -= 1;
        } else {
          ss->applied[id] += 1;
          ss->applied_n += 1;
        }
      }
      // GreedyDual: a session stays ahead of the floor by what its eviction
      // would cost (members to recount, or the copy when that is cheaper)
      ss->gd_h = s->gd_floor + 1.0 + (double)std::min<int64_t>(ss->applied_n, s->o.remat_max_members);
      ss->last_use = ++s->use_clock;
      SReq &d = rd[k];
      d.comp = s->slab + (int64_t)ss->slot * s->comp_bytes;
      d.view = r.dview;
      d.vpitch = (int32_t)r.pitch;
      d.mode = rebuild ? kModeSet : r.op == CMP_OP_REMOVE ? kModeSub : kModeAdd;
      if (rebuild) {
        std::vector<int32_t> &v = rebuilt[k];
        v.reserve(ss->applied_n);
        for (auto &kv : ss->applied) v.insert(v.end(), (size_t)kv.second, kv.first);
      }
      d.ids_off = (int32_t)nids;
      d.n = (int32_t)(rebuild ? rebuilt[k].size() : r.ids.size());
      d.vx0 = r.vx0;
      d.vy0 = r.vy0;
      d.vw = r.vw;
      d.vh = r.vh;
      // the row blocks holding the viewport, and this request's first item
      // among the step's viewport blocks and among the others
      d.vb0 = r.vy0 / rows;
      d.vb1 = (r.vy0 + r.vh + rows - 1) / rows;
      d.it_view = (int32_t)nview;
      d.it_rest = (int32_t)nrest;
      nview += (d.vb1 - d.vb0 + group - 1) / group;
      nrest += nb - (d.vb1 - d.vb0);
      nids += d.n;
    }
    lk.unlock();
    if (e != hipSuccess) {
      fail(s, CMP_EDEVICE);
      return;
    }
    // What this step puts on the compute stream (residency copies, launches)
    // follows the previous step's rest launch if it touches one of that
    // step's composite slots: the same session, or a slot given to another
    // session since (evicted or closed).  Every slot this step touches holds
    // one of its own composites (an evicted session's slot is handed to one).
    // Steps before the previous one have completed.
    std::vector<void *> comps(rd.size());
    for (size_t k = 0; k < rd.size(); ++k) comps[k] = rd[k].comp;
    std::sort(comps.begin(), comps.end());
    if (prev_split) {
      bool touch = false;
      for (void *c : comps) touch = touch || std::binary_search(prev_comps.begin(), prev_comps.end(), c);
      if (touch) {
        e = hipEventQuery(s->ev_rest[prev]);
        if (e == hipErrorNotReady) {
          (void)hipGetLastError();
          e = hipStreamWaitEvent(s->comp, s->ev_rest[prev], 0);
        }
      }
    }
    for (size_t i = 0; i < scopies.size() && e == hipSuccess; ++i)
      e = hipMemcpyAsync(scopies[i].dst, scopies[i].src, s->comp_bytes, scopies[i].kind, s->comp);
    const int64_t nall = (int64_t)step.size() * nb;  // work items of the step
    // blocks_per_cu 0 (automatic): steps of small requests (16 members on
    // average in the served workload) run one workgroup per item, with no
    // queue, atomic or barrier per item; steps whose requests average more
    // than kServeHeavy members (rebuilds of evicted sessions, ~300) run a
    // persistent grid of 2 workgroups per compute unit, whose lower
    // occupancy interleaves fewer member streams (both measured faster)
    const bool persistent = s->o.blocks_per_cu > 0 || nids > kServeHeavy * (int64_t)step.size() ||
                            nall > (int64_t)kServeMaxGrid;
    const int bpc = s->o.blocks_per_cu > 0 ? s->o.blocks_per_cu : 2;
    // descriptors: a small step's travel in the kernel arguments (a block of
    // the smallest size that holds them); a larger one's are uploaded
    // (requests, then ids) ahead of its launches
    const bool small = (int64_t)step.size() <= kArgReqs && nids <= kArgIds;
    ArgStep as;
    ArgStep1 as1;
    const bool tiny = (int64_t)step.size() <= ArgStep1::kReqs && nids <= ArgStep1::kIds;
    ArenaStep ar{};
    auto put_ids = [&](int32_t *dst) {
      for (size_t k = 0; k < step.size(); ++k) {
        const std::vector<int32_t> &v = rd[k].mode == kModeSet ? rebuilt[k] : step[k].ids;
        if (!v.empty()) std::memcpy(dst + rd[k].ids_off, v.data(), 4 * v.size());
      }
    };
    if (tiny) {
      std::memcpy(as1.reqs, rd.data(), sizeof(SReq) * rd.size());
      put_ids(as1.ids);
    } else if (small) {
      std::memcpy(as.reqs, rd.data(), sizeof(SReq) * rd.size());
      put_ids(as.ids);
    } else {
      const int64_t ids_off = ((int64_t)sizeof(SReq) * rd.size() + 63) / 64 * 64;
      const int64_t bytes = ids_off + 4 * nids;
      if (bytes > s->arena_cap) {
        fail(s, CMP_ENOMEM);
        return;
      }
      char *h = s->h_arena[half];
      std::memcpy(h, rd.data(), sizeof(SReq) * rd.size());
      put_ids(reinterpret_cast<int32_t *>(h + ids_off));
      if (e == hipSuccess) e = hipMemcpyAsync(s->d_arena[half], h, bytes, hipMemcpyHostToDevice, s->comp);
      ar.reqs = reinterpret_cast<const SReq *>(s->d_arena[half]);
      ar.ids = reinterpret_cast<const int32_t *>(s->d_arena[half] + ids_off);
    }
    if (e == hipSuccess && persistent) e = cmp::launch_fill(s->d_queue, 0, 4, s->comp);
    const bool copies = !scopies.empty();  // residency copies this step
    if (e == hipSuccess) e = hipEventRecord(s->ev_k0[half], s->comp);
    const int nreq = (int)step.size();
    auto launch = [&](hipStream_t st, int64_t items, int phase, uint32_t *q) {
      if (items <= 0) return hipSuccess;
      const unsigned g = q ? (unsigned)(s->pool->cus * bpc) : (unsigned)items;
      const int ni = (int)items;
#define CMP_SERVE(C16, D, arg)                                                                     \
  k_serve<C16, D><<<g, 256, phase == kPhaseView ? s->view_lds : 0, st>>>(                          \
      s->pool->base, s->pool->stride, s->W, s->H, rows, nb, nreq, group, phase, ni, (int)nview, q, arg)
      if (s->o.count_bits == 16) {
        if (tiny) CMP_SERVE(true, ArgStep1, as1);
        else if (small) CMP_SERVE(true, ArgStep, as);
        else CMP_SERVE(true, ArenaStep, ar);
      } else {
        if (tiny) CMP_SERVE(false, ArgStep1, as1);
        else if (small) CMP_SERVE(false, ArgStep, as);
        else CMP_SERVE(false, ArenaStep, ar);
      }
#undef CMP_SERVE
      return hipGetLastError();
    };
    const bool split = !persistent && !backlog && nrest > 0;
    if (persistent) {
      // one persistent grid over all items; the viewports are final at its end
      if (e == hipSuccess) e = launch(s->comp, nall, kPhaseAll, s->d_queue);
      if (e == hipSuccess) e = hipEventRecord(s->ev_view[half], s->comp);
    } else if (!split) {
      // the next step is full already (or every row holds a viewport): one
      // launch, the viewport rows first
      if (e == hipSuccess) e = launch(s->comp, nview + nrest, kPhaseViewFirst, nullptr);
      if (e == hipSuccess) e = hipEventRecord(s->ev_view[half], s->comp);
    } else {
      // The viewport rows' items on the compute stream: the step's requests
      // are complete when that launch is, and it is mostly the PCIe writes of
      // the viewports.  The other rows on the rest stream at the same time.
      // The rest launch follows what the compute stream holds before the
      // viewport launch (this step's residency copies and uploaded
      // descriptors, the previous step's launches): unless nothing is
      // pending there, it waits for an event recorded just before the
      // viewport launch.
      bool wait = copies || !small;
      if (!wait && e == hipSuccess) {
        const hipError_t q = hipEventQuery(s->ev_view[prev]);
        if (q == hipErrorNotReady) (void)hipGetLastError();
        wait = q != hipSuccess;
      }
      if (wait && e == hipSuccess) e = hipEventRecord(s->ev_pre[half], s->comp);
      if (wait && e == hipSuccess) e = hipStreamWaitEvent(s->rest, s->ev_pre[half], 0);
      if (e == hipSuccess) e = launch(s->comp, nview, kPhaseView, nullptr);
      if (e == hipSuccess) e = hipEventRecord(s->ev_view[half], s->comp);
      if (e == hipSuccess) e = launch(s->rest, nrest, kPhaseRest, nullptr);
      if (e == hipSuccess) e = hipEventRecord(s->ev_rest[half], s->rest);
    }
    prev_split = split;
    prev_comps = split ? std::move(comps) : std::vector<void *>();
    if (e != hipSuccess) {
      fail(s, CMP_EDEVICE);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      Step st;
      st.half = half;
      st.index = index;
      st.t_formed = t_formed;
      st.t_enq = now_ns();
      st.split = split;
      for (auto &r : step) {
        st.tickets.push_back(r.ticket);
        st.sids.push_back(r.sid);
      }
      s->steps.push_back(std::move(st));
      s->steps_launched += 1;
      s->st.steps += 1;
      s->st.max_step = std::max<int64_t>(s->st.max_step, (int64_t)step.size());
    }
    s->cv_steps.notify_all();
  }
}

void completer_loop(cmp_server *s) {
  if (hipSetDevice(s->dev) != hipSuccess) {
    fail(s, CMP_EDEVICE);
    return;
  }
  for (;;) {
    Step st;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_steps.wait(lk, [&] { return !s->steps.empty() || s->worker_done || s->failed != CMP_OK; });
      if (s->steps.empty()) {
        if (s->worker_done || s->failed != CMP_OK) return;
        continue;
      }
      st = s->steps.front();
    }
    // The step's requests are complete once the launch that writes their
    // viewports has ended (its writes to host memory are visible then): they
    // complete now, while the rows outside the viewports may still be
    // updating on the rest stream.
    const hipError_t e = hipEventSynchronize(s->ev_view[st.half]);
    const int64_t t = now_ns();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (e != hipSuccess) {
        // waiters of this step see the failure (their tickets stay pending)
        if (s->failed == CMP_OK) s->failed = CMP_EDEVICE;
      } else {
        for (size_t k = 0; k < st.tickets.size(); ++k) {
          auto it = s->done.find(st.tickets[k]);
          if (it != s->done.end()) {
            it->second.t_done = t;
            s->st.wait_ms += 1e-6 * (double)(st.t_formed - it->second.t_submit);
            s->st.host_ms += 1e-6 * (double)(st.t_enq - st.t_formed);
            s->st.flight_ms += 1e-6 * (double)(t - st.t_enq);
          }
          s->pending.erase(st.tickets[k]);
          s->sessions[st.sids[k]].inflight -= 1;
          s->st.requests += 1;
        }
      }
    }
    s->cv_done.notify_all();
    // device time: the step's span, from its start until its last launch has
    // ended, counted where it does not overlap the previous step's (steps
    // complete in order); the step's half is free again after that
    // (the span from events close in time; only where it starts, for the
    // overlap, from the reference event recorded at creation)
    float view_ms = 0.f, rest_ms = 0.f, t0 = 0.f;
    hipError_t e2 = e;
    if (e2 == hipSuccess) e2 = hipEventElapsedTime(&view_ms, s->ev_k0[st.half], s->ev_view[st.half]);
    if (e2 == hipSuccess && st.split) e2 = hipEventSynchronize(s->ev_rest[st.half]);
    if (e2 == hipSuccess && st.split) e2 = hipEventElapsedTime(&rest_ms, s->ev_k0[st.half], s->ev_rest[st.half]);
    if (e2 == hipSuccess) e2 = hipEventElapsedTime(&t0, s->ev_ref, s->ev_k0[st.half]);
    const double span = std::max(view_ms, rest_ms);
    std::lock_guard<std::mutex> lk(s->mu);
    s->steps.pop_front();
    if (e2 != hipSuccess && s->failed == CMP_OK) s->failed = CMP_EDEVICE;
    const double overlap = std::min(span, std::max(0.0, s->busy_until - (double)t0));
    s->st.device_ms += span - overlap;
    s->busy_until = std::max(s->busy_until, (double)t0 + span);
    s->st.view_ms += view_ms;
    s->steps_completed += 1;
    s->cv_done.notify_all();
    s->cv_steps.notify_all();
  }
}

}  // namespace

extern "C" {

void composite_default_server_opts(cmp_server_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->hbm_budget_bytes = int64_t(16) << 30;
  o->max_sessions = 1024;
  o->max_batch = 64;
  o->max_view_pixels = 1 << 20;
  // measured on the served workload (256 sessions of 4096x4096): one
  // workgroup per 256-vector item takes 0.082 ms of device time per request
  // (persistent, 2 per CU: 0.086 ms; 1024-vector items: 0.087 ms); steps of
  // rebuilds run persistent (automatic choice, blocks_per_cu 0)
  o->tile_vecs = 256;
  o->blocks_per_cu = 0;
  o->overlap = 1;
  o->remat_max_members = 2048;
  o->count_bits = 32;
  o->oversubscribe_pct = 0;
  o->max_queue = 1024;
  o->view_group = 0;
}

int composite_server_create(cmp_server **out, cmp_pool *pool, const cmp_server_opts *opts) {
  if (!out) return CMP_EINVAL;
  *out = nullptr;
  if (!pool) return CMP_EINVAL;
  cmp_server_opts o;
  composite_default_server_opts(&o);
  if (opts) o = *opts;
  for (int r : o.reserved)
    if (r) return CMP_EINVAL;
  if (o.max_batch < 1 || o.max_batch > 4096 || o.max_sessions < 1 || o.max_view_pixels < 1 ||
      o.tile_vecs < 64 || o.tile_vecs > 65536 || o.blocks_per_cu < 0 || o.blocks_per_cu > 16 ||
      (o.overlap != 0 && o.overlap != 1) || o.remat_max_members < 0 || o.remat_max_members > 65535 ||
      (o.count_bits != 16 && o.count_bits != 32) || o.oversubscribe_pct < 0 || o.max_queue < 1 ||
      o.view_group < 0 || o.view_group > 64 ||
      o.hbm_budget_bytes < 1)
    return CMP_EINVAL;
  if (pool->W % 16) return CMP_EUNSUPPORTED;
  {
    // a step's work items (max_batch sessions of row blocks) are counted in int32
    const int64_t rows = std::max<int64_t>(1, o.tile_vecs / (pool->W / 16));
    if ((int64_t)o.max_batch * ((pool->H + rows - 1) / rows) >= (int64_t(1) << 31)) return CMP_EUNSUPPORTED;
  }
  const int64_t comp_bytes = (int64_t)pool->W * pool->H * (o.count_bits / 8);
  // a step must fit in the slab: at least max_batch resident composites
  if (o.hbm_budget_bytes / comp_bytes < o.max_batch) return CMP_EINVAL;
  cmp_server *s = new (std::nothrow) cmp_server();
  if (!s) return CMP_ENOMEM;
  s->pool = pool;
  s->o = o;
  s->dev = pool->dev;
  s->W = pool->W;
  s->H = pool->H;
  s->comp_bytes = comp_bytes;
  const int64_t nslots = std::min<int64_t>(o.hbm_budget_bytes / comp_bytes, o.max_sessions);
  // admission: the sessions the slab holds resident, plus oversubscribe_pct
  // percent of them that live by eviction
  s->admit_limit = std::min<int64_t>(o.max_sessions, nslots + nslots * (int64_t)o.oversubscribe_pct / 100);
  int rc = CMP_EDEVICE;
  do {
    if (hipSetDevice(s->dev) != hipSuccess) break;
    if (hipStreamCreateWithFlags(&s->comp, hipStreamNonBlocking) != hipSuccess) break;
    if (hipStreamCreateWithFlags(&s->rest, hipStreamNonBlocking) != hipSuccess) break;
    bool ok = true;
    for (int i = 0; i < 2 && ok; ++i)
      ok = hipEventCreate(&s->ev_k0[i]) == hipSuccess && hipEventCreate(&s->ev_rest[i]) == hipSuccess &&
           hipEventCreateWithFlags(&s->ev_pre[i], hipEventDisableTiming) == hipSuccess &&
           hipEventCreate(&s->ev_view[i]) == hipSuccess;
    if (!ok) break;
    rc = CMP_ENOMEM;
    if (hipMalloc((void **)&s->slab, nslots * comp_bytes) != hipSuccess) break;
    s->slot_owner.assign(nslots, -1);
    if (hipMalloc((void **)&s->d_queue, 64) != hipSuccess) break;
    // ids per request are capped at 65535 by submit; a rebuilt composite
    // takes at most remat_max_members more (its working set before the request)
    s->arena_cap = (int64_t)sizeof(SReq) * o.max_batch + 64 +
                   4 * (int64_t)o.max_batch * (65535 + (int64_t)o.remat_max_members);
    for (int i = 0; i < 2 && rc == CMP_ENOMEM; ++i) {
      if (hipHostMalloc((void **)&s->h_arena[i], s->arena_cap, hipHostMallocDefault) != hipSuccess ||
          hipMalloc((void **)&s->d_arena[i], s->arena_cap) != hipSuccess) {
        rc = -100;  // marker: allocation failed
      }
    }
    if (rc == -100) {
      rc = CMP_ENOMEM;
      break;
    }
    rc = CMP_EDEVICE;
    if (hipEventCreate(&s->ev_ref) != hipSuccess || hipEventRecord(s->ev_ref, s->comp) != hipSuccess ||
        hipEventSynchronize(s->ev_ref) != hipSuccess)
      break;
    // The viewport launch of a split step is mostly waiting for its PCIe
    // writes; LDS it does not use caps it at two workgroups per compute unit,
    // so that the other rows' launch runs beside it (on the served workload:
    // 0.077 instead of 0.090 ms of device time per request, for 5 us more of
    // viewport launch).  No cap if the limits cannot be read.
    {
      int lds_cu = 0, lds_block = 0;
      hipFuncAttributes fa{};
      const void *kf = o.count_bits == 16 ? reinterpret_cast<const void *>(&k_serve<true, ArgStep>)
                                          : reinterpret_cast<const void *>(&k_serve<false, ArgStep>);
      if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, s->dev) ==
              hipSuccess &&
          hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, s->dev) == hipSuccess &&
          hipFuncGetAttributes(&fa, kf) == hipSuccess) {
        const int64_t want = (int64_t)lds_cu / 3 + 1024 - (int64_t)fa.sharedSizeBytes;
        s->view_lds = (size_t)std::max<int64_t>(0, std::min<int64_t>(want, lds_block - (int64_t)fa.sharedSizeBytes));
      } else {
        (void)hipGetLastError();
      }
    }
    s->st.resident_slots = nslots;
    rc = CMP_OK;
  } while (false);
  if (rc != CMP_OK) {
    composite_server_free(s);
    return rc;
  }
  s->worker = std::thread(worker_loop, s);
  s->completer = std::thread(completer_loop, s);
  *out = s;
  return CMP_OK;
}

void composite_server_free(cmp_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_queue.notify_all();
  s->cv_steps.notify_all();
  // the worker drains the queue and exits; the completer then drains the
  // launched steps and exits
  if (s->worker.joinable()) s->worker.join();
  else s->worker_done = true;
  s->cv_steps.notify_all();
  if (s->completer.joinable()) s->completer.join();
  (void)hipSetDevice(s->dev);
  if (s->comp) (void)hipStreamSynchronize(s->comp);
  if (s->rest) (void)hipStreamSynchronize(s->rest);
  for (auto &kv : s->sessions)
    if (kv.second.spill) (void)hipHostFree(kv.second.spill);
  (void)hipFree(s->slab);
  (void)hipFree(s->d_queue);
  for (int i = 0; i < 2; ++i) {
    if (s->h_arena[i]) (void)hipHostFree(s->h_arena[i]);
    (void)hipFree(s->d_arena[i]);
    if (s->ev_k0[i]) (void)hipEventDestroy(s->ev_k0[i]);
    if (s->ev_rest[i]) (void)hipEventDestroy(s->ev_rest[i]);
    if (s->ev_pre[i]) (void)hipEventDestroy(s->ev_pre[i]);
    if (s->ev_view[i]) (void)hipEventDestroy(s->ev_view[i]);
  }
  if (s->ev_ref) (void)hipEventDestroy(s->ev_ref);
  if (s->comp) (void)hipStreamDestroy(s->comp);
  if (s->rest) (void)hipStreamDestroy(s->rest);
  delete s;
}

int composite_session_open(cmp_server *s, int64_t *sid_out) {
  if (!s || !sid_out) return CMP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->failed != CMP_OK) return s->failed;
  if (s->open_sessions >= s->admit_limit) {
    // refused by the HBM budget (or max_sessions); nothing else changes
    s->st.refused_sessions += 1;
    return CMP_ENOMEM;
  }
  const int64_t sid = s->next_sid++;
  Session &ss = s->sessions[sid];
  ss.open = true;
  s->open_sessions += 1;
  *sid_out = sid;
  return CMP_OK;
}

int composite_session_close(cmp_server *s, int64_t sid) {
  if (!s) return CMP_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->sessions.find(sid);
  if (it == s->sessions.end() || !it->second.open) return CMP_EINVAL;
  if (it->second.inflight > 0) return CMP_EBUSY;
  // the slot is released; the worker never touches it again for this id
  if (it->second.slot >= 0) s->slot_owner[it->second.slot] = -1;
  uint8_t *spill = it->second.spill;
  s->sessions.erase(it);
  s->open_sessions -= 1;
  lk.unlock();
  if (spill) {
    // a spill copy into it may still be queued on the compute stream: free it
    // only once that stream has drained; if it cannot be drained the buffer
    // is left allocated (a copy may still write it) and the server fails
    if (hipSetDevice(s->dev) != hipSuccess || hipStreamSynchronize(s->comp) != hipSuccess) {
      fail(s, CMP_EDEVICE);
      return CMP_EDEVICE;
    }
    (void)hipHostFree(spill);
  }
  return CMP_OK;
}

int composite_session_submit(cmp_server *s, int64_t sid, int32_t op, const int32_t *ids, int32_t n,
                             int32_t vx0, int32_t vy0, int32_t vw, int32_t vh, void *dst,
                             int64_t dst_pitch, uint64_t *ticket) {
  if (!s || !ticket) return CMP_EINVAL;
  if (op != CMP_OP_ADD && op != CMP_OP_REMOVE) return CMP_EINVAL;
  if (n < 0 || n > 65535 || (n > 0 && !ids)) return CMP_EINVAL;
  if (vw < 1 || vh < 1 || vx0 < 0 || vy0 < 0 || (int64_t)vx0 + vw > s->W || (int64_t)vy0 + vh > s->H)
    return CMP_EINVAL;
  if ((int64_t)vw * vh > s->o.max_view_pixels || !dst || dst_pitch < vw || dst_pitch > INT32_MAX)
    return CMP_EINVAL;
  for (int32_t i = 0; i < n; ++i)
    if (ids[i] < 0 || ids[i] >= s->pool->count) return CMP_EINVAL;
  // the kernel writes the viewport into dst: it must be page-locked host
  // memory (which has a device address) aligned to a count
  if (reinterpret_cast<uintptr_t>(dst) % (uintptr_t)(s->o.count_bits / 8)) return CMP_EINVAL;
  // (the attributes may describe the allocation dst lies in: its device
  // address is the allocation's plus dst's offset from the allocation's host
  // address)
  hipPointerAttribute_t pa{};
  if (hipPointerGetAttributes(&pa, dst) != hipSuccess) {
    (void)hipGetLastError();  // leave no error behind for the caller's next HIP call
    return CMP_EINVAL;
  }
  if (pa.type != hipMemoryTypeHost || !pa.devicePointer || !pa.hostPointer ||
      reinterpret_cast<uintptr_t>(pa.hostPointer) > reinterpret_cast<uintptr_t>(dst))
    return CMP_EINVAL;
  void *dview = static_cast<char *>(pa.devicePointer) +
                (reinterpret_cast<uintptr_t>(dst) - reinterpret_cast<uintptr_t>(pa.hostPointer));
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->failed != CMP_OK) return s->failed;
  if (s->stop) return CMP_EINVAL;
  auto it = s->sessions.find(sid);
  if (it == s->sessions.end() || !it->second.open) return CMP_EINVAL;
  Session &ss = it->second;
  // every refusal below leaves the server as it was
  if ((int64_t)s->queue.size() >= s->o.max_queue) {
    s->st.refused_busy += 1;
    return CMP_EBUSY;
  }
  if (op == CMP_OP_REMOVE) {
    std::unordered_map<int32_t, int64_t> need;
    for (int32_t i = 0; i < n; ++i) need[ids[i]] += 1;
    for (auto &kv : need) {
      auto h = ss.projected.find(kv.first);
      if (h == ss.projected.end() || h->second < kv.second) return CMP_ENOTMEMBER;
    }
    for (auto &kv : need)
      if ((ss.projected[kv.first] -= kv.second) == 0) ss.projected.erase(kv.first);
    ss.projected_n -= n;
  } else {
    // a uint16 composite holds counts up to 65535 (a uint32 one 2^32 - 1,
    // beyond what a pool can be asked for here)
    const int64_t cap = s->o.count_bits == 16 ? 65535 : (int64_t(1) << 32) - 1;
    if (ss.projected_n + n > cap) return CMP_ERANGE;
    for (int32_t i = 0; i < n; ++i) ss.projected[ids[i]] += 1;
    ss.projected_n += n;
  }
  Request r;
  r.ticket = s->next_ticket++;
  r.sid = sid;
  r.op = op;
  r.ids.assign(ids, ids + n);
  r.vx0 = vx0;
  r.vy0 = vy0;
  r.vw = vw;
  r.vh = vh;
  r.dst = dst;
  r.dview = dview;
  r.pitch = dst_pitch;
  r.t_submit = now_ns();
  ss.inflight += 1;
  s->done[r.ticket] = Done{r.t_submit, 0};
  s->pending.insert(r.ticket);
  *ticket = r.ticket;
  s->queue.push_back(std::move(r));
  s->st.queue_peak = std::max<int64_t>(s->st.queue_peak, (int64_t)s->queue.size());
  s->cv_queue.notify_one();
  return CMP_OK;
}

int composite_server_pause(cmp_server *s, int32_t paused) {
  if (!s || (paused != 0 && paused != 1)) return CMP_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed != CMP_OK) return s->failed;
    s->paused = paused != 0;
  }
  s->cv_queue.notify_all();
  return CMP_OK;
}

int composite_session_wait(cmp_server *s, uint64_t ticket, int64_t timeout_us, int64_t *t_submit_ns,
                           int64_t *t_done_ns) {
  if (!s) return CMP_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->done.find(ticket);
  if (it == s->done.end()) return CMP_EINVAL;
  auto ready = [&] { return !s->pending.count(ticket) || s->failed != CMP_OK; };
  if (timeout_us < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return CMP_ETIMEDOUT;
  }
  if (s->pending.count(ticket)) return s->failed;
  if (t_submit_ns) *t_submit_ns = it->second.t_submit;
  if (t_done_ns) *t_done_ns = it->second.t_done;
  return CMP_OK;
}

int composite_server_stats(cmp_server *s, cmp_server_stats *st) {
  if (!s || !st) return CMP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *st = s->st;
  return CMP_OK;
}

int composite_server_replay(cmp_server *s, const cmp_replay_req *reqs, int64_t nreq, const int32_t *ids,
                            void *const *dst_ring, int32_t ring, int64_t dst_pitch,
                            int64_t *latency_ns, int32_t *status) {
  if (!s || nreq < 0 || (nreq > 0 && (!reqs || !dst_ring || ring < 1 || !latency_ns))) return CMP_EINVAL;
  std::vector<uint64_t> tickets(nreq, 0);
  std::vector<int64_t> arrival(nreq, 0);
  std::vector<int32_t> st(nreq, CMP_OK);
  const int64_t t0 = now_ns();
  int rc = CMP_OK;
  int64_t last = nreq;  // requests [last, nreq) were never submitted
  for (int64_t i = 0; i < nreq; ++i) {
    const cmp_replay_req &q = reqs[i];
    const int64_t target = t0 + q.t_ns;
    for (;;) {
      const int64_t d = target - now_ns();
      if (d <= 0) break;
      if (d > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(d - 100000));
      else std::this_thread::yield();
    }
    arrival[i] = target;
    const int r = composite_session_submit(s, q.sid, q.op, q.n ? ids + q.ids_off : nullptr, q.n, q.vx0,
                                           q.vy0, q.vw, q.vh, dst_ring[i % ring], dst_pitch, &tickets[i]);
    st[i] = r;
    if (r == CMP_OK) continue;
    // a refusal (full queue; a remove of ids that only a refused add would have
    // brought; a uint16 session at its limit) is recorded and the replay goes
    // on; any other failure ends it
    if (status && (r == CMP_EBUSY || r == CMP_ENOTMEMBER || r == CMP_ERANGE)) continue;
    rc = r;
    last = i + 1;
    break;
  }
  for (int64_t i = 0; i < last; ++i) {
    latency_ns[i] = -1;
    if (st[i] != CMP_OK) continue;
    int64_t ts = 0, td = 0;
    const int w = composite_session_wait(s, tickets[i], -1, &ts, &td);
    if (w != CMP_OK) {
      if (rc == CMP_OK) rc = w;
      st[i] = w;
      continue;
    }
    latency_ns[i] = td - arrival[i];
  }
  for (int64_t i = last; i < nreq; ++i) {
    latency_ns[i] = -1;
    st[i] = CMP_ECANCELED;
  }
  if (status) std::copy(st.begin(), st.end(), status);
  return rc;
}

}  // extern "C"
