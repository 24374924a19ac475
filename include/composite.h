/* composite.h -- C ABI of libcomposite.so: ensemble compositing of uint8
 * rasters on an AMD Instinct MI355X (gfx950).
 *
 * The operation (Johnson & Jankun-Kelly, arXiv 2104.14667): N input surfaces
 * are combined into one composite image whose value grows with their overlap,
 * and the user adds surfaces to, and removes them from, the working set in
 * real time (Section 2 and the caption of Figure 1).  The composite is built
 * iteratively: accumulators are cleared, then each input is uploaded and folded
 * in by an accumulation kernel (Section 4, the single- and dual-buffer
 * listings, Figures 2 and 3); with two staging buffers the upload of one input
 * overlaps the processing of the previous one (Section 4, Figure 4).
 *
 * Per pixel p, over the current multiset M of members m (W x H uint8 rasters,
 * row-major, pitch W):
 *     count[p] = #{m in M : m[p] != 0}          (uint16 or uint32)
 *     sum[p]   = sum of m[p] over M               (uint32)
 *     max[p]   = max({0} U {m[p] : m in M})       (uint8)
 * Results are exact; a call that could make a stored value overflow is refused
 * with CMP_ERANGE before anything is enqueued.
 *
 * Conventions for every function below:
 *   - The return value is CMP_OK (0) or a negative cmp_status.  No function
 *     aborts, throws, or prints.
 *   - Every argument is validated before any work is enqueued; on an error
 *     return the context is unchanged.
 *   - A HIP runtime failure returns CMP_EDEVICE and poisons the context: every
 *     later call on it returns CMP_EDEVICE, except composite_free.
 *   - The caller owns all input rasters and output buffers.  The library owns
 *     the device composite, its staging buffers, streams and events.
 *   - A context is used by one host thread at a time; distinct contexts are
 *     independent.
 */
#ifndef COMPOSITE_H
#define COMPOSITE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum cmp_status {
  CMP_OK = 0,
  CMP_EINVAL = -1,       /* bad argument: null pointer, size, window, flag   */
  CMP_ENOMEM = -2,       /* device or pinned host allocation failed          */
  CMP_ERANGE = -3,       /* the call could overflow a stored composite value */
  CMP_ENOTMEMBER = -4,   /* remove of an id the working set does not hold    */
  CMP_EUNSUPPORTED = -5, /* valid request this configuration cannot serve    */
  CMP_EDEVICE = -6,      /* no usable GPU, or a HIP call failed (poisoned)   */
  CMP_EBUSY = -7,        /* resource is in use, or a queue is full           */
  CMP_ETIMEDOUT = -8,    /* a bounded wait expired                           */
  CMP_ECANCELED = -9     /* not attempted: an earlier failure ended the call */
};

/* Output selection bits (composite_init `outputs`, composite_read `which`). */
enum cmp_outputs { CMP_COUNT = 1, CMP_SUM = 2, CMP_MAX = 4 };

/* Kind of memory composite_read writes to.  CMP_DST_HOST: any host memory;
 * the data passes through pinned buffers of the library.  CMP_DST_PINNED:
 * page-locked host memory the copy engine writes directly.  CMP_DST_DEVICE:
 * device memory, written by a kernel. */
enum cmp_dst_kind { CMP_DST_HOST = 0, CMP_DST_DEVICE = 1, CMP_DST_PINNED = 2 };

/* Layout of staged members on the device.  CMP_LINEAR reads the staged
 * rasters row-major as uploaded (the paper's buffers).  CMP_TILED first
 * repacks each staged raster into tiles of tile_w bytes x tile_h rows, stored
 * tile after tile, and composites from the tiled copy (the counterpart of the
 * paper's buffer-to-image transform and image reads, Section 4, third
 * implementation method).  Results are identical. */
enum cmp_layout { CMP_LINEAR = 0, CMP_TILED = 1 };
/* In a CMP_TILED context, rasters given in device memory (composite_add_device,
 * composite_remove with maps_on_device) are already in the tiled layout, as
 * composite_repack_tiled writes them (composite_tiled_bytes bytes each): the
 * counterpart of the paper's images kept on the device.  Host rasters are
 * always row-major and are repacked on the device after upload. */

typedef struct cmp_opts {
  int32_t nbuf;           /* staging slots for composite_add: 1 or 2.  1 is the
                             single-buffer control (upload and compositing
                             alternate), 2 the dual-buffer pipeline.  Default 2 */
  int32_t chunk_depth;    /* members uploaded per staging slot, 1..256.
                             Default 8 */
  int32_t layout;         /* cmp_layout.  Default CMP_LINEAR */
  int32_t tile_w;         /* CMP_TILED tile width in bytes: 16, 32, 64 or 128.
                             Default 64 */
  int32_t tile_h;         /* CMP_TILED tile height in rows, 1..256.  Default 64 */
  int32_t device;         /* HIP device ordinal.  Default 0 */
  void *copy_stream;      /* hipStream_t for uploads, or NULL: the library
                             creates a default-priority stream */
  void *compute_stream;   /* hipStream_t for kernels, or NULL (as above) */
  void *(*dev_alloc)(size_t bytes, void *alloc_ctx);
                          /* device allocator for the context's composite,
                             staging, tables and scratch (for instance a
                             framework's caching allocator), or NULL for
                             hipMalloc.  It must return memory of the context's
                             device, 256-byte aligned, or NULL (then the call
                             that needed it returns CMP_ENOMEM).  Given with
                             dev_free or not at all.  Default NULL */
  void (*dev_free)(void *ptr, void *alloc_ctx);
                          /* frees what dev_alloc returned; the library calls
                             it only once its streams no longer use the memory.
                             Default NULL */
  void *alloc_ctx;        /* passed to both hooks.  Default NULL */
  int32_t retain_members; /* 1: remember the device pointer of every member
                             added with composite_add_device, so a remove can
                             recompute max.  The caller keeps those rasters
                             alive while they are members.  Default 0 */
  int32_t debug_poison;   /* 1: fill each staging slot with 0xA5 once the
                             kernel that read it is done (hazard testing).
                             Default 0 */
  int32_t profile;        /* 1: time every compositing kernel with HIP events
                             on the compute stream (composite_kernel_stats).
                             Default 0 */
  int32_t pageable_host;  /* 0: host rasters given to composite_add/remove are
                             page-locked (hipHostMalloc, torch pin_memory) and
                             the copy engine reads them directly.  1: they may
                             be ordinary pageable memory; the host first copies
                             each chunk into a pinned bounce buffer of the
                             library (one per staging slot).  Default 0 */
  int32_t host_paced;     /* 0: the copy stream waits on the event of the
                             kernel that last read a slot: ordering by events
                             only, no host synchronisation inside the loop
                             (Section 4, Figure 4).  1: the host waits for that
                             kernel before queueing the slot's next upload
                             (the previous chunk's upload is still in flight
                             then).  Default 0 */
  int32_t verify_members; /* 1: keep a 64-bit fingerprint of every member with
                             its id, so that composite_remove can refuse a
                             raster that is not one that was added under that
                             id (CMP_EINVAL, nothing changed).  The fingerprint
                             is sum_j d_j * w_j mod 2^64 over the raster's
                             little-endian 32-bit words d_j (the last one
                             zero-padded), with w_j = lowbias32(j) | 1
                             (Wellons' integer hash: x ^= x >> 16;
                             x *= 0x7feb352d; x ^= x >> 15; x *= 0x846ca68b;
                             x ^= x >> 16).  Costs one more device read of
                             every added raster, makes add and remove wait for
                             their kernels, and a remove of host rasters
                             uploads them twice.  In a CMP_TILED context the
                             fingerprint is taken over the tiled layout's bytes.
                             Default 0 */
  int32_t pingpong;       /* 1: two accumulators per output, used in turn: each
                             compositing launch reads the current one and writes
                             the other (the paper's image kernels and its
                             buffer-kernel 2, Section 5.3); 0: one accumulator
                             updated in place (its buffer-kernel 1).  Results
                             are identical; pingpong doubles the composite's
                             device memory.  Default 0 */
  int32_t copy_streams;   /* streams the uploads of composite_add/remove run on:
                             0 or 1, the copy stream; 2 (with nbuf = 2), slot
                             k's uploads on a stream of their own, so that one
                             slot's upload can start while the other's is still
                             running and the copy engines are not idle between
                             chunks (the second stream is created by the
                             library).  Ordering per slot is unchanged: each
                             upload waits for the kernel that last read its
                             slot.  Default 0 */
} cmp_opts;

typedef struct cmp_ctx cmp_ctx;

/* Fills *opts with the defaults above.  NULL is ignored. */
void composite_default_opts(cmp_opts *opts);

/* Creates a context holding a cleared W x H composite on the device.
 * outputs: non-empty OR of cmp_outputs.  count_bits: 16 or 32 (ignored
 * without CMP_COUNT).  opts: NULL for defaults.  W, H >= 1 and
 * W*H <= 2^32 - 16 (larger rasters are split spatially by the caller).
 * Returns CMP_EDEVICE when no GPU is usable, CMP_ENOMEM when the composite
 * does not fit.  On success *out owns the context (composite_free). */
int composite_init(cmp_ctx **out, int32_t W, int32_t H, uint32_t outputs,
                   int32_t count_bits, const cmp_opts *opts);

/* Clears the composite and forgets every member (both listings, step 1). */
int composite_clear(cmp_ctx *ctx);

/* Streams n members from host memory into the composite.
 * host_maps[i]: W*H bytes, row-major, page-locked unless opts.pageable_host
 * is set (then the host first copies each chunk into a pinned bounce buffer,
 * the counterpart of the paper's first implementation method, Section 4).
 * Members are uploaded in chunks of
 * chunk_depth into nbuf staging slots on the copy stream; the compute stream
 * waits for each chunk's upload and the copy stream waits for a slot to be
 * released by the kernel that read it, so no host synchronisation happens
 * inside the loop.  ids: NULL, or n ids recorded in the member registry
 * (needed to remove by id).  Returns when the library no longer reads
 * host_maps; compositing may still run (composite_sync / composite_read wait
 * for it).  n == 0 is a no-op. */
int composite_add(cmp_ctx *ctx, const uint8_t *const *host_maps,
                  const int64_t *ids, int32_t n);

/* Composites n members that are already in device memory (one kernel pass over
 * all of them, no staging): the accumulation kernel step of the paper's two
 * listings (Section 4) with the load from client memory left out, as for data
 * already resident on the device.  dev_maps[i]: device pointers to W*H bytes, any
 * alignment (in a CMP_TILED context: to the tiled layout, see cmp_layout).  The rasters must stay valid until composite_sync returns, and,
 * with retain_members, for as long as they are members.  Returns without
 * waiting for the device. */
int composite_add_device(cmp_ctx *ctx, const uint8_t *const *dev_maps,
                         const int64_t *ids, int32_t n);

/* Removes n members, the counterpart of adding one: surfaces are added and
 * removed in real time and the composite follows (Figure 1 and its caption;
 * the paper names no mechanism).  Count and sum are decremented exactly; max, when
 * selected, is recomputed from the retained members (retain_members = 1 and
 * every member added with composite_add_device), else CMP_EUNSUPPORTED.
 * maps: the rasters removed (host memory if maps_on_device == 0, else device
 * memory), or NULL with retain_members = 1 and ids given: the retained rasters
 * of those ids are used.  ids: NULL, or n ids; an id the registry does not
 * hold (counting multiplicity) gives CMP_ENOTMEMBER.  Without ids the caller
 * vouches that the rasters are members, unless the context verifies members
 * (cmp_opts.verify_members): then a raster whose fingerprint is not held
 * under its id (or among the members added without ids) gives CMP_EINVAL. */
int composite_remove(cmp_ctx *ctx, const uint8_t *const *maps,
                     const int64_t *ids, int32_t n, int32_t maps_on_device);

/* Copies the window [x0, x0+w) x [y0, y0+h) of one output (`which` is exactly
 * one of CMP_COUNT, CMP_SUM, CMP_MAX and must have been selected at init) to
 * dst, row by row with dst_pitch_bytes between rows (>= w * element size:
 * 2 or 4 bytes for count, 4 for sum, 1 for max).  dst_kind (cmp_dst_kind)
 * says what memory dst is.  Waits for all work enqueued on the context before
 * it and returns when dst holds the data.  The result is the composite of the
 * members, restricted to the window (the retrieval of results, Section 1). */
int composite_read(cmp_ctx *ctx, uint32_t which, int32_t x0, int32_t y0,
                   int32_t w, int32_t h, void *dst, int64_t dst_pitch_bytes,
                   int32_t dst_kind);

/* Waits for all work enqueued on the context: the end of the listings'
 * loop (Section 4), after which the accumulators hold the composite of every
 * member (the point where the paper's timing stops, Section 5.1). */
int composite_sync(cmp_ctx *ctx);

/* Number of members currently composited (with multiplicity): the N of the
 * composite, i.e. the length of the list of selected surfaces (Figure 1). */
int composite_members(const cmp_ctx *ctx, int64_t *n_out);

/* Device address of one output of the composite (row-major, pitch W elements),
 * valid until composite_free.  For zero-copy consumers; the caller orders its
 * own accesses after composite_sync. */
int composite_device_buffer(cmp_ctx *ctx, uint32_t which, void **dev_ptr);

/* With opts.profile = 1: number of compositing kernel launches and their
 * summed duration in milliseconds (HIP events around each launch on the
 * compute stream) since init or the last reset (reset != 0 clears them after
 * reading).  Synchronises the context. */
int composite_kernel_stats(cmp_ctx *ctx, int64_t *launches, double *total_ms,
                           int32_t reset);

/* ------------------------------------------------------------------------
 * Batched requests against a device-resident pool of rasters.
 *
 * A request asks for the member count composite of a subset of the pool,
 * restricted to a crop window: the paper's compositing of a chosen set of
 * surfaces (Figure 1) applied to a spatial segment (Section 1, spatial
 * subdivision).  Many requests of uneven set sizes and windows are served by
 * one persistent launch whose workgroups pull (request, band of rows) work
 * items from a queue in device memory.
 */
typedef struct cmp_pool cmp_pool;

/* Wraps `count` rasters of W x H bytes already in device memory at
 * dev_base + i * stride_bytes (row-major, pitch W).  pool_bytes is the size
 * of the allocation that starts at dev_base; it must extend at least 16
 * bytes past the end of the last raster (the kernels read whole 16-byte
 * vectors and may touch up to 15 bytes past a window's right edge).  The
 * caller keeps the memory alive until composite_pool_free.  The pool owns a
 * compute stream (default priority) and its descriptor buffers; one thread at
 * a time may call composite_batch_run on it (servers created on the pool only
 * read its rasters and may run concurrently). */
int composite_pool_create(cmp_pool **out, const uint8_t *dev_base, int64_t count, int32_t W,
                          int32_t H, int64_t stride_bytes, int64_t pool_bytes, int32_t device);

/* Waits for the pool's stream, then releases what the pool owns (not the
 * rasters).  NULL is ignored. */
void composite_pool_free(cmp_pool *pool);

typedef struct cmp_request {
  const int32_t *ids;     /* host array of n pool indices (repeats count twice) */
  int32_t n;              /* 0 .. 65535 */
  int32_t x0, y0, w, h;   /* crop window inside W x H, w, h >= 1 */
  uint32_t *dev_count;    /* device memory: h rows of w uint32 counts */
  int64_t out_pitch;      /* elements between output rows, >= w */
} cmp_request;

/* PERSISTENT: one persistent launch over (request, band of crop rows) work
 * items; every item reads its request's members.  PER_REQUEST: one plain
 * launch per request, in order (the baseline).  SHARED: one persistent
 * launch over tiles of 1024 pixels of a raster row; a tile reads each pool
 * member that any request covering it holds once, and adds it to every such
 * request (accumulators in LDS, up to 32 requests per pass over a tile).  It
 * needs distinct ids within each request and a pool of at most 65536
 * rasters whose member masks fit in LDS; a batch that does not qualify runs
 * in the PERSISTENT mode with the same parameters (composite_batch_last
 * reports which mode ran).  MATRIX: one persistent launch over (block of 64
 * requests, tile of 512 pixels of a raster row); the counts of a tile for
 * all 64 requests are an int8 matrix-core product of the members' nonzero
 * flags with the requests' membership, so a tile reads each pool member that
 * a covering request holds once, with no limit on the covering requests per
 * pass.  It needs distinct ids within each request, a pool of at most 8192
 * rasters and 31 * stride + W + 8 < 2^32; a batch that does not qualify runs
 * in the SHARED mode (and from there maybe PERSISTENT) with the same
 * parameters. */
enum cmp_batch_mode {
  CMP_BATCH_PERSISTENT = 0,
  CMP_BATCH_PER_REQUEST = 1,
  CMP_BATCH_SHARED = 2,
  CMP_BATCH_MATRIX = 3
};

/* Order of the work queue.  COST: largest items first.  ROWS: by the first
 * raster row an item reads, so that concurrently running items of different
 * requests read the same rows of the members they share while those rows are
 * still in the L2 / Infinity Cache. */
enum cmp_batch_order { CMP_ORDER_COST = 0, CMP_ORDER_ROWS = 1 };

typedef struct cmp_tune {
  int32_t mode;           /* cmp_batch_mode.  PER_REQUEST launches one plain
                             kernel per request, in order (the baseline) */
  int32_t tile_vecs;      /* persistent mode: 16-pixel vectors per work item
                             (a band of whole crop rows), 64 .. 65536; checked
                             in the shared mode too (its fallback) */
  int32_t blocks_per_cu;  /* persistent, shared and matrix modes: workgroups
                             per compute unit, 1 .. 16 (the matrix mode uses
                             at most 2, all it fits at once) */
  int32_t use_graph;      /* persistent and shared modes: 1 replays a captured
                             hipGraph of [queue reset, kernel]; captured once
                             per mode, grid size and load kind, and reused */
  int32_t order;          /* persistent mode: cmp_batch_order */
  int32_t stream_loads;   /* 1: member loads carry the non-temporal hint
                             (nothing is re-read); 0: plain loads, so rows
                             shared by requests can hit in the caches */
  int32_t slots;          /* shared mode: requests per pass over a tile, 4 .. 32,
                             or 0 for as many as LDS holds.  Fewer slots use
                             less LDS (more workgroups per compute unit) but
                             need more passes where many requests overlap */
  int32_t reserved[1];    /* must be zero */
} cmp_tune;

/* Fills *t with the defaults (matrix, tile_vecs 1024, blocks_per_cu 4,
 * use_graph 1, order ROWS, stream_loads 1, slots 24).  NULL is ignored. */
void composite_default_tune(cmp_tune *t);

/* Runs nreq requests and returns when every output is written.  Every
 * request is validated first (ids < pool count, window inside the raster,
 * dev_count non-NULL, out_pitch >= w); nothing is launched on error.
 * tune: NULL for the defaults. */
int composite_batch_run(cmp_pool *pool, const cmp_request *reqs, int32_t nreq,
                        const cmp_tune *tune);

/* Device time in milliseconds of the last composite_batch_run, measured with
 * HIP events around its launches on the pool's stream (descriptor upload
 * excluded), the number of work items it ran (tiles in the shared mode), and
 * (mode: NULL or a cmp_batch_mode out) the mode that ran. */
int composite_batch_last(const cmp_pool *pool, double *ms, int64_t *items, int32_t *mode);

/* ------------------------------------------------------------------------
 * Served sessions: interactive add/remove against per-session composites.
 *
 * Each session is one user's working set (Figure 1: surfaces are added and
 * removed in real time, and the composite follows) over the rasters of a
 * pool, with its own device-resident uint32 count composite of the pool's
 * W x H (uint32, or uint16 with count_bits = 16).  A request adds or removes
 * pool members and asks for a viewport of the updated composite; the viewport
 * is returned in the composite's width (uint16 counts with count_bits = 16,
 * uint32 with 32).  One server thread batches continuously: every step takes
 * the oldest queued request of each session (at most max_batch) and updates
 * all their composites, the kernel writing each viewport straight into the
 * caller's page-locked memory: the rows holding viewports in a first launch,
 * after which the step's requests are complete, and the other rows in a
 * second beside it (one launch when a full step's worth of requests already
 * waits).  Requests of one session are applied in submission order; sessions
 * interleave.  Session
 * composites live in a device slab of hbm_budget_bytes; when a request needs
 * a session that is not resident and the slab is full, a session that is not
 * part of the step is evicted: the one with the lowest GreedyDual priority
 * (Young 1994; Cao and Irani 1997), which is the priority of the last evicted
 * session at its last use plus the cost of bringing it back, so cheap
 * sessions go first and the policy is LRU when costs are equal.  An evicted
 * composite is dropped and later rebuilt from the session's members (the
 * cost: its member count) or copied to pinned host memory and back (the
 * cost: remat_max_members), see cmp_server_opts.remat_max_members.
 *
 * Admission and backpressure.  The budget holds hbm_budget_bytes / (W*H*
 * count_bits/8) composites resident (the slots).  composite_session_open
 * admits a session only while the open sessions number fewer than the slots
 * plus oversubscribe_pct percent of them (and fewer than max_sessions), and
 * refuses with CMP_ENOMEM otherwise: with the default oversubscribe_pct = 0
 * every admitted session keeps its composite resident and nothing is ever
 * evicted; above 0 the sessions beyond the slots live by eviction.
 * composite_session_submit refuses with CMP_EBUSY while max_queue requests
 * wait for a step, so a server that cannot keep up sheds load instead of
 * letting the queue, and the latency, grow without bound.  A refused call
 * changes nothing.
 */
typedef struct cmp_server cmp_server;

enum cmp_op { CMP_OP_ADD = 0, CMP_OP_REMOVE = 1 };

typedef struct cmp_server_opts {
  int64_t hbm_budget_bytes; /* device bytes for resident session composites;
                               at least one composite (W*H*4).  Default 16 GiB */
  int32_t max_sessions;     /* open sessions at most.  Default 1024 */
  int32_t max_batch;        /* requests per step, 1 .. 4096; 1 = unbatched FIFO.
                               Default 64 */
  int32_t max_view_pixels;  /* largest viewport w*h accepted.  Default 2^20 */
  int32_t tile_vecs;        /* 16-pixel vectors per work item.  Default 256 */
  int32_t blocks_per_cu;    /* persistent workgroups per compute unit, 1 .. 16, or 0
                               (automatic): one workgroup per work item (no
                               queue) for steps whose requests average at most
                               64 members, else 2 persistent per compute unit.
                               Default 0 */
  int32_t overlap;          /* 1: a step may be formed and launched while the
                               previous step is still on the device; 0: each
                               step completes before the next starts.
                               Default 1 */
  int32_t remat_max_members; /* eviction of a resident composite when a step
                               needs its slot: a session holding at most this
                               many members is dropped, and rebuilt by counting
                               its members in the resident pool when next used
                               (reads members * W*H bytes of HBM); a larger one
                               is copied to pinned host memory and back (2 *
                               W*H*4 bytes over PCIe).  0 copies all but empty
                               sessions; at most 65535.  Default 2048 */
  int32_t count_bits;       /* width of the session composites: 32, or 16
                               (half the HBM and half the read-modify-write
                               per request; a request that would take a
                               session past 65535 members is refused with
                               CMP_ERANGE).  Default 32 */
  int32_t oversubscribe_pct; /* sessions admitted beyond the resident slots,
                               in percent of the slots, >= 0.  Default 0 */
  int32_t max_queue;        /* requests waiting for a step at most, >= 1;
                               submit refuses beyond it (CMP_EBUSY).
                               Default 1024 */
  int32_t view_group;       /* row blocks (of tile_vecs vectors) per workgroup
                               of the launch that writes a step's viewports,
                               1 .. 64, or 0 (automatic: 1, the lowest
                               latency; larger groups trade latency for less
                               device time).  Default 0 */
  int32_t reserved[1];      /* must be zero */
} cmp_server_opts;

void composite_default_server_opts(cmp_server_opts *opts);

/* Creates a server over the rasters of `pool` (W must be a multiple of 16;
 * the pool must outlive the server).  Allocates the composite slab and the
 * staging buffers up front; the serving loop allocates only a session's
 * pinned spill buffer, on its first spill. */
int composite_server_create(cmp_server **out, cmp_pool *pool, const cmp_server_opts *opts);

/* Finishes every submitted request, stops the server and frees it.  NULL is
 * ignored. */
void composite_server_free(cmp_server *srv);

/* Opens a session with an empty working set (all-zero composite): the
 * interactive user of Figure 1, whose composite is kept on the device.
 * CMP_ENOMEM when the HBM budget admits no more sessions (see "Admission and
 * backpressure" above) or max_sessions are open; nothing changes then. */
int composite_session_open(cmp_server *srv, int64_t *sid_out);

/* Closes a session; CMP_EBUSY while it has unfinished requests.  CMP_EDEVICE
 * if the device fails while the session's spilled composite is released (the
 * session is closed and the server is failed). */
int composite_session_close(cmp_server *srv, int64_t sid);

/* Queues one request: op (cmp_op) of n pool ids, then the viewport
 * (vx0, vy0, vw, vh) of the session's count composite written to dst (host
 * memory allocated page-locked, vh rows of vw counts with dst_pitch elements
 * between rows; a count is a uint16 with count_bits = 16, else a uint32; the
 * update kernel writes it there directly).  CMP_EINVAL if dst is not
 * page-locked memory the device can address, or not aligned to a count.  The
 * request is validated against the session's working set as it will be after
 * all its earlier requests: removing an id it will not hold gives
 * CMP_ENOTMEMBER, and with count_bits = 16 an add that would take it past
 * 65535 members gives CMP_ERANGE.  CMP_EBUSY when max_queue requests are
 * waiting.  A refused request changes nothing.  Thread-safe; returns
 * without waiting: the real-time add and remove of surfaces of Figure 1.
 * *ticket identifies the request to composite_session_wait.  dst must stay
 * valid and untouched until the request completes. */
int composite_session_submit(cmp_server *srv, int64_t sid, int32_t op, const int32_t *ids,
                             int32_t n, int32_t vx0, int32_t vy0, int32_t vw, int32_t vh,
                             void *dst, int64_t dst_pitch, uint64_t *ticket);

/* Waits until the request is complete (its viewport is in dst) or timeout_us
 * passes (CMP_ETIMEDOUT; negative waits forever).  Optionally returns the
 * submit and completion times (CLOCK_MONOTONIC nanoseconds).  The server keeps
 * 16 bytes of timing per ticket until it is freed. */
int composite_session_wait(cmp_server *srv, uint64_t ticket, int64_t timeout_us,
                           int64_t *t_submit_ns, int64_t *t_done_ns);

typedef struct cmp_server_stats {
  int64_t requests, steps, max_step;
  int64_t spills, restores;  /* evictions copied to host memory, and copies back */
  int64_t resident_slots;
  double device_ms;          /* device time of the steps: each step's span from
                                its start to the end of its last launch,
                                overlaps between steps counted once */
  int64_t drops, rebuilds;   /* evictions without a copy, and composites
                                rebuilt from their members */
  int64_t refused_sessions;  /* session opens refused by admission */
  int64_t refused_busy;      /* submits refused because the queue was full */
  int64_t queue_peak;        /* most requests waiting for a step at once */
  /* Where the latency goes, summed over completed requests (divide by
   * `requests` for means): from submit until a step takes the request; from
   * then until the step's launches are enqueued (residency, descriptors,
   * launches); from then until its viewport is in host memory and the
   * completion is seen. */
  double wait_ms, host_ms, flight_ms;
  /* Device time summed over steps (divide by `steps`): from the step's start
   * until its viewports are in host memory (the end of the launch that writes
   * them). */
  double view_ms;
} cmp_server_stats;

/* Counters since the server was created. */
int composite_server_stats(cmp_server *srv, cmp_server_stats *st);

/* paused = 1: the server launches no new step (steps already launched
 * finish); submitted requests wait in the queue, up to max_queue.  paused = 0
 * resumes.  For maintenance windows and for tests of the queue bound.
 * composite_server_free still drains everything. */
int composite_server_pause(cmp_server *srv, int32_t paused);

/* One request of an open-loop replay: t_ns is its arrival time after the
 * replay starts; its ids are ids[ids_off .. ids_off + n). */
typedef struct cmp_replay_req {
  int64_t t_ns;
  int64_t sid;
  int64_t ids_off;
  int32_t op, n;
  int32_t vx0, vy0, vw, vh;
} cmp_replay_req;

/* Submits the requests at their arrival times from the calling thread (an
 * open-loop Poisson schedule does not wait for completions), then waits for
 * all of them.  Request i writes its viewport to dst_ring[i % ring] (pinned
 * host buffers of at least vh * dst_pitch counts of the composite's width).
 * latency_ns[i] = completion time - scheduled arrival time, or -1 for a
 * request that did not complete.
 * status: NULL, or nreq entries that receive each request's status.  With
 * status, a request refused by submit with CMP_EBUSY, CMP_ENOTMEMBER (it
 * removes ids that only a refused request would have added) or CMP_ERANGE is
 * recorded and the replay goes on; any other failure, and any refusal when
 * status is NULL, ends the replay (requests after it get CMP_ECANCELED).
 * Returns the first status that ended it, else CMP_OK. */
int composite_server_replay(cmp_server *srv, const cmp_replay_req *reqs, int64_t nreq,
                            const int32_t *ids, void *const *dst_ring, int32_t ring,
                            int64_t dst_pitch, int64_t *latency_ns, int32_t *status);

/* Histogram of overlap classes (Figure 1, lower-left panel: the frequency of
 * each overlap class of the composite): bins[k] = number of pixels whose count
 * is exactly k, for k = 0 .. nbins - 1, and *overflow = number of pixels with
 * count >= nbins.  Needs CMP_COUNT.  bins: host array of nbins int64;
 * 1 <= nbins <= 2^24.  Waits for work enqueued before it. */
int composite_histogram(cmp_ctx *ctx, int64_t *bins, int32_t nbins, int64_t *overflow);

/* Repacks n row-major W x H rasters (device memory, src + i * src_stride) into
 * the tiled layout of CMP_TILED (tiles of tile_w bytes x tile_h rows, stored
 * tile after tile; padding bytes of edge tiles are zero) at dst + i *
 * dst_stride (device memory, at least composite_tiled_bytes each): the
 * counterpart of the paper's buffer-to-image transform (Section 4; its rate
 * over image dimensions is the experiment of Section 5.2).  Enqueued on
 * `stream` (a hipStream_t, or NULL for the null stream); returns without
 * waiting.  Any W; the streamed CMP_TILED path needs W a multiple of 16. */
int composite_repack_tiled(const uint8_t *src, int64_t src_stride, uint8_t *dst,
                           int64_t dst_stride, int32_t n, int32_t W, int32_t H,
                           int32_t tile_w, int32_t tile_h, void *stream);

/* Bytes of one raster in the tiled layout (edge tiles padded). */
int64_t composite_tiled_bytes(int32_t W, int32_t H, int32_t tile_w, int32_t tile_h);

/* For callers that cannot allocate memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): composite_add_device
 * without a context and without any allocation.  It folds n device-resident
 * members (dev_maps[i]: W*H bytes, row-major, any alignment) into
 * caller-owned device accumulators: count (uint16 or uint32 per count_bits),
 * sum (uint32) and max (uint8), each W*H elements, row-major, 16-byte
 * aligned, for the outputs selected (non-empty OR of cmp_outputs; unselected
 * pointers are ignored).  set = 1: the accumulators' previous contents are
 * ignored and the composite of the n members is written, as after
 * composite_clear (n == 0 writes zeros); set = 0: the members are added to
 * what they hold.  The caller keeps the totals in range (at most 65535 or
 * 2^32 - 1 members in a count, 16843009 in a sum).  Enqueued on `stream` (a
 * hipStream_t, or NULL for the null stream) on the current device; returns
 * without waiting, and dev_maps may be reused on return.
 * The member table lives in one fixed device array per GPU of
 * CMP_STATIC_MAX_MEMBERS pointers (64 KiB) that every call on that GPU
 * shares: n above it gives CMP_ERANGE.  Calls on one GPU must therefore be
 * ordered (the same stream, or ordered by the caller); calls that overlap race
 * on the table.  Returns CMP_EINVAL for bad arguments, CMP_EDEVICE if a
 * launch fails. */
#define CMP_STATIC_MAX_MEMBERS 8192
int composite_accumulate_static(const uint8_t *const *dev_maps, int32_t n, int32_t W, int32_t H,
                                uint32_t outputs, int32_t count_bits, void *dev_count,
                                uint32_t *dev_sum, uint8_t *dev_max, int32_t set, void *stream);

/* Static description of a status code; never NULL. */
const char *composite_strerror(int status);

/* Waits for in-flight work, then releases everything the context owns: the
 * accumulators and staging buffers of the listings (Section 4), which the
 * paper keeps for the life of its program.  NULL is ignored. */
void composite_free(cmp_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* COMPOSITE_H */
