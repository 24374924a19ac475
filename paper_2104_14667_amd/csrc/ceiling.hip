// Same-traffic reference kernel for the roofline of the resident compositing
// kernel (measurement only; built as its own library, libceiling.so, and
// loaded by the benchmark, never by the compositing library).
//
// It issues the loads and stores of the compositing kernel's linear path with
// trivial arithmetic in place of the compositing: n member streams read with
// non-temporal 16-byte loads, 16 pixels per thread, then, by mode,
//   0: nothing more (the read-only rate),
//   1: 9 bytes per pixel of composite read and written (uint32 count, uint32
//      sum, uint8 max),
//   2: 4 bytes per pixel read and written (uint32 count, the served sessions'
//      composite),
//   3: 2 bytes per pixel read and written (uint16 count),
//   4: the 9 bytes per pixel written without being read (a composite set from
//      cleared accumulators),
//   5: the 9 bytes per pixel read without being written,
//   6: as 4, with each workgroup starting at member blockIdx.x mod n and
//      wrapping around (the members' order rotated per workgroup),
//   7 .. 12: as 4, phased (k_phased below): V = 2, 4, 8 vectors per thread per
//      round, with 2 (modes 7 .. 9) or 4 (modes 10 .. 12) workgroups per
//      compute unit,
//   13: as 4, with the members interleaved in 1 KiB blocks (block b of member i
//      at (b * n + i) * 1024): a wave's 64 vectors are one block, and its n
//      member loads walk n KiB of contiguous memory (stride is ignored; the
//      members take n * npix bytes).
// Its rate is what the memory system sustains for that access pattern, the
// attainable bound for the compositing kernel on the same data; modes 0, 4, 5
// and 1 side by side split the cost of the composite's read and write.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) u32x4 gu32x4;

// Byte offset of vector t (16 bytes) of member i: member-major (i * stride +
// 16 t), or interleaved in 1 KiB blocks of 64 vectors (mode 13).
template <int RMW>
__device__ __forceinline__ int64_t member_off(int i, int64_t stride, int n, uint32_t t) {
  if constexpr (RMW == 13)
    return ((int64_t)(t >> 6) * n + i) * 1024 + (int64_t)(t & 63u) * 16;
  else
    return (int64_t)i * stride + (int64_t)t * 16;
}

template <int RMW>
__global__ __launch_bounds__(256) void k_ceiling(const uint8_t *__restrict__ mem, int64_t stride, int n,
                                                 uint32_t *__restrict__ cnt, uint32_t *__restrict__ sum,
                                                 uint8_t *__restrict__ mx, uint32_t nvec, uint32_t never) {
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  if (t >= nvec) return;
  uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  // member of step j: (rot + j) mod n
  const int rot = RMW == 6 ? (int)(blockIdx.x % (unsigned)n) : 0;
  auto member = [&](int j) {
    const int m = rot + j;
    return m >= n ? m - n : m;
  };
  int i = 0;
  for (; i + 8 <= n; i += 8) {
    u32x4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      v[u] = __builtin_nontemporal_load((gu32x4 *)(mem + member_off<RMW>(member(i + u), stride, n, t)));
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a0 += v[u].x;
      a1 += v[u].y;
      a2 += v[u].z;
      a3 ^= v[u].w;
    }
  }
  for (; i < n; ++i) {
    const u32x4 v = __builtin_nontemporal_load((gu32x4 *)(mem + member_off<RMW>(member(i), stride, n, t)));
    a0 += v.x;
    a1 += v.y;
    a2 += v.z;
    a3 ^= v.w;
  }
  uint4 *c = reinterpret_cast<uint4 *>(cnt + t * 16u);
  uint4 *s = reinterpret_cast<uint4 *>(sum + t * 16u);
  uint4 *x = reinterpret_cast<uint4 *>(mx + t * 16u);
  if (RMW == 3) {
    uint4 *c16 = reinterpret_cast<uint4 *>(reinterpret_cast<uint16_t *>(cnt) + t * 16u);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint4 o = c16[q];
      c16[q] = make_uint4(o.x + a0, o.y + a1, o.z + a2, o.w + a3);
    }
  } else if (RMW == 4 || RMW == 6 || RMW == 13) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      c[q] = make_uint4(a0 + q, a1, a2, a3);
      s[q] = make_uint4(a0 ^ q, a1, a2, a3);
    }
    x[0] = make_uint4(a0 | 1u, a1, a2, a3);
  } else if (RMW == 5) {
    uint32_t r = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint4 o = c[q], p = s[q];
      r += o.x ^ o.y ^ o.z ^ o.w ^ p.x ^ p.y ^ p.z ^ p.w;
    }
    const uint4 o = x[0];
    r += o.x ^ o.y ^ o.z ^ o.w;
    if (r == never && a0 == never) c[0] = make_uint4(a0, a1, a2, a3);  // keeps the loads live; not taken
  } else if (RMW == 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint4 o = c[q];
      c[q] = make_uint4(o.x + a0, o.y + a1, o.z + a2, o.w + a3);
    }
  } else if (RMW == 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint4 o = c[q], p = s[q];
      c[q] = make_uint4(o.x + a0, o.y + a1, o.z + a2, o.w + a3);
      s[q] = make_uint4(p.x ^ a0, p.y ^ a1, p.z ^ a2, p.w ^ a3);
    }
    const uint4 o = x[0];
    x[0] = make_uint4(o.x | a0, o.y | a1, o.z | a2, o.w | a3);
  } else if (a0 == never && a1 == never && a2 == never && a3 == never) {
    c[0] = make_uint4(a0, a1, a2, a3);  // keeps the loads live; not taken
  }
}

// Phased variant of mode 4: a grid of `blocks` workgroups walks the pixels in
// rounds of gridDim.x * 256 * V vectors.  In each round a thread first reads
// all n members for its V vectors (vector base + u * nthreads + thread, two
// members' loads in flight at a time), then writes the 9 bytes per pixel of
// those V vectors.  Every thread has the same work, so the writes of a round
// cluster in time instead of trickling out between the reads.
template <int V>
__global__ __launch_bounds__(256) void k_phased(const uint8_t *__restrict__ mem, int64_t stride, int n,
                                                uint32_t *__restrict__ cnt, uint32_t *__restrict__ sum,
                                                uint8_t *__restrict__ mx, uint32_t nvec) {
  const uint32_t nthreads = gridDim.x * 256u;
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  for (uint32_t base = 0; base < nvec; base += nthreads * V) {
    uint32_t a[V][4];
#pragma unroll
    for (int u = 0; u < V; ++u) a[u][0] = a[u][1] = a[u][2] = a[u][3] = 0u;
    for (int i = 0; i < n; i += 2) {
      u32x4 x[2][V];
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const uint32_t idx = base + u * nthreads + t;
          x[m][u] = (idx < nvec && i + m < n)
                        ? __builtin_nontemporal_load((gu32x4 *)(mem + (int64_t)(i + m) * stride + idx * 16u))
                        : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int u = 0; u < V; ++u) {
          a[u][0] += x[m][u].x;
          a[u][1] += x[m][u].y;
          a[u][2] += x[m][u].z;
          a[u][3] ^= x[m][u].w;
        }
    }
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const uint32_t idx = base + u * nthreads + t;
      if (idx >= nvec) continue;
      uint4 *c = reinterpret_cast<uint4 *>(cnt + idx * 16u);
      uint4 *s = reinterpret_cast<uint4 *>(sum + idx * 16u);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c[q] = make_uint4(a[u][0] + q, a[u][1], a[u][2], a[u][3]);
        s[q] = make_uint4(a[u][0] ^ q, a[u][1], a[u][2], a[u][3]);
      }
      reinterpret_cast<uint4 *>(mx + idx * 16u)[0] = make_uint4(a[u][0] | 1u, a[u][1], a[u][2], a[u][3]);
    }
  }
}

// The batched matrix kernel's read pattern with trivial arithmetic: a grid of
// `blocks` workgroups of four waves takes tiles of 512 pixels of one row
// (tile = row * segs + segment) in turn; for each tile every wave reads 128
// pixels (8 bytes per lane: 16 lanes per member, 4 members per load) of every
// one of the pool's `count` rasters, 32 rasters (8 loads) per step, two steps
// in flight.  Raster k's row y is at base + k * stride + y * pitch.  One
// 16-byte store per lane per tile keeps the loads live.
__global__ __launch_bounds__(256) void k_tile_reads(const uint8_t *__restrict__ base, int64_t stride,
                                                    int64_t pitch, int32_t count, int32_t W, int32_t H,
                                                    uint32_t *__restrict__ sink,
                                                    uint32_t *__restrict__ wout, int32_t wsegs) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  typedef const __attribute__((address_space(1))) u32x2 gu32x2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row16 = lane & 15, kg = lane >> 4;
  const int segs = (W + 511) / 512;
  const int ntiles = H * segs;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int y = tile / segs;
    const int xw = (tile - y * segs) * 512 + 128 * wave;
    uint32_t a0 = 0, a1 = 0;
    if (xw < W) {
      const int x = min(xw + 8 * row16, W - 8);
      const uint8_t *rb = base + (int64_t)y * pitch + x;
      for (int c = 0; c + 32 <= count; c += 64) {
        u32x2 v[16];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int k = c + 32 * h + 8 * kg + i;
            v[8 * h + i] = k < count ? __builtin_nontemporal_load((gu32x2 *)(rb + (int64_t)k * stride))
                                     : u32x2{0u, 0u};
          }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          a0 += v[j].x;
          a1 ^= v[j].y;
        }
      }
    }
    sink[(int64_t)tile * 256 + threadIdx.x] = a0 ^ a1;
    // then, with wsegs > 0, wsegs pieces of the tile's 512 pixels of u32
    // (2 KiB each, a wave's 128 pixels as 8 bytes per lane): the output
    // volume of the batched kernel's covering requests
    if (xw < W) {
      for (int s = 0; s < wsegs; ++s) {
        typedef __attribute__((address_space(1))) u32x2 gw32x2;
        *(gw32x2 *)(wout + ((int64_t)tile * wsegs + s) * 512 + 128 * wave + 2 * lane) =
            u32x2{a0 + (uint32_t)s, a1 ^ (uint32_t)s};
      }
    }
  }
}

// Grid-wide barrier of a co-resident (cooperatively launched) grid: every
// workgroup adds one to *bar per barrier, and barrier k is passed once *bar
// reaches k * gridDim.x.  The wait is bounded: after `limit` polls the
// workgroup sets *err and goes on, so the kernel always ends (its result is
// then void and the host reports the error).
__device__ __forceinline__ void grid_barrier(uint32_t *bar, uint32_t *err, uint32_t &target,
                                             uint32_t limit) {
  __syncthreads();
  target += gridDim.x;
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(bar, 1u);
    uint32_t polls = 0;
    // once any wait has given up, no later one waits at all
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target &&
           __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
      if (++polls >= limit) {
        atomicOr(err, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
  }
  __syncthreads();
}

// Mode 4's traffic with the reads and the writes of the whole grid kept apart:
// the pixels go in bands of gridDim.x * 256 * V vectors; in each band every
// thread reads all n members for its V vectors (non-temporal 16-byte loads,
// two members' loads in flight), then, after a grid-wide barrier, writes
// those vectors' 9 bytes per pixel, and a second barrier closes the band, so
// that no read of the grid is in flight while the band is written.
template <int V>
__global__ __launch_bounds__(256) void k_two_phase(const uint8_t *__restrict__ mem, int64_t stride,
                                                   int n, uint32_t *__restrict__ cnt,
                                                   uint32_t *__restrict__ sum, uint8_t *__restrict__ mx,
                                                   uint32_t nvec, uint32_t *bar, uint32_t *err,
                                                   uint32_t limit) {
  const uint32_t nthreads = gridDim.x * 256u;
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  uint32_t target = 0;
  for (uint32_t base = 0; base < nvec; base += nthreads * V) {
    uint32_t a[V][4];
#pragma unroll
    for (int u = 0; u < V; ++u) a[u][0] = a[u][1] = a[u][2] = a[u][3] = 0u;
    for (int i = 0; i < n; i += 2) {
      u32x4 x[2][V];
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const uint32_t idx = base + u * nthreads + t;
          x[m][u] = (idx < nvec && i + m < n)
                        ? __builtin_nontemporal_load((gu32x4 *)(mem + (int64_t)(i + m) * stride + idx * 16u))
                        : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int u = 0; u < V; ++u) {
          a[u][0] += x[m][u].x;
          a[u][1] += x[m][u].y;
          a[u][2] += x[m][u].z;
          a[u][3] ^= x[m][u].w;
        }
    }
    grid_barrier(bar, err, target, limit);
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const uint32_t idx = base + u * nthreads + t;
      if (idx >= nvec) continue;
      uint4 *c = reinterpret_cast<uint4 *>(cnt + idx * 16u);
      uint4 *s = reinterpret_cast<uint4 *>(sum + idx * 16u);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c[q] = make_uint4(a[u][0] + q, a[u][1], a[u][2], a[u][3]);
        s[q] = make_uint4(a[u][0] ^ q, a[u][1], a[u][2], a[u][3]);
      }
      reinterpret_cast<uint4 *>(mx + idx * 16u)[0] = make_uint4(a[u][0] | 1u, a[u][1], a[u][2], a[u][3]);
    }
    grid_barrier(bar, err, target, limit);
  }
}

}  // namespace

extern "C" {

// Runs k_two_phase<V> (V = 2, 4 or 8) reps times on `stream` with
// blocks_per_cu workgroups per compute unit, launched cooperatively (the
// runtime refuses a grid that cannot be resident at once), over n rasters at
// members + i * stride (npix bytes each, a multiple of 16, 16-byte aligned)
// and composite buffers as traffic_ceiling's; *best_ms: the fastest run after
// the first.  scratch: 8 bytes of device memory (barrier counter and error
// flag).  Returns 0, a hipError_t, or -1 if a barrier wait gave up.
int two_phase_ceiling(const uint8_t *members, int64_t stride, int32_t n, int64_t npix, void *count,
                      void *sum, void *max, int32_t V, int32_t blocks_per_cu, void *scratch,
                      int32_t reps, void *stream, float *best_ms) {
  if (!members || !count || !sum || !max || !scratch || !best_ms || n < 1 || reps < 2 ||
      npix < 16 || npix % 16 || npix > (int64_t(1) << 32) - 16 || stride < npix ||
      (V != 2 && V != 4 && V != 8) || blocks_per_cu < 1 || blocks_per_cu > 8)
    return (int)hipErrorInvalidValue;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  uint32_t nvec = (uint32_t)(npix / 16);
  uint32_t *bar = static_cast<uint32_t *>(scratch), *err = bar + 1;
  uint32_t limit = 1u << 20;  // polls of at most a few us: a wait gives up within seconds
  const void *fn = V == 2 ? (const void *)k_two_phase<2>
                   : V == 4 ? (const void *)k_two_phase<4> : (const void *)k_two_phase<8>;
  void *args[] = {(void *)&members, (void *)&stride, (void *)&n, (void *)&count, (void *)&sum,
                  (void *)&max, (void *)&nvec, (void *)&bar, (void *)&err, (void *)&limit};
  hipEvent_t e0, e1;
  e = hipEventCreate(&e0);
  if (e != hipSuccess) return (int)e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return (int)e;
  }
  float best = 0.f;
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipMemsetAsync(scratch, 0, 8, s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess)
      e = hipLaunchCooperativeKernel(fn, dim3((unsigned)(cus * blocks_per_cu)), dim3(256), args, 0, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && r > 0 && (r == 1 || ms < best)) best = ms;
  }
  uint32_t h[2] = {0u, 0u};
  if (e == hipSuccess) e = hipMemcpy(h, scratch, 8, hipMemcpyDeviceToHost);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best_ms = best;
  if (e != hipSuccess) return (int)e;
  return h[1] ? -1 : 0;
}

// Runs k_tile_reads reps times on `stream` with `blocks` workgroups over a
// pool of count rasters of W x H (W >= 8), raster k's row y at
// base + k * stride + y * pitch, and returns the fastest run after the first
// in *best_ms.  sink: H * ceil(W / 512) * 256 uint32 of device memory.
// wsegs > 0: each 512-pixel tile also writes wsegs pieces of 2 KiB to wout
// (H * ceil(W / 512) * wsegs * 512 uint32 of device memory; NULL with 0).
// Returns 0 or a hipError_t.
int tile_read_ceiling(const uint8_t *base, int64_t stride, int64_t pitch, int32_t count, int32_t W,
                      int32_t H, void *sink, void *wout, int32_t wsegs, int32_t blocks, int32_t reps,
                      void *stream, float *best_ms) {
  if (!base || !sink || !best_ms || count < 32 || W < 8 || H < 1 || blocks < 1 || reps < 2 ||
      stride < 1 || pitch < W || wsegs < 0 || (wsegs > 0 && !wout))
    return (int)hipErrorInvalidValue;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return (int)e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return (int)e;
  }
  float best = 0.f;
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, s);
    if (e != hipSuccess) break;
    k_tile_reads<<<blocks, 256, 0, s>>>(base, stride, pitch, count, W, H, (uint32_t *)sink,
                                        (uint32_t *)wout, wsegs);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && r > 0 && (r == 1 || ms < best)) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best_ms = best;
  return (int)e;
}

// Runs the kernel reps times on `stream` (a hipStream_t, or NULL) over n
// rasters at members + i * stride (npix bytes each, npix a multiple of 16,
// 16-byte aligned) and composite buffers count, sum (npix uint32 each) and
// max (npix bytes), and returns in *best_ms the fastest of the runs after the
// first.  rmw: the mode, 0 .. 13 as above.  Returns 0 or a hipError_t.  The
// composite buffers are overwritten.
int traffic_ceiling(const uint8_t *members, int64_t stride, int32_t n, int64_t npix, void *count,
                    void *sum, void *max, int32_t rmw, int32_t reps, void *stream, float *best_ms) {
  if (!members || !count || !sum || !max || !best_ms || n < 1 || reps < 2 || npix < 16 ||
      npix % 16 || npix > (int64_t(1) << 32) - 16 || stride < npix || rmw < 0 || rmw > 13 ||
      (rmw == 13 && npix % 1024))  // whole 1 KiB blocks: the n blocks of a wave end at n * npix
    return (int)hipErrorInvalidValue;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0, cus = 0;
  hipError_t ea = hipGetDevice(&dev);
  if (ea == hipSuccess) ea = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (ea != hipSuccess) return (int)ea;
  const unsigned pgrid = (unsigned)cus * (rmw >= 10 ? 4u : 2u);
  const uint32_t nvec = (uint32_t)(npix / 16);
  const unsigned grid = (nvec + 255) / 256;
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return (int)e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return (int)e;
  }
  float best = 0.f;
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, s);
    if (e != hipSuccess) break;
#define CMP_CEIL(M)                                                                       \
  k_ceiling<M><<<grid, 256, 0, s>>>(members, stride, n, (uint32_t *)count, (uint32_t *)sum, \
                                    (uint8_t *)max, nvec, 0x9e3779b9u)
    switch (rmw) {
      case 13: CMP_CEIL(13); break;
      case 7: case 10: k_phased<2><<<pgrid, 256, 0, s>>>(members, stride, n, (uint32_t *)count, (uint32_t *)sum, (uint8_t *)max, nvec); break;
      case 8: case 11: k_phased<4><<<pgrid, 256, 0, s>>>(members, stride, n, (uint32_t *)count, (uint32_t *)sum, (uint8_t *)max, nvec); break;
      case 9: case 12: k_phased<8><<<pgrid, 256, 0, s>>>(members, stride, n, (uint32_t *)count, (uint32_t *)sum, (uint8_t *)max, nvec); break;
      case 6: CMP_CEIL(6); break;
      case 5: CMP_CEIL(5); break;
      case 4: CMP_CEIL(4); break;
      case 3: CMP_CEIL(3); break;
      case 2: CMP_CEIL(2); break;
      case 1: CMP_CEIL(1); break;
      default: CMP_CEIL(0); break;
    }
#undef CMP_CEIL
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && r > 0 && (r == 1 || ms < best)) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best_ms = best;
  return (int)e;
}

}  // extern "C"
