// Device helpers shared by the compositing kernels (gfx950): byte lanes of
// uint8 rasters are split into packed 16-bit lanes with v_perm_b32 and updated
// with packed integer instructions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace cmp {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t lanes_lo(uint32_t w) {  // bytes 0,2 -> u16 lanes
  return __builtin_amdgcn_perm(0u, w, 0x0c020c00u);
}
__device__ __forceinline__ uint32_t lanes_hi(uint32_t w) {  // bytes 1,3 -> u16 lanes
  return __builtin_amdgcn_perm(0u, w, 0x0c030c01u);
}
__device__ __forceinline__ u16x2 as16(uint32_t a) { return __builtin_bit_cast(u16x2, a); }
__device__ __forceinline__ uint32_t as32(u16x2 a) { return __builtin_bit_cast(uint32_t, a); }
// min(lane, 1) on both 16-bit lanes.  Written as the instruction itself:
// the compiler otherwise rewrites min(x, 1) as (x != 0) and splits the lanes
// into compares and selects, three times the work.
__device__ __forceinline__ uint32_t pmin1(uint32_t a) {
  uint32_t r;
  asm("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(a), "s"(0x00010001u));
  return r;
}
__device__ __forceinline__ uint32_t pmax(uint32_t a, uint32_t b) {
  return as32(__builtin_elementwise_max(as16(a), as16(b)));
}
__device__ __forceinline__ uint32_t padd(uint32_t a, uint32_t b) { return as32(as16(a) + as16(b)); }
__device__ __forceinline__ uint32_t psub(uint32_t a, uint32_t b) { return as32(as16(a) - as16(b)); }
// Bytewise max of two dwords.
__device__ __forceinline__ uint32_t bmax(uint32_t a, uint32_t b) {
  const uint32_t l = pmax(lanes_lo(a), lanes_lo(b));
  const uint32_t h = pmax(lanes_hi(a), lanes_hi(b));
  return __builtin_amdgcn_perm(h, l, 0x06020400u);
}

typedef unsigned int u32x4u __attribute__((ext_vector_type(4), aligned(1)));
typedef const __attribute__((address_space(1))) u32x4u gu32x4u;

// 16 member bytes from global memory at base + off, any alignment: one
// global_load_dwordx4 with the non-temporal hint.  Every member byte is read
// exactly once, so the loads should not displace the composite's lines in the
// caches (measured: +4% bandwidth over plain loads for 128 members of 8192^2).
__device__ __forceinline__ uint4 ld16(const uint8_t *base, uint32_t off) {
  const u32x4u v = __builtin_nontemporal_load((gu32x4u *)(base + off));
  return make_uint4(v.x, v.y, v.z, v.w);
}
// The same load without the hint, for bytes other workgroups read again soon
// (batched requests that share pool members): they may stay in L2/MALL.
__device__ __forceinline__ uint4 ld16_cached(const uint8_t *base, uint32_t off) {
  const u32x4u v = *(gu32x4u *)(base + off);
  return make_uint4(v.x, v.y, v.z, v.w);
}
template <bool NT>
__device__ __forceinline__ uint4 ld16_t(const uint8_t *base, uint32_t off) {
  if constexpr (NT) return ld16(base, off);
  else return ld16_cached(base, off);
}

// Packed accumulators of 16 pixels.  Lane pair k*2 holds pixels 4k and 4k+2,
// lane pair k*2+1 holds pixels 4k+1 and 4k+3 (low half first).
template <uint32_t OUTS>
struct Acc {
  uint32_t c[8], s[8], m[8];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = s[k] = m[k] = 0u;
  }
  __device__ __forceinline__ void fold(const uint4 x) {
    const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t lo = lanes_lo(w[k]), hi = lanes_hi(w[k]);
      if constexpr (OUTS & kCount) {
        c[2 * k] += pmin1(lo);
        c[2 * k + 1] += pmin1(hi);
      }
      if constexpr (OUTS & kSum) {
        s[2 * k] += lo;
        s[2 * k + 1] += hi;
      }
      if constexpr (OUTS & kMax) {
        m[2 * k] = pmax(m[2 * k], lo);
        m[2 * k + 1] = pmax(m[2 * k + 1], hi);
      }
    }
  }
};

// Value of pixel j (0..15) held in packed lanes a[8].
__device__ __forceinline__ uint32_t lane_px(const uint32_t *a, int j) {
  const int k = j >> 2, r = j & 3;
  const uint32_t d = a[2 * k + (r & 1)];
  return (r & 2) ? (d >> 16) : (d & 0xffffu);
}

template <int UNROLL, uint32_t OUTS>
__device__ __forceinline__ void fold_members(const uint8_t *const *__restrict__ tab,
                                             int i0, int i1, uint32_t off, Acc<OUTS> &a) {
  int i = i0;
  for (; i + UNROLL <= i1; i += UNROLL) {
    uint4 x[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) x[u] = ld16(tab[i + u], off);
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) a.fold(x[u]);
  }
  for (; i < i1; ++i) a.fold(ld16(tab[i], off));
}


}  // namespace cmp
