// Fingerprint kernel for the member registry (see verify.h).  Off the
// compositing path: it runs only in contexts that ask for member verification.
#include "lanes.h"
#include "verify.h"

namespace cmp {
namespace {

__device__ __forceinline__ uint32_t weight(uint32_t j) {
  j ^= j >> 16;
  j *= 0x7feb352du;
  j ^= j >> 15;
  j *= 0x846ca68bu;
  j ^= j >> 16;
  return j | 1u;
}

__device__ __forceinline__ unsigned long long term(uint32_t d, uint32_t j) {
  return (unsigned long long)d * weight(j);
}

// Grid: x strides over the 16-byte vectors of one member, y picks the member.
__global__ __launch_bounds__(256) void k_fingerprint(const uint8_t *const *__restrict__ tab,
                                                     const uint8_t *__restrict__ base,
                                                     int64_t stride, int member0, int64_t npix,
                                                     unsigned long long *__restrict__ out) {
  const int m = member0 + (int)blockIdx.y;
  const uint8_t *p = tab ? tab[m] : base + (int64_t)m * stride;
  const uint32_t nvec = (uint32_t)(npix / 16);
  unsigned long long acc = 0;
  for (uint32_t v = blockIdx.x * 256 + threadIdx.x; v < nvec; v += gridDim.x * 256) {
    const uint4 x = ld16_cached(p, v * 16);
    const uint32_t j = v * 4;
    acc += term(x.x, j) + term(x.y, j + 1) + term(x.z, j + 2) + term(x.w, j + 3);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // ragged tail of fewer than 16 bytes, word by word, zero-padded
    for (int64_t b = (int64_t)nvec * 16; b < npix; b += 4) {
      uint32_t d = 0;
      for (int k = 0; k < 4 && b + k < npix; ++k) d |= (uint32_t)p[b + k] << (8 * k);
      acc += term(d, (uint32_t)(b / 4));
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  __shared__ unsigned long long part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out + m, part[0] + part[1] + part[2] + part[3]);
}

}  // namespace

hipError_t launch_fingerprint(const uint8_t *const *tab, const uint8_t *base, int64_t stride,
                              int n, int64_t npix, unsigned long long *out, hipStream_t s) {
  if (n <= 0 || npix <= 0) return hipSuccess;
  const int64_t nvec = npix / 16;
  const int64_t per_member = std::max<int64_t>(1, (nvec + 255) / 256);
  // about 4096 workgroups in all, at least one per member
  const int64_t bx = std::min<int64_t>(per_member, std::max<int64_t>(1, 4096 / n));
  for (int m0 = 0; m0 < n; m0 += 65535) {
    const int cnt = std::min(65535, n - m0);
    k_fingerprint<<<dim3((unsigned)bx, (unsigned)cnt), 256, 0, s>>>(tab, base, stride, m0, npix, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace cmp
