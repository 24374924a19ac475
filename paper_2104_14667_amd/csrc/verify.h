// Member fingerprints: a 64-bit value per raster that lets the registry tell
// whether the raster handed to a remove is the one that was added.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmp {

// out[i] += fingerprint of member i, for i < n, where member i is tab[i] when
// tab is non-null, else base + i * stride; each member is npix bytes, any
// alignment.  The fingerprint is the sum over the raster's little-endian
// 32-bit words d_j (the last one zero-padded) of d_j * weight(j), modulo
// 2^64, with weight(j) an integer hash of j (Wellons' "lowbias32" mixer)
// forced odd, so that a change to any single word always changes the value.
// out must be zeroed by the caller.
hipError_t launch_fingerprint(const uint8_t *const *tab, const uint8_t *base, int64_t stride,
                              int n, int64_t npix, unsigned long long *out, hipStream_t s);

}  // namespace cmp
