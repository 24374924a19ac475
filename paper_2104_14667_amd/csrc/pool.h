// The pool of device-resident rasters behind composite_pool_* (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>

struct cmp_pool {
  int dev = 0;
  const uint8_t *base = nullptr;
  int64_t count = 0, stride = 0, bytes = 0;
  int32_t W = 0, H = 0;
  int cus = 0;
  int max_lds = 0;  // LDS bytes a workgroup may use (0: shared mode unavailable)
  int max_lds_matrix = 0;  // dynamic LDS k_matrix may use (0: matrix mode unavailable)
  int static_lds_shared = 0;  // static LDS of the k_shared instances, as compiled
  bool poisoned = false;
  hipStream_t s = nullptr;
  char *d_arena = nullptr, *h_arena = nullptr;
  int64_t arena_cap = 0;
  uint32_t *d_queue = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0.0;
  int64_t last_items = 0;
  int32_t last_mode = 0;
  std::map<int, hipGraphExec_t> graphs;  // by mode, grid size, load kind, slots; they capture d_arena
};
