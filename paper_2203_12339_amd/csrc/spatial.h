// Device side of the spatially compressed transport (Eq. 10; Steps 2, 4, 5
// of Sec. 4): argument block and launchers of k_spatial.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tlt {

constexpr int SP_MAX_K = 128;      // terms addressable by the column word

struct SpatialArgs {
  // kept entries of Z (CSR over u): column word (k << 24) | j, value
  const uint32_t *col;
  const void *val;           // compute precision
  // work items: entries [e0, e1) of one row u; y[c, u] is the sum of the
  // partials of u's items
  int n_items;
  int lanes_per_item;        // 16, 32 or 64 (narrow form)
  int unroll;                // entries per lane and pass: 4, 8 or 16 (narrow form)
  const int64_t *item_e0, *item_e1;
  void *part;                // [n_items][C] partial sums (compute precision)
  const void *ehat;          // [n_rows][Cs]
  const void *gcol;          // [K][Cs]
  int Cs, C, K, N;
  // w_1^{-1} expanded over work items, padded CSR over the output position:
  // syn_len entries per position, a multiple of syn_lanes, and of 4 syn_lanes
  // beyond 8 syn_lanes (padding: item 0, weight 0)
  int syn_len, syn_lanes;    // syn_lanes: 8, 16 or 32 lanes per output position
  const int32_t *syn_col;    // [N][syn_len] work item
  const void *syn_w;         // [N][syn_len] compute precision
  const int32_t *perm;       // Morton position -> vertex
  void *B;                   // [n_out][N][3]
};

// y from the kept entries and Ehat (Steps 2 and 4), then B = w_1^{-1} y in
// original vertex order (Step 5).
hipError_t launch_spatial_rows(const SpatialArgs &a, bool fp64, hipStream_t st);
hipError_t launch_spatial_synthesis(const SpatialArgs &a, bool fp64, hipStream_t st);

}  // namespace tlt
