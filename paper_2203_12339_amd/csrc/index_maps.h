// Index arithmetic of the kernels that their parity tests cannot pin one
// map at a time: workgroup-to-block mapping of the tile kernel, the slot
// swizzle of its staged irradiance, the contraction order of the float32
// folded product and the coefficient rows of the chunked Haar transform.
// The kernels call these functions, and the host-side tests compile this
// same header with a host compiler and check each map exhaustively
// (bijectivity, bank spread, agreement between writer and reader).
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define TLT_HD __host__ __device__ __forceinline__
#else
#define TLT_HD inline
#endif

namespace tlt {
namespace idx {

// ---- tile kernel launch (k_tiles) ----
// Workgroup h of a grid of 8 * per_xcd * ng runs on XCD h % 8 (the
// dispatcher's round robin).  Each XCD takes a contiguous range of per_xcd
// blocks, and the ng column groups of one block occupy consecutive slots
// h / 8 of that XCD, so they run together and share the block's W through
// the XCD's L2.  Workgroups whose slot falls past the blocks exit.
// (h is the unsigned workgroup index, so its slot h >> 3 is known to be
// non-negative and the divisions by ng stay unsigned.)
TLT_HD int tile_per_xcd(int n_blocks) { return (n_blocks + 7) / 8; }
TLT_HD int tile_slot(unsigned h) { return (int)(h >> 3); }
TLT_HD int tile_block(unsigned h, int per_xcd, int ng) { return (int)(h & 7) * per_xcd + tile_slot(h) / ng; }
TLT_HD int tile_group(unsigned h, int ng) { return tile_slot(h) % ng; }
TLT_HD bool tile_runs(unsigned h, int per_xcd, int ng, int n_blocks) {
  return tile_slot(h) / ng < per_xcd && tile_block(h, per_xcd, ng) < n_blocks;
}

// ---- staged irradiance of the 16-bit tiles ----
// The B-operand fragment of (step, column tile nt, half) holds lane l's 16
// bytes at slot l ^ tile_swizzle(nt, l / 16, bit 3 of l).  The swizzle
// permutes slots inside groups of four only (so a fragment read stays one
// contiguous 1 KB).  The LDS serves 16-byte accesses eight lanes at a time
// over 32 four-byte banks (measured: with the earlier swizzle (nt + NT lg)
// mod 4, built for sixteen lanes over 64 banks, the reads had no bank
// conflicts and the staging stores 28 M conflict cycles per launch at
// batch64-bf16-40962); this one puts every group of eight consecutive lanes
// of a read, and of a staging store of eight consecutive items, on eight
// distinct 16-byte units modulo 8, for one to four column tiles per group.
TLT_HD int tile_swizzle(int nt, int lane_group, int col_hi) {
  return (col_hi ^ ((nt & 1) << 1) ^ ((nt >> 1) & 1) ^ (3 * (lane_group & 1)) ^ ((lane_group >> 1) & 1)) & 3;
}
TLT_HD int tile_read_slot(int lane, int nt) { return lane ^ tile_swizzle(nt, lane >> 4, (lane >> 3) & 1); }
// Staging item (column quad starting at column n of the group, lane group
// lg): the lane of its first column, the swizzle of its four slots (the
// quad lies in one half of a 16-column tile), and the slot its column
// n + jj is stored at (jj = 0..3).
TLT_HD int tile_stage_lane(int n, int lg) { return lg * 16 + n % 16; }
TLT_HD int tile_stage_swizzle(int n, int lg) { return tile_swizzle(n / 16, lg, (n % 16) >> 3); }
TLT_HD int tile_stage_slot(int stage_lane, int jj, int sw) { return (stage_lane + jj) ^ sw; }

// ---- float32 folded product (k_folded_lds) ----
// Lane group lk of a 16-byte P load of group g holds contraction indices
// 16 g + 4 lk .. 16 g + 4 lk + 3; component v enters matrix step (g, v).
// The MS % 4 steps left over (Psh not a multiple of 16) take one index per
// lane: step q of the tail is index 16 G4 + 4 q + lk.
TLT_HD int fold_group_index(int g, int lk, int v) { return 16 * g + 4 * lk + v; }
TLT_HD int fold_tail_index(int g4, int q, int lk) { return 16 * g4 + 4 * q + lk; }

// ---- chunked Haar transform (k_prep) ----
// At the level where each chunk of n_chunks has `half` detail coefficients,
// detail i of chunk `chunk` is coefficient row half (n_chunks + chunk) + i
// (the level's rows of all chunks follow each other, coarser levels first).
TLT_HD int64_t haar_row(int half, int n_chunks, int chunk, int i) {
  return (int64_t)half * (n_chunks + chunk) + i;
}
// Thread-local levels of the register schedule: thread g of 16 holds R
// consecutive rows of the chunk; at a level with n values left per thread,
// its pair p is detail g (n / 2) + p of the chunk.
TLT_HD int haar_reg_detail(int g, int n, int p) { return g * (n / 2) + p; }

}  // namespace idx
}  // namespace tlt
