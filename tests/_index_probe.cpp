// Host build of the kernels' index maps (paper_2203_12339_amd/csrc/
// index_maps.h, the header the kernels include) for the CPU tests.
#include "index_maps.h"

namespace m = tlt::idx;

extern "C" {
int tile_per_xcd(int n_blocks) { return m::tile_per_xcd(n_blocks); }
int tile_block(unsigned h, int per_xcd, int ng) { return m::tile_block(h, per_xcd, ng); }
int tile_group(unsigned h, int ng) { return m::tile_group(h, ng); }
int tile_runs(unsigned h, int per_xcd, int ng, int n_blocks) { return m::tile_runs(h, per_xcd, ng, n_blocks); }
int tile_swizzle(int nt, int lane_group, int col_hi) { return m::tile_swizzle(nt, lane_group, col_hi); }
int tile_read_slot(int lane, int nt) { return m::tile_read_slot(lane, nt); }
int tile_stage_lane(int n, int lg) { return m::tile_stage_lane(n, lg); }
int tile_stage_swizzle(int n, int lg) { return m::tile_stage_swizzle(n, lg); }
int tile_stage_slot(int stage_lane, int jj, int sw) { return m::tile_stage_slot(stage_lane, jj, sw); }
int fold_group_index(int g, int lk, int v) { return m::fold_group_index(g, lk, v); }
int fold_tail_index(int g4, int q, int lk) { return m::fold_tail_index(g4, q, lk); }
long long haar_row(int half, int n_chunks, int chunk, int i) { return m::haar_row(half, n_chunks, chunk, i); }
int haar_reg_detail(int g, int n, int p) { return m::haar_reg_detail(g, n, p); }
}
