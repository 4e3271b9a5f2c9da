"""Workgroup-to-block mapping of the tile kernel (tile_block, tile_group,
tile_runs in csrc/index_maps.h, compiled for the host): workgroup h runs on
XCD h % 8; each XCD takes a contiguous range of blocks and a block's column
groups sit in consecutive slots of one XCD.  Every (block, column group)
must be taken by exactly one workgroup of the grid, and the surplus
workgroups must exit."""
import pytest

from _index_maps import lib


def mapping(n_blocks, ng):
    L = lib()
    per_xcd = L.tile_per_xcd(n_blocks)
    grid = 8 * per_xcd * ng           # the launch's grid (tiles_launch)
    seen = {}
    for h in range(grid):
        if not L.tile_runs(h, per_xcd, ng, n_blocks):
            continue                  # exits
        seen.setdefault((L.tile_block(h, per_xcd, ng), L.tile_group(h, ng)), []).append(h)
    return seen, per_xcd


@pytest.mark.parametrize("n_blocks", [1, 7, 8, 9, 641, 1281, 2561, 5121, 10241])
@pytest.mark.parametrize("ng", [1, 3, 4])
def test_every_block_and_group_once(n_blocks, ng):
    seen, per_xcd = mapping(n_blocks, ng)
    assert set(seen) == {(b, g) for b in range(n_blocks) for g in range(ng)}
    assert all(len(v) == 1 for v in seen.values())
    # a block's groups run on one XCD, in consecutive slots
    for b in range(n_blocks):
        hs = sorted(seen[(b, g)][0] for g in range(ng))
        assert len({h % 8 for h in hs}) == 1
        assert [h >> 3 for h in hs] == list(range(hs[0] >> 3, (hs[0] >> 3) + ng))
        assert hs[0] % 8 == b // per_xcd
