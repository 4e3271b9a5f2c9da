"""Workgroup-to-block mapping of the tile kernel, emulated on the host:
workgroup h runs on XCD h % 8; each XCD takes a contiguous range of blocks
and a block's column groups sit in consecutive slots of one XCD.  Every
(block, column group) must be taken by exactly one workgroup of the grid,
and the surplus workgroups must exit."""
import pytest


def mapping(n_blocks, ng):
    per_xcd = (n_blocks + 7) // 8
    grid = 8 * per_xcd * ng
    seen = {}
    for h in range(grid):
        slot = h >> 3
        b = (h & 7) * per_xcd + slot // ng
        grp = slot % ng
        if slot // ng >= per_xcd or b >= n_blocks:
            continue                      # exits
        seen.setdefault((b, grp), []).append(h)
    return seen, per_xcd


@pytest.mark.parametrize("n_blocks", [1, 7, 8, 9, 641, 1281, 2561, 10241])
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
