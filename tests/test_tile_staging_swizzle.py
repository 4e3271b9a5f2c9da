"""LDS layout of the staged irradiance in the 16-bit tile kernel, with the
kernel's own index functions (tile_swizzle, tile_read_slot,
tile_stage_lane, tile_stage_slot in csrc/index_maps.h, compiled for the
host): B-operand fragments hold lane l's 16 bytes at slot
l ^ ((tile + NT (l / 16)) & 3); a quarter-wave of a fragment read then
covers all 16 sixteen-byte bank groups, and the staging stores of 16
consecutive work items land in 16 different groups."""
import pytest

from _index_maps import lib

KPL, H = 8, 2          # 16-bit values per lane and operand; hi and lo halves


def store_groups(NT, jj, items):
    """16-byte bank group of each item's store number jj (hi half); the
    item decomposition is the staging loop's (column quad q, lane group lg,
    step sl)."""
    L = lib()
    cq = NT * 16 // 4                      # column quads per (step, lane group)
    groups = []
    for item in items:
        q = item % cq
        lg = (item // cq) % 4
        sl = item // (cq * 4)
        n = 4 * q
        base = (sl * NT + n // 16) * H * 64 * KPL      # fragment base (elements)
        ph = L.tile_stage_slot(L.tile_stage_lane(n, lg), jj, L.tile_swizzle(n // 16, lg, NT)) * KPL
        groups.append((2 * (base + ph) // 16) % 16)
    return groups


@pytest.mark.parametrize("NT", [1, 2, 3, 4])
def test_fragment_reads_cover_all_bank_groups(NT):
    L = lib()
    for nt in range(NT):
        slots = [L.tile_read_slot(l, nt, NT) for l in range(64)]
        assert sorted(slots) == list(range(64))          # a permutation of the lanes
        for quarter in range(4):
            qs = slots[16 * quarter:16 * quarter + 16]
            assert len({s % 16 for s in qs}) == 16


@pytest.mark.parametrize("NT", [2, 3, 4])
def test_staging_stores_spread_over_bank_groups(NT):
    for jj in range(4):
        for start in range(0, 64, 16):
            g = store_groups(NT, jj, range(start, start + 16))
            assert len(set(g)) == 16, (NT, jj, start, g)


@pytest.mark.parametrize("NT", [1, 2, 3, 4])
def test_store_and_read_agree_on_slots(NT):
    """Column n of lane group lg is written where the read of its column
    tile expects lane lg * 16 + n % 16."""
    L = lib()
    for lg in range(4):
        for n in range(0, NT * 16):
            nt = n // 16
            q0 = (n // 4) * 4                            # the item's column quad
            written = L.tile_stage_slot(L.tile_stage_lane(q0, lg), n - q0, L.tile_swizzle(q0 // 16, lg, NT))
            assert written == L.tile_read_slot(lg * 16 + n % 16, nt, NT)
