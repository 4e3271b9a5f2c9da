"""LDS layout of the staged irradiance in the 16-bit tile kernel, with the
kernel's own index functions (tile_swizzle, tile_read_slot,
tile_stage_lane, tile_stage_swizzle, tile_stage_slot in
csrc/index_maps.h, compiled for the host).  B-operand fragments hold lane
l's 16 bytes at a slot permuted inside groups of four.  The LDS serves
16-byte accesses eight lanes at a time over 32 four-byte banks, so every
group of eight consecutive lanes of a fragment read, and of a staging store
(eight consecutive items, in the staging loop's item order), must touch
eight distinct 16-byte units modulo 8; the reads are also checked for
sixteen lanes over 64 banks."""
import pytest

from _index_maps import lib

KPL, H = 8, 2          # 16-bit values per lane and operand; hi and lo halves


def worst(units, group, mod):
    w = 1
    for g0 in range(0, len(units), group):
        cnt = {}
        for u in units[g0:g0 + group]:
            cnt[u % mod] = cnt.get(u % mod, 0) + 1
        w = max(w, max(cnt.values()))
    return w


def store_units(NT, jj, h, items):
    """16-byte unit written by each item's store jj of half h; the item
    decomposition is the staging loop's (column quad q, lane group lg, step
    sl)."""
    L = lib()
    cq = NT * 16 // 4                      # column quads per (step, lane group)
    units = []
    for item in items:
        q = item % cq
        lg = (item // cq) % 4
        sl = item // (cq * 4)
        n = 4 * q
        slot = L.tile_stage_slot(L.tile_stage_lane(n, lg), jj, L.tile_stage_swizzle(n, lg))
        units.append(((sl * NT + n // 16) * H + h) * 64 + slot)
    return units


@pytest.mark.parametrize("NT", [1, 2, 3, 4])
def test_fragment_reads_are_conflict_free(NT):
    L = lib()
    for nt in range(NT):
        slots = [L.tile_read_slot(l, nt) for l in range(64)]
        assert sorted(slots) == list(range(64))          # a permutation of the lanes
        assert all(s // 4 == l // 4 for l, s in enumerate(slots))   # inside groups of four
        assert worst(slots, 8, 8) == 1
        assert worst(slots, 16, 16) == 1


@pytest.mark.parametrize("NT", [1, 2, 3, 4])
def test_staging_stores_are_conflict_free(NT):
    for wave in range(24):
        items = range(64 * wave, 64 * wave + 64)
        for h in range(H):
            for jj in range(4):
                assert worst(store_units(NT, jj, h, items), 8, 8) == 1, (NT, wave, h, jj)


@pytest.mark.parametrize("NT", [1, 2, 3, 4])
def test_store_and_read_agree_on_slots(NT):
    """Column n of lane group lg is written where the read of its column
    tile expects lane lg * 16 + n % 16."""
    L = lib()
    for lg in range(4):
        for n in range(0, NT * 16):
            nt = n // 16
            q0 = (n // 4) * 4                            # the item's column quad
            written = L.tile_stage_slot(L.tile_stage_lane(q0, lg), n - q0, L.tile_stage_swizzle(q0, lg))
            assert written == L.tile_read_slot(lg * 16 + n % 16, nt)
