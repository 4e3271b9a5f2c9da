"""Index arithmetic of the float32 folded-lighting kernel, with its own
index functions (fold_group_index, fold_tail_index in csrc/index_maps.h,
compiled for the host): the permuted contraction order visits every
coefficient index of a term exactly once for every supported row length,
and the B-operand reads of one matrix step hit 64 distinct LDS banks with
rows padded to 68 floats."""
import pytest

from _index_maps import lib

LDW = 64 + 4          # staged Lg row length in floats
CASES = [1, 2, 3, 4, 6, 7, 8, 9, 12, 16]   # Psh / 4 values the kernel compiles


@pytest.mark.parametrize("ms", CASES)
def test_contraction_order_is_a_permutation(ms):
    L = lib()
    g4, r4 = ms // 4, ms % 4
    seen = []
    for g in range(g4):            # 16-byte loads: lane group lk, component v
        for v in range(4):
            for lk in range(4):
                seen.append(L.fold_group_index(g, lk, v))
    for q in range(r4):            # the leftover steps: one value per lane
        for lk in range(4):
            seen.append(L.fold_tail_index(g4, q, lk))
    assert sorted(seen) == list(range(4 * ms))


@pytest.mark.parametrize("ms", CASES)
def test_loads_are_contiguous_16_bytes(ms):
    """Component v of a lane's 16-byte load is index v of four consecutive
    ones (the load reads the row at fold_group_index(g, lk, 0))."""
    L = lib()
    for g in range(ms // 4):
        for lk in range(4):
            base = L.fold_group_index(g, lk, 0)
            assert base % 4 == 0
            assert [L.fold_group_index(g, lk, v) for v in range(4)] == [base + v for v in range(4)]


@pytest.mark.parametrize("g,v", [(0, 0), (1, 3), (3, 2)])
def test_b_operand_reads_use_distinct_banks(g, v):
    L = lib()
    for nt in range(4):
        banks = set()
        for lane in range(64):
            lk, li = lane >> 4, lane & 15
            row = L.fold_group_index(g, lk, v)
            banks.add((row * LDW + nt * 16 + li) % 64)
        assert len(banks) == 64
