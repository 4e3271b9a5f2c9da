"""Index arithmetic of the float32 folded-lighting kernel, emulated on the
host: its permuted contraction order visits every coefficient index of a
term exactly once for every supported row length, and the B-operand reads
of one matrix step hit 64 distinct LDS banks with rows padded to 68 floats."""
import pytest

LDW = 64 + 4          # staged Lg row length in floats
CASES = [1, 2, 3, 4, 6, 7, 8, 9, 12, 16]   # Psh / 4 values the kernel compiles


@pytest.mark.parametrize("ms", CASES)
def test_contraction_order_is_a_permutation(ms):
    g4, r4 = ms // 4, ms % 4
    seen = []
    for g in range(g4):            # 16-byte loads: lane group lk, component v
        for v in range(4):
            for lk in range(4):
                seen.append(16 * g + 4 * lk + v)
    for q in range(r4):            # the leftover steps: one value per lane
        for lk in range(4):
            seen.append(16 * g4 + 4 * q + lk)
    assert sorted(seen) == list(range(4 * ms))


@pytest.mark.parametrize("g,v", [(0, 0), (1, 3), (3, 2)])
def test_b_operand_reads_use_distinct_banks(g, v):
    for nt in range(4):
        banks = set()
        for lane in range(64):
            lk, li = lane >> 4, lane & 15
            row = 16 * g + 4 * lk + v
            banks.add((row * LDW + nt * 16 + li) % 64)
        assert len(banks) == 64
