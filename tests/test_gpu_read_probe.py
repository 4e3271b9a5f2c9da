"""The library's read probe (a measurement kernel, no part of the method):
each wave's folded word over a seeded buffer, checked against the same fold
computed on the host, at grid sizes that leave ragged and empty workgroups."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2203_12339_amd import tlt  # noqa: E402


def _expected(words, blocks):
    """Per workgroup and wave: lanes xor the word sums of their 16-byte
    loads (zeros past the end), waves add their 64 lanes (mod 2^32)."""
    nbytes = words.size * 4
    per = -(-nbytes // blocks)
    chunk = -(-per // 4096) * 4096
    out = np.zeros(blocks * 4, np.uint64)
    for b in range(blocks):
        begin, end = chunk * b, min(nbytes, chunk * b + chunk)
        if begin >= end:
            continue
        seg = words[begin // 4:end // 4].astype(np.uint64)
        pad = -seg.size % 16384
        seg = np.concatenate([seg, np.zeros(pad, np.uint64)]).reshape(-1, 16, 256, 4)
        lane = seg.sum(axis=3) % (1 << 32)
        acc = np.bitwise_xor.reduce(lane.reshape(-1, 256), axis=0)
        out[b * 4:b * 4 + 4] = acc.reshape(4, 64).sum(axis=1) % (1 << 32)
    return out.astype(np.uint32)


@pytest.mark.parametrize("nwords,blocks", [(1 << 20, 64), (300_004, 7), (5000, 40), (0, 3)])
def test_read_probe_fold(nwords, blocks):
    rng = np.random.default_rng(nwords + blocks)
    words = rng.integers(0, 1 << 32, size=nwords, dtype=np.uint64).astype(np.uint32)
    buf = torch.from_numpy(words.view(np.int32)).to("cuda:0")
    out = torch.full((blocks * 4,), -1, dtype=torch.int32, device="cuda:0")
    tlt.read_probe(buf, out, blocks)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got, _expected(words, blocks))


def test_read_probe_rejects_ragged_length():
    buf = torch.zeros(6, dtype=torch.int32, device="cuda:0")
    out = torch.zeros(16, dtype=torch.int32, device="cuda:0")
    with pytest.raises(tlt.TltError):
        tlt.read_probe(buf, out, 4)
