"""The atomic-rate probe (mr_probe_atomics): every operation lands exactly
once, under no contention and under heavy contention, and the addresses are
spread over the buffer. The random-access probe (mr_probe_random): every lane's
read sum and every written word match a numpy recomputation from the same
index vector."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # collected on CPU-only hosts too
    pytest.skip("no GPU", allow_module_level=True)

from paper_1311_0378_amd import mrecon  # noqa: E402


@pytest.mark.parametrize("kind", [mrecon.MR_PROBE_ADD, mrecon.MR_PROBE_CAS], ids=["add", "cas"])
@pytest.mark.parametrize("n_words,waves,per_lane", [(1 << 20, 1024, 32), (64, 64, 8),
                                                    (1 << 16, 3, 1)])
def test_probe_counts_every_operation(kind, n_words, waves, per_lane):
    print(f"[gpu] probe kind={kind} n_words={n_words} waves={waves} per_lane={per_lane}",
          flush=True)
    words = torch.zeros(n_words, dtype=torch.int32, device="cuda:0")
    mrecon.probe_atomics(words, kind, per_lane, waves, seed=7)
    torch.cuda.synchronize()
    total = waves * 64 * per_lane
    w = words.cpu().to(torch.int64)
    assert int(w.sum()) == total
    assert int(w.min()) >= 0
    if n_words == 1 << 20:
        # about 2 operations per word: a uniform spread leaves ~1 - e^-2 of the words touched
        touched = int((w > 0).sum()) / n_words
        assert touched > 0.8, touched


def test_probe_twice_adds_up():
    words = torch.zeros(1 << 12, dtype=torch.int32, device="cuda:0")
    mrecon.probe_atomics(words, mrecon.MR_PROBE_CAS, 4, 16, seed=1)
    mrecon.probe_atomics(words, mrecon.MR_PROBE_ADD, 2, 8, seed=2)
    torch.cuda.synchronize()
    assert int(words.cpu().to(torch.int64).sum()) == 16 * 64 * 4 + 8 * 64 * 2


def _lane_sums(words_np, idx_np, lanes):
    """Per-lane wrapping 32-bit sums: lane g reads the operations g, g + lanes, ..."""
    n = idx_np.size
    pos = idx_np.astype(np.int64) & (words_np.size - 1)
    vals = np.zeros(((n + lanes - 1) // lanes) * lanes, dtype=np.uint64)
    vals[:n] = words_np.astype(np.uint32)[pos]
    return (vals.reshape(-1, lanes).sum(axis=0) & 0xFFFFFFFF).astype(np.uint32)


@pytest.mark.parametrize("log2_words,n_ops,waves", [(16, 100003, 37), (6, 1000, 1),
                                                    (20, 1 << 20, 512), (12, 1, 3),
                                                    (24, 3 * 64 * 8 + 5, 3)])
def test_probe_random_read_sums(log2_words, n_ops, waves):
    print(f"[gpu] random read n_words=2^{log2_words} n_ops={n_ops} waves={waves}", flush=True)
    rng = np.random.default_rng(log2_words * 1000 + waves)
    words_np = rng.integers(0, 1 << 32, 1 << log2_words, dtype=np.uint64).astype(np.uint32)
    # indices beyond the matrix are taken modulo its size
    idx_np = rng.integers(0, 1 << 32, n_ops, dtype=np.uint64).astype(np.uint32)
    words = torch.from_numpy(words_np.view(np.int32)).to("cuda:0")
    idx = torch.from_numpy(idx_np.view(np.int32)).to("cuda:0")
    sums = torch.full((waves * 64,), -1, dtype=torch.int32, device="cuda:0")
    mrecon.probe_random(words, idx, mrecon.MR_RANDOM_READ, waves, sums)
    torch.cuda.synchronize()
    got = sums.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got, _lane_sums(words_np, idx_np, waves * 64))
    np.testing.assert_array_equal(words.cpu().numpy().view(np.uint32), words_np)  # not written


@pytest.mark.parametrize("log2_words,waves", [(14, 5), (18, 64)])
def test_probe_random_write_permutation(log2_words, waves):
    """Distinct positions: every word ends up holding its operation's number."""
    print(f"[gpu] random write permutation n_words=2^{log2_words} waves={waves}", flush=True)
    n = 1 << log2_words
    rng = np.random.default_rng(log2_words)
    perm = rng.permutation(n).astype(np.uint32)
    high = rng.integers(0, 1 << (32 - log2_words), n, dtype=np.uint64).astype(np.uint32)
    idx_np = perm | (high << log2_words)  # the same positions, modulo n
    words = torch.full((n,), -7, dtype=torch.int32, device="cuda:0")
    idx = torch.from_numpy(idx_np.view(np.int32)).to("cuda:0")
    mrecon.probe_random(words, idx, mrecon.MR_RANDOM_WRITE, waves)
    torch.cuda.synchronize()
    expect = np.empty(n, dtype=np.uint32)
    expect[perm] = np.arange(n, dtype=np.uint32)
    np.testing.assert_array_equal(words.cpu().numpy().view(np.uint32), expect)


def test_probe_random_write_with_repeats():
    """Repeated positions: each written word holds the number of one of the
    operations aimed at it; untouched words keep their value."""
    n, n_ops, waves = 1 << 12, 50000, 7
    print(f"[gpu] random write repeats n_words={n} n_ops={n_ops} waves={waves}", flush=True)
    rng = np.random.default_rng(5)
    idx_np = rng.integers(0, n - 100, n_ops, dtype=np.uint32)  # the last 100 words untouched
    words = torch.full((n,), -7, dtype=torch.int32, device="cuda:0")
    idx = torch.from_numpy(idx_np.view(np.int32)).to("cuda:0")
    mrecon.probe_random(words, idx, mrecon.MR_RANDOM_WRITE, waves)
    torch.cuda.synchronize()
    got = words.cpu().numpy().view(np.uint32)
    assert (got[n - 100:] == np.uint32(0xFFFFFFF9)).all()
    ops = got[: n - 100].astype(np.int64)
    touched = np.zeros(n - 100, dtype=bool)
    touched[idx_np] = True
    assert (ops[~touched] == 0xFFFFFFF9).all()
    assert (ops[touched] < n_ops).all()
    assert (idx_np[ops[touched]] == np.nonzero(touched)[0]).all()
