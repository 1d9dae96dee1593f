"""The atomic-rate probe (mr_probe_atomics): every operation lands exactly
once, under no contention and under heavy contention, and the addresses are
spread over the buffer."""
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
