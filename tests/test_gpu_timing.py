"""Per-launch timing (mr_timing_*): one record per tile-round, seed and queue
launch, in launch order, with positive device times."""
import pytest

from paper_1311_0378_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # collected on CPU-only hosts too
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import gpu_recon  # noqa: E402
from paper_1311_0378_amd import mrecon  # noqa: E402


@pytest.mark.parametrize("tune", [dict(sweep_rounds=-1, tail_rounds=0),
                                  dict(sweep_rounds=2, max_sweeps=2),
                                  dict(sweep_rounds=-1, tail_rounds=2), None],
                         ids=["converge", "rounds+queue", "rounds+tile_queue", "default"])
def test_timing_records_every_launch(tune):
    marker, mask = synth.make_tile(700, 900, 130, 5, "u8", 0.0)
    mrecon.timing_enable(True)
    try:
        out, c = gpu_recon(marker, mask, 8, tune=tune, counters=True)
    finally:
        mrecon.timing_enable(False)
    recs = mrecon.timing_collect()
    tiles = [r for r in recs if r[0] == "tile_round"]
    assert [r[1] for r in tiles] == list(range(1, c["rounds"] + 1))
    assert all(r[3] == 1 for r in recs)
    kinds = [r[0] for r in recs]
    if tune is None or tune.get("tail_rounds", 0) > 0:
        # rounds, then the tile queue (the default: 8 rounds)
        assert c["rounds"] == (tune or {}).get("tail_rounds", 8)
        assert kinds == ["tile_round"] * c["rounds"] + ["tile_queue"]
    elif tune["sweep_rounds"] < 0:
        assert kinds == ["tile_round"] * c["rounds"]
    else:
        assert kinds == ["tile_round"] * 2 + ["seed", "queue"]
    assert all(ms > 0.0 for _, _, ms, _ in recs)
    assert mrecon.timing_collect() == []


@pytest.mark.parametrize("tune", [dict(sweep_rounds=-1, tail_rounds=0),
                                  dict(sweep_rounds=3, max_sweeps=2), None],
                         ids=["converge", "rounds+queue", "default"])
def test_timing_spans(tune):
    """Span mode: one record per run of consecutive tile rounds between host
    waits, covering every round exactly once; other launches as before."""
    marker, mask = synth.make_tile(700, 900, 130, 5, "u8", 0.0)
    mrecon.timing_enable("spans")
    try:
        out, c = gpu_recon(marker, mask, 8, tune=tune, counters=True)
    finally:
        mrecon.timing_enable(False)
    recs = mrecon.timing_collect()
    spans = [r for r in recs if r[0] == "tile_round"]
    covered = [r for kind, first, _, n in spans for r in range(first, first + n)]
    assert covered == list(range(1, c["rounds"] + 1))
    if tune is None or tune.get("tail_rounds", 0) > 0 or tune["sweep_rounds"] > 0:
        assert len(spans) == 1  # no host wait between the rounds
    else:
        # round 1 and then 8 rounds before each host poll
        assert len(spans) == max(1, -(-(c["rounds"] - 1) // 8))
    others = [r[0] for r in recs if r[0] != "tile_round"]
    if tune is None:
        assert others == ["tile_queue"]
    elif tune["sweep_rounds"] > 0:
        assert others == ["seed", "queue"]
    assert all(ms > 0.0 for _, _, ms, _ in recs)


def test_timing_off_records_nothing():
    marker, mask = synth.make_tile(300, 300, 20, 6, "u8", 0.0)
    gpu_recon(marker, mask, 8)
    assert mrecon.timing_collect() == []
