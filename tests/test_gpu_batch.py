"""Batched reconstruction / fill-holes: every image of a batch must equal the
oracle and the same image run alone (bit-exact), also through a HIP graph
replayed several times and under autotuned settings."""
import numpy as np
import pytest

import oracle
from paper_1311_0378_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import DEV, first_mismatch  # noqa: E402
from paper_1311_0378_amd import mrecon  # noqa: E402


def make_batch(n, dt="u8", seed=0, fill_frac=0.3, lo=16, hi=400):
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        H, W = (int(v) for v in np.exp(rng.uniform(np.log(lo), np.log(hi), 2)).round())
        fill = rng.random() < fill_frac
        mask = synth.quantize(synth.make_field(H, W, synth.density_disks(H, W) + 1,
                                               seed * 1000 + i, 0.3 if fill else 0.0), dt)
        if fill:
            jobs.append(("fill", synth.binary_from_mask(mask), None))
        else:
            jobs.append(("recon", synth.marker_from_mask(mask), mask))
    return jobs


def oracle_of(job, conn):
    kind, a, m = job
    return (oracle.recon_dilate(a, m, conn) if kind == "recon" else oracle.fill_holes(a, conn))[0]


def to_items(jobs, pad=0):
    items = []
    for kind, a, m in jobs:
        d = torch.from_numpy(a).to(DEV)
        items.append((d, torch.from_numpy(m).to(DEV) if m is not None else None,
                      mrecon.MR_OP_RECON if kind == "recon" else mrecon.MR_OP_FILL))
    return items


@pytest.mark.parametrize("dt", ["u8", "i32"])
@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("tune", [None, dict(sweep_rounds=3), dict(sweep_rounds=1, max_sweeps=1),
                                  dict(sweep_rounds=-1, tail_rounds=2)], ids=str)
def test_batch_matches_oracle(dt, conn, tune):
    jobs = make_batch(24, dt, seed=conn)
    items = to_items(jobs)
    print(f"[gpu] batch of {len(items)} {dt} conn{conn} tune={tune}", flush=True)
    mrecon.batch(items, conn, tune=tune)
    torch.cuda.synchronize()
    for i, (job, (d, _, _)) in enumerate(zip(jobs, items)):
        got, want = d.cpu().numpy(), oracle_of(job, conn)
        assert np.array_equal(got, want), f"image {i} ({job[0]} {got.shape}): " + first_mismatch(got, want)


def test_batch_equals_single_calls():
    jobs = make_batch(12, "u8", seed=7)
    items = to_items(jobs)
    mrecon.batch(items, 8)
    for (kind, a, m), (d, _, _) in zip(jobs, items):
        s = torch.from_numpy(a).to(DEV)
        if kind == "recon":
            mrecon.recon_dilate(s, torch.from_numpy(m).to(DEV), 8)
        else:
            mrecon.fill_holes(s, 8)
        assert torch.equal(s, d)


@pytest.mark.parametrize("tune", [dict(sweep_rounds=6), dict(sweep_rounds=-1, tail_rounds=3)],
                         ids=["rounds+queue", "rounds+tile_queue"])
def test_graph_replays(tune):
    jobs = make_batch(16, "u8", seed=3)
    wants = [oracle_of(j, 8) for j in jobs]
    items = to_items(jobs)
    src = [d.clone() for d, _, _ in items]
    g = mrecon.BatchGraph(items, 8, tune=tune)
    for rep in range(3):
        for (d, _, _), s in zip(items, src):
            d.copy_(s)  # eager work between replays
        torch.cuda.synchronize()
        print(f"[gpu] graph replay {rep}", flush=True)
        g.launch()
        torch.cuda.synchronize()
        for i, ((d, _, _), w) in enumerate(zip(items, wants)):
            got = d.cpu().numpy()
            assert np.array_equal(got, w), f"replay {rep} image {i}: " + first_mismatch(got, w)
    g.close()


def test_autotune_restores_and_tunes():
    jobs = make_batch(10, "u8", seed=5)
    items = to_items(jobs)
    before = [d.clone() for d, _, _ in items]
    t = mrecon.autotune(items, 8)
    for b, (d, _, _) in zip(before, items):
        assert torch.equal(b, d), "the autotuner must leave the data as it found it"
    assert t.sweep_rounds != 0 and t.max_sweeps >= 1
    mrecon.batch(items, 8, tune=t)
    for i, (job, (d, _, _)) in enumerate(zip(jobs, items)):
        assert np.array_equal(d.cpu().numpy(), oracle_of(job, 8)), f"image {i}"


def test_autotune_cache_stores_then_reuses(tmp_path):
    import json
    jobs = make_batch(6, "u8", seed=9)
    items = to_items(jobs)
    path = str(tmp_path / "tunes.json")
    t1 = mrecon.autotune(items, 8, cache=path)          # timed, then stored
    stored = json.load(open(path))
    key = mrecon.tune_cache_key(items, 8)
    assert stored[key]["tail_rounds"] == t1.tail_rounds
    assert stored[key]["first_sweeps"] == t1.first_sweeps
    t2 = mrecon.autotune(items, 8, cache=path)          # taken from the cache
    assert all(getattr(t1, f) == getattr(t2, f) for f, _ in mrecon.Tune._fields_)
    mrecon.batch(items, 8, tune=t2)
    for i, (job, (d, _, _)) in enumerate(zip(jobs, items)):
        assert np.array_equal(d.cpu().numpy(), oracle_of(job, 8)), f"image {i}"
