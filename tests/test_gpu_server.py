"""Continuous-batching server: jobs that arrive while others are on the GPU
join the next tile round; every job's result must equal the oracle and the
same job run alone (tolerance 0), admission must back off when the arena is
full and refuse jobs that can never fit."""
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
from test_gpu_batch import make_batch, oracle_of  # noqa: E402


def alone(job, conn):
    kind, a, m = job
    d = torch.from_numpy(a).to(DEV)
    if kind == "recon":
        mrecon.recon_dilate(d, torch.from_numpy(m).to(DEV), conn)
    else:
        mrecon.fill_holes(d, conn)
    return d.cpu().numpy()


def run_server(jobs, arena, conn=8, per_step=3, dtype=torch.uint8, max_jobs=16, rounds=None):
    srv = mrecon.Server(arena, max_jobs=max_jobs, dtype=dtype, conn=conn, rounds_per_step=rounds)
    pending = list(enumerate(jobs))
    ids, results, eagain = {}, {}, 0
    steps = 0
    while pending or srv.stats()["resident"]:
        # a few arrivals per step, so new jobs join rounds already running
        for _ in range(per_step):
            if not pending:
                break
            i, (kind, a, m) = pending[0]
            jid = srv.submit(a, m if kind == "recon" else None)
            if jid is None:
                eagain += 1
                break
            ids[jid] = i
            pending.pop(0)
        srv.step()
        steps += 1
        for jid, res in srv.poll():
            results[ids[jid]] = res.numpy()
        assert steps < 100000
    srv.close()
    return results, eagain


@pytest.mark.parametrize("rounds", [1, 2, 3, None], ids=lambda r: f"rounds{r}")
@pytest.mark.parametrize("conn", [4, 8])
def test_server_results_equal_alone_and_oracle(conn, rounds):
    jobs = make_batch(30, "u8", seed=11 + conn, lo=20, hi=600)
    print(f"[gpu] server 30 jobs conn{conn} rounds/step {rounds}", flush=True)
    results, _ = run_server(jobs, 256 << 20, conn=conn, rounds=rounds)
    assert len(results) == len(jobs)
    for i, job in enumerate(jobs):
        want = oracle_of(job, conn)
        assert np.array_equal(results[i], want), f"job {i}: " + first_mismatch(results[i], want)
        assert np.array_equal(results[i], alone(job, conn)), f"job {i} differs from its solo run"


def test_server_i32():
    jobs = make_batch(12, "i32", seed=4, lo=20, hi=300)
    results, _ = run_server(jobs, 128 << 20, dtype=torch.int32)
    for i, job in enumerate(jobs):
        assert np.array_equal(results[i], oracle_of(job, 8)), f"job {i}"


def test_server_backpressure_and_reject():
    # 16 jobs of about 7 MiB in all through a 3 MiB arena
    jobs = make_batch(16, "u8", seed=2, lo=200, hi=900)
    results, eagain = run_server(jobs, 3 << 20, per_step=16)
    assert eagain > 0, "a small arena must push back"
    assert len(results) == len(jobs)
    for i, job in enumerate(jobs):
        assert np.array_equal(results[i], oracle_of(job, 8)), f"job {i}"
    srv = mrecon.Server(8 << 20, max_jobs=4)
    big = np.zeros((4000, 4000), np.uint8)
    with pytest.raises(mrecon.MrError) as e:
        srv.submit(big, big)
    assert e.value.code == mrecon.MR_EINVAL
    srv.close()


def test_server_windows_of_a_larger_image():
    # jobs given as windows of one pinned image (host row pitch > width),
    # results written into windows of one pinned output
    big_m, big_k = synth.make_tile(700, 900, 60, 5, "u8", 0.0)
    big_f = synth.binary_from_mask(synth.quantize(synth.make_field(700, 900, 60, 6, 0.3), "u8"))
    tm, tk, tf = (torch.from_numpy(x).pin_memory() for x in (big_m, big_k, big_f))
    out = torch.zeros((700, 900), dtype=torch.uint8, pin_memory=True)
    outf = torch.zeros((700, 900), dtype=torch.uint8, pin_memory=True)
    wins = [(0, 0, 300, 400), (310, 17, 390, 233), (50, 500, 129, 400), (400, 300, 300, 600)]
    srv = mrecon.Server(64 << 20, max_jobs=8)
    ids = {}
    for k, (y, x, h, w) in enumerate(wins):
        sl = (slice(y, y + h), slice(x, x + w))
        ids[srv.submit(tm[sl], tk[sl], out=out[sl])] = ("recon", sl)
        ids[srv.submit(tf[sl], out=outf[sl])] = ("fill", sl)
        if k == 1:
            srv.step()
    srv.drain()
    got = dict(srv.poll())
    srv.close()
    assert sorted(got) == sorted(ids)
    for jid, (kind, sl) in ids.items():
        if kind == "recon":
            want = oracle.recon_dilate(np.ascontiguousarray(big_m[sl]),
                                       np.ascontiguousarray(big_k[sl]), 8)[0]
            src = out
        else:
            want = oracle.fill_holes(np.ascontiguousarray(big_f[sl]), 8)[0]
            src = outf
        assert np.array_equal(src[sl].numpy(), want), f"{kind} window {sl}"
        # pixels outside the windows were never written
    mask = np.zeros((700, 900), bool)
    for _, (_, sl) in ids.items():
        mask[sl] = True
    assert not out.numpy()[~mask].any() and not outf.numpy()[~mask].any()


@pytest.mark.parametrize("conn", [4, 8])
def test_server_device_jobs(conn):
    # jobs whose inputs and results are device memory (MR_JOB_DEVICE): the
    # same answers as the oracle; inputs are windows with a row pitch wider
    # than the job, results land in pitched device buffers
    jobs = make_batch(24, seed=40 + conn)
    want = [oracle_of(j, conn) for j in jobs]
    srv = mrecon.Server(256 << 20, max_jobs=8, conn=conn)
    pending = list(range(len(jobs)))
    owned, got = {}, {}
    keep = []
    print(f"[gpu] server device jobs conn{conn}", flush=True)
    while pending or owned:
        while pending:
            i = pending[0]
            kind, a, m = jobs[i]
            H, W = a.shape
            big = torch.zeros((H, W + 37), dtype=torch.uint8, device=DEV)
            big[:, :W] = torch.from_numpy(a).to(DEV)
            d = big[:, :W]
            mk = None
            if kind == "recon":
                bigm = torch.zeros_like(big)
                bigm[:, :W] = torch.from_numpy(m).to(DEV)
                mk = bigm[:, :W]
            out = torch.full((H, W + 5), 7, dtype=torch.uint8, device=DEV)[:, :W]
            jid = srv.submit(d, mk, out=out)
            if jid is None:
                break
            keep.append((big, mk, out))
            owned[jid] = i
            pending.pop(0)
        srv.step()
        for jid, res in srv.poll():
            got[owned.pop(jid)] = res.cpu().numpy()
    srv.close()
    for i in range(len(jobs)):
        assert np.array_equal(got[i], want[i]), f"job {i}: " + first_mismatch(got[i], want[i])
