"""CPU replay of the union rules of the GPU CCL (local phase and border
merge), against scipy's labelling.

The GPU kernels do not link every pixel with every backward neighbour:
a pixel starts at its horizontal run's first pixel, and a run makes one
union per run above it that it touches; the border merge applies the same
rule along each tile's first row and keeps the column rules whole. This test
restates those rules in plain Python on small multi-tile images and checks
that they give the same partition as a full labelling, with every label the
component's smallest linear index + 1 (the labels the GPU path returns).
The kernels themselves are compared with the oracle in test_gpu_ops.py."""
import numpy as np
import pytest
from scipy import ndimage

TH, TW = 32, 64  # the local phase's tile


def _structure(conn):
    return ndimage.generate_binary_structure(2, 1 if conn == 4 else 2)


def _run_rules(fg, conn):
    H, W = fg.shape
    F = np.zeros(H * W, np.int64)  # parent + 1, 0 = background

    def find(a):
        while F[a] - 1 != a:
            a = F[a] - 1
        return a

    def union(a, b):
        a, b = find(a), find(b)
        if a != b:
            a, b = min(a, b), max(a, b)
            F[b] = a + 1

    def above_rules(p, left, aL, aC, aR, up):
        # one union per run above that the run of p touches
        if conn == 4:
            if aC and not (left and aL):
                union(p, p - up)
        else:
            if not left:
                if aL:
                    union(p, p - up - 1)
                if aC and not aL:
                    union(p, p - up)
            if aR and not aC:
                union(p, p - up + 1)

    # local phase, tile by tile
    for y0 in range(0, H, TH):
        for x0 in range(0, W, TW):
            for y in range(y0, min(y0 + TH, H)):
                for x in range(x0, min(x0 + TW, W)):
                    if fg[y, x]:
                        s = x
                        while s > x0 and fg[y, s - 1]:
                            s -= 1
                        F[y * W + x] = y * W + s + 1
            for y in range(y0 + 1, min(y0 + TH, H)):
                for x in range(x0, min(x0 + TW, W)):
                    if not fg[y, x]:
                        continue
                    x1 = min(x0 + TW, W) - 1
                    above_rules(y * W + x, x > x0 and fg[y, x - 1], x > x0 and fg[y - 1, x - 1],
                                fg[y - 1, x], x < x1 and fg[y - 1, x + 1], W)
    # border merge
    for y0 in range(0, H, TH):
        for x0 in range(0, W, TW):
            for y in range(y0, min(y0 + TH, H)):
                for x in range(x0, min(x0 + TW, W)):
                    first_row, first_col = y == y0, x == x0
                    last_col = x == x0 + TW - 1
                    if not (first_row or first_col or last_col) or not fg[y, x]:
                        continue
                    p = y * W + x
                    if first_col and x > 0 and fg[y, x - 1]:
                        union(p, p - 1)
                    if first_row and y > 0:
                        above_rules(p, x > x0 and fg[y, x - 1], x > 0 and fg[y - 1, x - 1],
                                    fg[y - 1, x], x + 1 < W and fg[y - 1, x + 1], W)
                    elif conn == 8 and y > 0:
                        if first_col and x > 0 and fg[y - 1, x - 1]:
                            union(p, p - W - 1)
                        if last_col and x + 1 < W and fg[y - 1, x + 1]:
                            union(p, p - W + 1)
    out = np.zeros(H * W, np.int64)
    for q in np.flatnonzero(F):
        out[q] = find(q) + 1
    return out.reshape(H, W)


@pytest.mark.parametrize("conn", [4, 8])
def test_run_rules_match_full_labelling(conn):
    rng = np.random.default_rng(conn)
    for _ in range(12):
        H, W = int(rng.integers(1, 100)), int(rng.integers(1, 200))
        fg = rng.random((H, W)) < rng.uniform(0.2, 0.8)
        ref, n = ndimage.label(fg, _structure(conn))
        got = _run_rules(fg, conn)
        assert len(set(zip(ref[fg].tolist(), got[fg].tolist()))) == n
        assert len(set(got[fg].tolist())) == n
        for lab in set(got[fg].tolist()):
            assert np.flatnonzero(got.ravel() == lab).min() + 1 == lab


@pytest.mark.parametrize("conn", [4, 8])
def test_run_rules_runs_touching_at_one_end(conn):
    # runs that meet only at a run's last pixel, across a tile border: the
    # right-hand rule and the first-row merge must join them
    fg = np.zeros((40, 70), bool)
    fg[33, 10:20] = True   # a run below a tile border
    fg[32, 19:30] = True   # touches it only at its right end (first row of the lower tile)
    fg[31, 29] = True      # and the row above the border
    ref, n = ndimage.label(fg, _structure(conn))
    got = _run_rules(fg, conn)
    assert len(set(got[fg].tolist())) == n
