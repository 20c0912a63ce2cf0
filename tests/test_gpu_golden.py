"""The hand-worked golden cases of the nearest-cell rule, run through the GPU library.

The oracle is pinned to these files (tests/oracle_pins.py); here the same rows go through the HIP
path, so the GPU's rounding (round half to even on one FP64 product, Section 6.2.4 as read by the
library) and its strict N/2 edge are checked on the cases where they decide the cell: products
that land exactly on a half (u k = +-0.5, +-1.5, +-2.5, 3.5) and cells on either side of the edge.

Every row is run at its own grid size and at a second one (8 and 256) with the pixel scale chosen
so that k = (f/c)(N dl) is the same double: the hand-worked (iu, iv) of the row then fix the
expected cell at the other size as well ((iv mod N) N + (iu mod N), kept iff |iu|, |iv| < N/2).
Visibilities are small integers, so every cell sum is exact in FP32 whatever the order of the
additions, and the grids are compared bit for bit.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle_pins import C_LIGHT, read_cell_fixture, read_tiny_fixture

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2505_15204_amd as blink
    c = blink.Context(0)
    yield c
    c.close()


def expected_cell(iu, iv, N):
    if abs(iu) >= N // 2 or abs(iv) >= N // 2:
        return -2
    return (iv % N) * N + (iu % N)


def fixture_cases():
    """Rows of cell_index_worked.txt grouped by (f, N, dl), each at its own N and at the other one
    with dl scaled so that N dl (hence k) is unchanged bit for bit."""
    groups = {}
    for f, n, dl, u, v, iu, iv, cell in read_cell_fixture():
        groups.setdefault((f, n, dl), []).append((u, v, iu, iv, cell))
    cases = []
    for (f, n, dl), rows in groups.items():
        for N in (n, 256 if n != 256 else 8):
            dlN = dl * (n / N)                     # a power-of-two ratio: N dl is the same double
            assert N * dlN == n * dl
            cases.append((f"f{f / 1e6:g}MHz-n{n}-at-N{N}", f, N, dlN, rows, N == n))
    return cases


CASES = fixture_cases()


def run_grid(torch, ctx, vis, uvw, f, N, dl, weighting, flags=None):
    d = "cuda:0"
    B = uvw.shape[0]
    v = torch.from_numpy(np.ascontiguousarray(vis.reshape(1, 1, -1, B))).to(d)
    fl = None if flags is None else torch.from_numpy(flags.reshape(1, 1, B)).to(d)
    u = torch.from_numpy(uvw.reshape(1, B, 3)).to(d)
    fr = torch.tensor([f], dtype=torch.float64, device=d)
    res = ctx.blink_grid(v, fl, u, fr, N, dl, weighting)
    torch.cuda.synchronize()
    return {k: (None if t is None else t.cpu().numpy()) for k, t in res.items()}


@pytest.mark.parametrize("name,f,N,dl,rows,own", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("weighting", [0, 1], ids=["natural", "uniform"])
def test_worked_cells_on_gpu(torch, ctx, name, f, N, dl, rows, own, weighting):
    say(f"blink_grid golden cells {name} weighting={weighting}")
    uvw = np.zeros((len(rows), 3))
    uvw[:, 0] = [r[0] for r in rows]
    uvw[:, 1] = [r[1] for r in rows]
    # distinct small integers: every cell sum is exact in FP32
    B = len(rows)
    vis = (np.arange(1, B + 1) + 1j * np.arange(B, 0, -1)).astype(np.complex64)
    got = run_grid(torch, ctx, vis, uvw, f, N, dl, weighting)
    expect = np.array([expected_cell(r[2], r[3], N) for r in rows], np.int32)
    if own:
        assert np.array_equal(expect, np.array([r[4] for r in rows], np.int32))
    assert np.array_equal(got["cell_idx"][0, 0], expect), (got["cell_idx"][0, 0], expect)
    kept = int((expect >= 0).sum())
    assert int(got["n_out"][0, 0]) == B - kept
    ref = oracle.grid(vis, None, uvw, f, N, dl, weighting)
    assert np.array_equal(ref["cell_idx"], expect)
    assert np.array_equal(got["counts"][0, 0], ref["counts"])
    assert int(got["counts"][0, 0].sum()) == 2 * kept
    assert float(got["weight_sum"][0, 0, 0]) == ref["weight_sum"]
    assert np.array_equal(got["grids"][0, 0, 0], ref["grid"][0].astype(np.complex64))


def tiny_fixture_problem():
    fx = read_tiny_fixture()
    bl = np.array([[float(x) for x in r] for r in fx["baselines"]])
    uvw = np.zeros((bl.shape[0], 3))
    uvw[:, :2] = bl[:, 0:2]
    flags = bl[:, 2].astype(np.uint8)
    vis = (bl[:, 3] + 1j * bl[:, 4]).astype(np.complex64)
    return fx, vis, flags, uvw


@pytest.mark.parametrize("weighting,wname", [(0, "natural"), (1, "uniform")])
def test_tiny_grid_n8_on_gpu(torch, ctx, weighting, wname):
    """The hand-enumerated 7-baseline N = 8 case: cells, grid, counts, W, n_out and image pixels."""
    say(f"blink_grid / blink_image_batch tiny N=8 {wname}")
    fx, vis, flags, uvw = tiny_fixture_problem()
    got = run_grid(torch, ctx, vis, uvw, C_LIGHT, 8, 1.0 / 64.0, weighting, flags)
    assert list(got["cell_idx"][0, 0]) == [int(x) for x in fx["cell_idx"][0]]
    weights = {r[0]: float(r[1]) for r in fx["weights"]}
    assert int(got["n_out"][0, 0]) == int(weights["n_out"])
    assert float(got["weight_sum"][0, 0, 0]) == weights[wname]
    expect = np.zeros(64, np.complex64)
    counts = np.zeros(64, np.int32)
    for cell, re, im, cnt in fx[f"{wname}_grid"]:
        expect[int(cell)] = float(re) + 1j * float(im)
        counts[int(cell)] = int(cnt)
    assert np.array_equal(got["grids"][0, 0, 0].reshape(-1), expect)
    assert np.array_equal(got["counts"][0, 0].reshape(-1), counts)
    # the fused path on the same inputs: the hand-worked pixels
    d = "cuda:0"
    res = ctx.blink_image_batch(torch.from_numpy(vis.reshape(1, 1, 1, -1)).to(d),
                                torch.from_numpy(flags.reshape(1, 1, -1)).to(d),
                                torch.from_numpy(uvw.reshape(1, -1, 3)).to(d),
                                torch.tensor([C_LIGHT], dtype=torch.float64, device=d), 8, 1.0 / 64.0, weighting)
    torch.cuda.synchronize()
    assert float(res["weight_sum"][0, 0, 0]) == weights[wname]
    assert int(res["n_out"][0, 0]) == int(weights["n_out"])
    img = res["images"][0, 0, 0].cpu().numpy()
    for w, x, y, val in fx["pixels"]:
        if w == wname:
            assert abs(float(img[int(y), int(x)]) - float(val)) <= 1e-6 * max(1.0, abs(float(val))), (x, y)


@pytest.mark.parametrize("weighting", [0, 1], ids=["natural", "uniform"])
def test_tiny_grid_at_n256_on_gpu(torch, ctx, weighting):
    """The same baselines on a 256 grid with k still 1/8 exactly: baseline 4 (u k = 5) is now kept;
    cells, counts, W and n_out bit-exact and the grid exact against the oracle."""
    say(f"blink_grid tiny fixture at N=256 weighting={weighting}")
    fx, vis, flags, uvw = tiny_fixture_problem()
    dl = 1.0 / 2048.0
    assert 256 * dl == 8 * (1.0 / 64.0)
    got = run_grid(torch, ctx, vis, uvw, C_LIGHT, 256, dl, weighting, flags)
    ref = oracle.grid(vis, flags, uvw, C_LIGHT, 256, dl, weighting)
    assert int(ref["cell_idx"][4]) == 5             # u k = 40/8 = 5 < 128
    assert np.array_equal(got["cell_idx"][0, 0], ref["cell_idx"])
    assert np.array_equal(got["counts"][0, 0], ref["counts"])
    assert int(got["n_out"][0, 0]) == ref["n_out"] == 0
    assert float(got["weight_sum"][0, 0, 0]) == ref["weight_sum"]
    assert np.array_equal(got["grids"][0, 0, 0], ref["grid"][0].astype(np.complex64))


def test_ties_on_many_channels(torch, ctx):
    """Exact dyadic products in every (t, c) pair of a batch: f_c = c / 2^j makes k = 2^-j / 8 exact,
    so the products are exact halves, quarters, ... and the GPU's cells must follow ties-to-even in
    every pair (u at t = 0, v at t = 1), not only in the first."""
    say("blink_grid ties over 6 channels x 2 times")
    N, dl = 64, 1.0 / 512.0                          # N dl = 1/8
    C, T = 6, 2
    freq = np.array([C_LIGHT / 2.0 ** j for j in range(C)])
    us = np.array([4.0, 12.0, 20.0, -4.0, -12.0, -20.0, 28.0, 252.0, 260.0, -252.0])   # u k/2^-j: 0.5, 1.5, ...
    B = us.size
    d = "cuda:0"
    uvw = np.zeros((T, B, 3))
    uvw[0, :, 0] = us
    uvw[1, :, 1] = us
    # channel j sees u k = us / 8 / 2^j: exact halves at j = 0, exact quarters, eighths, ... after
    vis = np.ones((T, C, 1, B), np.complex64)
    res = ctx.blink_grid(torch.from_numpy(vis).to(d), None, torch.from_numpy(uvw).to(d),
                         torch.from_numpy(freq).to(d), N, dl, 0)
    torch.cuda.synchronize()
    cells = res["cell_idx"].cpu().numpy()
    for t in range(T):
        for c in range(C):
            ref = oracle.grid(vis[t, c], None, uvw[t], freq[c], N, dl)
            assert np.array_equal(cells[t, c], ref["cell_idx"]), (t, c)
            x = us * (1.0 / 8.0) / 2.0 ** c        # exact: a power-of-two scaling of integers
            iu = np.rint(x).astype(np.int64)        # numpy's rint rounds halves to even
            kept = np.abs(iu) < N // 2
            ex = np.where(kept, (iu % N) * (N if t == 1 else 1), -2)
            assert np.array_equal(cells[t, c], ex.astype(np.int32)), (t, c, cells[t, c], ex)
