"""GPU parity of the column-extent pruning of the fused path: the half-spectrum columns beyond the
last strip that holds a placement are neither transformed nor stored by the column pass, and the
row pass reads them as zero without loading them.

The cases image uv coverages that reach only part of the half plane into a workspace filled with
0xFF bytes (NaN in every float of the intermediate), so a column that the row pass wrongly loaded
instead of treating as zero would show up as NaN or as a wrong image; a second call reuses the
workspace that a full-coverage call left behind. Bars as for the other parity tests: weight sums
and out-of-grid counts bit-exact, images within a relative L2 of 1e-5 (FP32) or the 1e-3 bars of
the split forms.
"""
import sys

import numpy as np
import pytest

import oracle
from image_checks import peak_error, rel_l2
from paper_2505_15204_amd import synth

pytestmark = pytest.mark.gpu

IMAGE_TOL = {0: 1e-5, 1: 1e-3, 2: 1e-3}
PRECS = [(0, "fp32"), (1, "split-f16"), (2, "split-bf16")]


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
def blink(torch):
    import paper_2505_15204_amd as _b
    return _b


@pytest.fixture(scope="module")
def ctx(blink):
    c = blink.Context(0)
    yield c
    c.close()


def spec(N, dl, weighting, T=1, C=3, P=2, n_tiles=40, flag_frac=0.1):
    freqs = np.array([140.0e6, 155.5e6, 171.25e6])[:C]
    return synth.Spec(f"extent-{N}", 17, n_tiles, T, P, freqs, N, dl, 3, flag_frac, weighting=weighting)


def to_device(torch, prob):
    d = "cuda:0"
    return (torch.from_numpy(prob.vis).to(d), torch.from_numpy(prob.flags).to(d),
            torch.from_numpy(prob.uvw_m).to(d), torch.from_numpy(prob.freq_hz).to(d))


def max_column(prob, N, dl):
    """Largest |ku| over the kept visibilities (the half-plane columns that carry data)."""
    k = prob.freq_hz[None, :, None] / 299792458.0 * N * dl
    u = np.rint(prob.uvw_m[:, None, :, 0] * k)
    v = np.rint(prob.uvw_m[:, None, :, 1] * k)
    keep = (np.abs(u) < N / 2) & (np.abs(v) < N / 2) & (prob.flags == 0)
    return int(np.abs(u[keep]).max()) if keep.any() else -1


def image_and_check(torch, blink, ctx, prob, N, dl, weighting, prec, ws, what):
    vis, flags, uvw, freq = to_device(torch, prob)
    res = ctx.blink_image_batch(vis, flags, uvw, freq, N, dl, weighting, precision=prec, workspace=ws)
    torch.cuda.synchronize()
    ref = oracle.image_batch(prob.vis, prob.flags, prob.uvw_m, prob.freq_hz, N, dl, weighting)
    assert np.array_equal(res["weight_sum"].cpu().numpy(), ref["weight_sum"]), what
    assert np.array_equal(res["n_out"].cpu().numpy(), ref["n_out"]), what
    got = res["images"].cpu().numpy()
    assert np.isfinite(got).all(), what
    worst = 0.0
    for idx in np.ndindex(*got.shape[:3]):
        if ref["weight_sum"][idx] == 0:
            assert not got[idx].any(), (what, idx)
            continue
        e = rel_l2(got[idx], ref["images"][idx])
        worst = max(worst, e)
        assert e <= IMAGE_TOL[prec], (what, idx, e)
        if prec:
            assert peak_error(got[idx], ref["images"][idx]) <= IMAGE_TOL[prec], (what, idx)
    say(f"  {what}: worst rel_l2 {worst:.2e}")


@pytest.mark.parametrize("prec,pname", PRECS, ids=[p[1] for p in PRECS])
@pytest.mark.parametrize("weighting", [0, 1], ids=["natural", "uniform"])
@pytest.mark.parametrize("N,dl", [(256, 1.0e-4), (1024, 2.9e-4)])
def test_partial_extent_nan_workspace(torch, blink, ctx, N, dl, weighting, prec, pname):
    s = spec(N, dl, weighting)
    prob = synth.make_problem(s)
    umax = max_column(prob, N, dl)
    say(f"extent N={N} dl={dl} {pname} weighting={weighting}: largest kept |ku| = {umax} of {N // 2}")
    assert 0 <= umax < N // 2 - 16, "the case must leave whole strips of the half plane empty"
    nbytes = blink.image_batch_workspace_size(s.T, s.C, s.P, s.B, N, weighting, prec)
    ws = torch.full((nbytes,), 0xFF, dtype=torch.uint8, device="cuda:0")
    image_and_check(torch, blink, ctx, prob, N, dl, weighting, prec, ws, "NaN-filled workspace")


@pytest.mark.parametrize("prec,pname", PRECS, ids=[p[1] for p in PRECS])
def test_partial_extent_after_full_extent(torch, blink, ctx, prec, pname):
    N = 512
    wide = synth.make_problem(spec(N, 4.5e-4, 0))
    narrow = synth.make_problem(spec(N, 0.8e-4, 0))
    say(f"extent reuse N={N} {pname}: |ku| max wide {max_column(wide, N, 4.5e-4)}, "
        f"narrow {max_column(narrow, N, 0.8e-4)}")
    nbytes = blink.image_batch_workspace_size(1, 3, 2, wide.uvw_m.shape[1], N, 0, prec)
    ws = torch.empty((nbytes,), dtype=torch.uint8, device="cuda:0")
    image_and_check(torch, blink, ctx, wide, N, 4.5e-4, 0, prec, ws, "full extent")
    image_and_check(torch, blink, ctx, narrow, N, 0.8e-4, 0, prec, ws, "partial extent, same workspace")


@pytest.mark.parametrize("prec,pname", PRECS, ids=[p[1] for p in PRECS])
@pytest.mark.parametrize("weighting", [0, 1], ids=["natural", "uniform"])
def test_no_kept_visibility_nan_workspace(torch, blink, ctx, weighting, prec, pname):
    """Channel 0 fully flagged, and (second call) every baseline beyond the grid edge: extent 0,
    nothing is stored, and those images are exactly zero with W = 0."""
    N = 256
    s = spec(N, 1.0e-4, weighting)
    prob = synth.make_problem(s)
    prob.flags[:, 0, :] = 1
    say(f"extent zero N={N} {pname} weighting={weighting}")
    nbytes = blink.image_batch_workspace_size(s.T, s.C, s.P, s.B, N, weighting, prec)
    ws = torch.full((nbytes,), 0xFF, dtype=torch.uint8, device="cuda:0")
    image_and_check(torch, blink, ctx, prob, N, 1.0e-4, weighting, prec, ws, "channel 0 all flagged")
    far = prob.uvw_m.copy()
    far[:, :, 0] = 1.0e6
    prob_far = synth.Problem(s, far, prob.freq_hz, np.zeros_like(prob.flags), prob.vis)
    ws.fill_(0xFF)
    image_and_check(torch, blink, ctx, prob_far, N, 1.0e-4, weighting, prec, ws, "all out of grid")


@pytest.mark.parametrize("prec,pname", PRECS, ids=[p[1] for p in PRECS])
def test_conv_partial_extent_nan_workspace(torch, blink, ctx, prec, pname):
    """Convolutional gridding (W = 8) skips the strips no tap reaches and the row pass reads their
    columns as zero: a partial coverage imaged into a NaN-filled workspace matches the oracle on
    the central half (the FP32 bar, or the split forms' 1e-3) and, multiplied back by the grid
    correction, on the whole image."""
    N, dl, width, beta = 256, 1.0e-4, 8, 18.4
    s = spec(N, dl, 0)
    prob = synth.make_problem(s)
    umax = max_column(prob, N, dl)
    say(f"conv extent N={N} {pname}: largest kept |ku| = {umax} of {N // 2}")
    assert umax + width < N // 2 - 16
    nbytes = blink.image_batch_conv_workspace_size(s.T, s.C, s.P, s.B, N, width)
    ws = torch.full((nbytes,), 0xFF, dtype=torch.uint8, device="cuda:0")
    vis, flags, uvw, freq = to_device(torch, prob)
    res = ctx.blink_image_batch_conv(vis, flags, uvw, freq, N, dl, width, beta, precision=prec, workspace=ws)
    torch.cuda.synchronize()
    ref = oracle.image_batch_conv(prob.vis, prob.flags, prob.uvw_m, prob.freq_hz, N, dl, width, beta)
    assert np.array_equal(res["weight_sum"].cpu().numpy(), ref["weight_sum"])
    got = res["images"].cpu().numpy()
    assert np.isfinite(got).all()
    c = oracle.conv_correction(N, width, beta, True)
    back = np.outer(c, c) / c.max() ** 2
    q = slice(N // 4, 3 * N // 4)
    for idx in np.ndindex(*got.shape[:3]):
        ec = rel_l2(got[idx][q, q], ref["images"][idx][q, q])
        ef = rel_l2(got[idx] * back, ref["images"][idx] * back)
        say(f"  {idx}: centre {ec:.2e}, corrected back {ef:.2e}")
        assert ec <= IMAGE_TOL[prec] and ef <= IMAGE_TOL[prec], (idx, ec, ef)
