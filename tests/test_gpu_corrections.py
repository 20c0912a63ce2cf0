"""GPU parity of the pre-gridding visibility corrections (blink_image_batch_corrected):
per-antenna solutions and the phase-centre rotation with the w term, against the FP64 oracle.

The GPU evaluates each corrected visibility in FP64 and rounds it once to complex64, so the
images meet the FP32 bar of the uncorrected path (rel-L2 <= 1e-5 per image); weight sums and
out-of-grid counts are untouched by the corrections and stay bit-exact. The synthetic array is
coplanar (w = 0), so every case here adds random w components to exercise the w term.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from image_checks import rel_l2
from paper_2505_15204_amd import synth

pytestmark = pytest.mark.gpu

IMAGE_TOL = 1e-5
SPLIT_TOL = 1e-3


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


def with_w(prob, seed, scale=30.0):
    """The problem's baselines with random w components (metres), fixed per baseline."""
    uvw = prob.uvw_m.copy()
    w = np.random.default_rng(seed).uniform(-scale, scale, size=uvw.shape[1])
    uvw[:, :, 2] = w[None, :]
    return uvw


def random_gains(seed, C, P, A):
    g = np.random.default_rng(seed)
    return (g.uniform(0.5, 1.5, size=(C, P, A)) * np.exp(2j * np.pi * g.uniform(size=(C, P, A)))).astype(np.complex64)


def dev(torch, a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


SMALL = lambda N, w, nt=11: synth.Spec(f"small-{N}", 31, nt, 2, 2, np.array([140.0e6, 155.5e6, 171.25e6]), N, 4.5e-4,
                                       3, 0.15, weighting=w)
CASES = [
    # name, spec, gains?, (l0, m0)
    ("small-64-natural", SMALL(64, 0), True, (0.012, -0.02)),
    ("small-32-uniform", SMALL(32, 1), True, (-0.03, 0.004)),
    ("small-64-gains-only", SMALL(64, 0), True, (0.0, 0.0)),
    ("small-64-rotation-only", SMALL(64, 1), False, (0.05, 0.05)),
    ("tiny-256", synth.spec_tiny(), True, (0.01, 0.02)),
    ("vcs-1024-1x2x2", synth.spec_vcs(T=1, C=2, P=2), True, (0.02, -0.015)),
    ("phase2-2048-uniform", synth.Spec("phase2-2048", 3, 144, 1, 2, np.array([185.005e6]), 2048, 0.75 * synth.ARCMIN,
                                       50, 0.1, weighting=1), False, (-0.04, 0.01)),
]


@pytest.fixture(scope="module")
def generated():
    cache = {}

    def get(name, spec, use_gains, lm):
        if name not in cache:
            prob = synth.make_problem(spec)
            uvw = with_w(prob, 7)
            gains = random_gains(8, spec.C, spec.P, spec.n_tiles) if use_gains else None
            ref = oracle.image_batch_corrected(prob.vis, prob.flags, uvw, prob.freq_hz, spec.grid_n, spec.pixel_scale,
                                               spec.weighting, gains, lm[0], lm[1])
            cache[name] = (prob, uvw, gains, ref)
        return cache[name]
    return get


@pytest.mark.parametrize("name,spec,use_gains,lm", CASES, ids=[c[0] for c in CASES])
def test_corrected_images_match_oracle(torch, ctx, generated, name, spec, use_gains, lm):
    prob, uvw, gains, ref = generated(name, spec, use_gains, lm)
    say(f"blink_image_batch_corrected {name} N={spec.grid_n} gains={use_gains} l0,m0={lm}")
    res = ctx.blink_image_batch_corrected(dev(torch, prob.vis), dev(torch, prob.flags), dev(torch, uvw),
                                          dev(torch, prob.freq_hz), spec.grid_n, spec.pixel_scale, spec.weighting,
                                          gains=dev(torch, gains), l0=lm[0], m0=lm[1])
    torch.cuda.synchronize()
    assert np.array_equal(res["weight_sum"].cpu().numpy(), ref["weight_sum"])
    assert np.array_equal(res["n_out"].cpu().numpy(), ref["n_out"])
    img = res["images"].cpu().numpy()
    for idx in np.ndindex(spec.T, spec.C, spec.P):
        e = rel_l2(img[idx], ref["images"][idx])
        assert e <= IMAGE_TOL, (idx, e)


@pytest.mark.parametrize("prec", [1, 2], ids=["split-f16", "split-bf16"])
def test_corrected_split_precision(torch, ctx, generated, prec):
    name, spec, use_gains, lm = CASES[5]
    prob, uvw, gains, ref = generated(name, spec, use_gains, lm)
    say(f"blink_image_batch_corrected {name} precision={prec}")
    img = ctx.blink_image_batch_corrected(dev(torch, prob.vis), dev(torch, prob.flags), dev(torch, uvw),
                                          dev(torch, prob.freq_hz), spec.grid_n, spec.pixel_scale, spec.weighting,
                                          gains=dev(torch, gains), l0=lm[0], m0=lm[1],
                                          precision=prec)["images"].cpu().numpy()
    for idx in np.ndindex(spec.T, spec.C, spec.P):
        assert rel_l2(img[idx], ref["images"][idx]) <= SPLIT_TOL


def test_point_source_moves_to_phase_centre(torch, ctx):
    """A point source at (l0, m0) with the w term, rotated to (l0, m0), images at the centre pixel
    with its flux (natural weighting; the corrected visibilities are all S)."""
    spec = synth.Spec("small-128", 32, 40, 1, 1, np.array([150.0e6, 170.0e6]), 128, 1.0e-3, 1, 0.0)
    prob = synth.make_problem(spec)
    uvw = with_w(prob, 9, scale=50.0)
    l0, m0, S = 0.021, -0.034, 3.0
    n0 = math.sqrt(1.0 - l0 * l0 - m0 * m0)
    vis = np.empty((1, 2, 1, spec.B), dtype=np.complex64)
    for c, f in enumerate(spec.freq_hz):
        ph = (uvw[0, :, 0] * l0 + uvw[0, :, 1] * m0 + uvw[0, :, 2] * (n0 - 1.0)) * f / synth.C_LIGHT
        vis[0, c, 0] = S * np.exp(-2j * np.pi * ph)
    say("point source rotated to the phase centre, N=128")
    img = ctx.blink_image_batch_corrected(dev(torch, vis), None, dev(torch, uvw), dev(torch, prob.freq_hz), 128,
                                          spec.pixel_scale, 0, l0=l0, m0=m0)["images"].cpu().numpy()
    ref = oracle.image_batch_corrected(vis, None, uvw, prob.freq_hz, 128, spec.pixel_scale, 0, None, l0, m0)
    for c in range(2):
        assert abs(img[0, c, 0, 64, 64] - S) <= 1e-5 * S
        assert rel_l2(img[0, c, 0], ref["images"][0, c, 0]) <= IMAGE_TOL
        assert np.abs(img[0, c, 0]).max() <= S * (1 + 1e-5)


def test_identity_corrections_equal_plain_imaging(torch, ctx, generated):
    name, spec, _, _ = CASES[0]
    prob, uvw, _, _ = generated(name, spec, True, CASES[0][3])
    args = (dev(torch, prob.vis), dev(torch, prob.flags), dev(torch, uvw), dev(torch, prob.freq_hz), spec.grid_n,
            spec.pixel_scale, spec.weighting)
    say("identity corrections vs blink_image_batch")
    ones = torch.ones((spec.C, spec.P, spec.n_tiles), dtype=torch.complex64, device="cuda:0")
    a = ctx.blink_image_batch(*args)
    b = ctx.blink_image_batch_corrected(*args, gains=ones)
    assert torch.equal(a["weight_sum"], b["weight_sum"])
    x, y = a["images"].cpu().numpy(), b["images"].cpu().numpy()
    for idx in np.ndindex(spec.T, spec.C, spec.P):
        assert rel_l2(y[idx], x[idx]) <= 1e-6


def test_corrected_chunked_and_degenerate(torch, ctx, generated):
    import paper_2505_15204_amd as blink
    name, spec, use_gains, lm = CASES[0]
    prob, uvw, gains, ref = generated(name, spec, use_gains, lm)
    args = (dev(torch, prob.vis), dev(torch, prob.flags), dev(torch, uvw), dev(torch, prob.freq_hz), spec.grid_n,
            spec.pixel_scale, spec.weighting)
    say("corrected, one (t,c) pair per chunk")
    one = blink.image_batch_corrected_workspace_size(1, 1, spec.P, spec.B, spec.grid_n, spec.weighting)
    ws = torch.empty(one, dtype=torch.uint8, device="cuda:0")
    img = ctx.blink_image_batch_corrected(*args, gains=dev(torch, gains), l0=lm[0], m0=lm[1],
                                          workspace=ws)["images"].cpu().numpy()
    for idx in np.ndindex(spec.T, spec.C, spec.P):
        assert rel_l2(img[idx], ref["images"][idx]) <= IMAGE_TOL
    say("corrected, no baselines")
    r = ctx.blink_image_batch_corrected(args[0][..., :0].contiguous(), args[1][..., :0].contiguous(),
                                        args[2][:, :0].contiguous(), args[3], spec.grid_n, spec.pixel_scale, 0,
                                        l0=0.01, m0=0.0)
    assert not r["images"].any()
    say("corrected, bad arguments")
    with pytest.raises(blink.BlinkError):
        ctx.blink_image_batch_corrected(*args, gains=dev(torch, gains[..., :-1]))
    with pytest.raises(blink.BlinkError):
        ctx.blink_image_batch_corrected(*args, l0=0.9, m0=0.5)
