"""GPU parity of the split-precision matrix-core FFT forms (BLINK_PREC_SPLIT_F16 / _BF16) against the
FP64 oracle, through the C ABI.

Bar for the reduced-precision forms: relative L2 <= 1e-3 per image, relative error <= 1e-3 at
the peak pixel, and the 6-sigma detections (local maxima above 6 x the oracle image's robust
sigma) at exactly the same pixels. Gridding is FP32 in every form, so weight sums and
out-of-grid counts stay bit-exact. The measured errors are printed per case.
"""
import sys

import numpy as np
import pytest

import oracle
from image_checks import peak_error, recovery, rel_l2
from paper_2505_15204_amd import synth

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-3
SPLITS = [(1, "split-f16"), (2, "split-bf16")]


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


def check_image(got, ref, what):
    e, pk = rel_l2(got, ref), peak_error(got, ref)
    missing, spurious = recovery(got, ref)
    say(f"  {what}: rel_l2={e:.3e} peak={pk:.3e} missing={len(missing)} spurious={len(spurious)}")
    assert np.isfinite(got).all(), what
    assert e <= MIXED_TOL, (what, e)
    assert pk <= MIXED_TOL, (what, pk)
    assert not missing and not spurious, (what, sorted(missing)[:5], sorted(spurious)[:5])
    return e


@pytest.mark.parametrize("prec,pname", SPLITS, ids=[s[1] for s in SPLITS])
@pytest.mark.parametrize("N", [8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
def test_split_ifft2d_random_grids(torch, ctx, N, prec, pname):
    say(f"blink_ifft2d {pname} random grids N={N}")
    g = np.random.default_rng(100 + N)
    n = 3 if N <= 1024 else 1
    G = (g.normal(size=(n, N, N)) + 1j * g.normal(size=(n, N, N))).astype(np.complex64)
    W = np.array([2.5, 1.0, 7.0][:n])
    dev = torch.from_numpy(G).to("cuda:0")
    for shift in (True, False):
        out = ctx.blink_ifft2d(dev, torch.from_numpy(W).to("cuda:0"), shift=shift, precision=prec).cpu().numpy()
        for i in range(n):
            ref, _ = oracle.ifft2d(G[i], W[i], shift=shift)
            e = rel_l2(out[i], ref)
            say(f"  N={N} shift={shift} img={i}: rel_l2={e:.3e}")
            assert e <= MIXED_TOL, (N, shift, i, e)


def split_problems():
    return [
        ("small-64-natural", synth.Spec("small-64", 11, 30, 1, 2, np.array([140.0e6, 155.5e6]), 64, 4.5e-4, 3, 0.15)),
        ("small-32-uniform", synth.Spec("small-32", 11, 20, 1, 1, np.array([171.25e6]), 32, 4.5e-4, 3, 0.15,
                                        weighting=1)),
        ("tiny-256", synth.spec_tiny()),
        ("vcs-1024-1x3x2", synth.spec_vcs(T=1, C=3, P=2)),
        ("phase2-2048-uniform-1x2x2", synth.spec_phase2(T=1, C=2, P=2)),
        ("precision-4096-1x2", synth.spec_precision(T=1, C=2)),
    ]


PROBLEMS = split_problems()


@pytest.fixture(scope="module")
def generated():
    cache = {}

    def get(name, spec):
        if name not in cache:
            prob = synth.make_problem(spec)
            ref = oracle.image_batch(prob.vis, prob.flags, prob.uvw_m, prob.freq_hz, spec.grid_n, spec.pixel_scale,
                                     spec.weighting)
            cache[name] = (prob, ref)
        return cache[name]
    return get


def to_device(torch, prob):
    d = "cuda:0"
    return (torch.from_numpy(prob.vis).to(d), torch.from_numpy(prob.flags).to(d),
            torch.from_numpy(prob.uvw_m).to(d), torch.from_numpy(prob.freq_hz).to(d))


@pytest.mark.parametrize("prec,pname", SPLITS, ids=[s[1] for s in SPLITS])
@pytest.mark.parametrize("name,spec", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_split_image_batch(torch, ctx, generated, name, spec, prec, pname):
    prob, ref = generated(name, spec)
    say(f"blink_image_batch {pname} {name} T={spec.T} C={spec.C} P={spec.P} N={spec.grid_n} w={spec.weighting}")
    vis, flags, uvw, freq = to_device(torch, prob)
    res = ctx.blink_image_batch(vis, flags, uvw, freq, spec.grid_n, spec.pixel_scale, spec.weighting, precision=prec)
    torch.cuda.synchronize()
    assert np.array_equal(res["weight_sum"].cpu().numpy(), ref["weight_sum"])
    assert np.array_equal(res["n_out"].cpu().numpy(), ref["n_out"])
    img = res["images"].cpu().numpy()
    for idx in np.ndindex(spec.T, spec.C, spec.P):
        check_image(img[idx], ref["images"][idx], f"{name} {idx}")


@pytest.mark.parametrize("prec,pname", SPLITS, ids=[s[1] for s in SPLITS])
def test_split_every_plan(torch, ctx, generated, prec, pname):
    """Every compiled (strip width, row block) variant of the split kernels at 1024^2 and 4096^2, and
    four strips per column workgroup."""
    import paper_2505_15204_amd as blink
    for name, spec in (PROBLEMS[3], PROBLEMS[5]):
        prob, ref = generated(name, spec)
        vis, flags, uvw, freq = to_device(torch, prob)
        N = spec.grid_n
        cols, rows = blink.plan_options(N, spec.weighting)
        saved = ctx.get_plan(N, spec.weighting, prec)
        try:
            for col in cols:
                for row, loop in [(r, 1) for r in rows] + [(rows[0], 4)]:
                    say(f"{pname} plan N={N} col={col} row={row} col_loop={loop}")
                    ctx.set_plan(N, spec.weighting, col, row, 0, precision=prec, col_loop=loop)
                    img = ctx.blink_image_batch(vis, flags, uvw, freq, N, spec.pixel_scale, spec.weighting,
                                                precision=prec)["images"].cpu().numpy()
                    for idx in np.ndindex(spec.T, spec.C, spec.P):
                        assert rel_l2(img[idx], ref["images"][idx]) <= MIXED_TOL, (col, row, loop, idx)
        finally:
            ctx.set_plan(N, spec.weighting, saved["col_strip"], saved["row_block"], saved["group"], precision=prec,
                         col_loop=saved["col_loop"])


def test_split_grid_zero_and_huge_values(torch, ctx):
    """FP16 range handling: an all-zero grid gives a zero image; grids scaled by 2^60 and 2^-60
    give the scaled images (the per-block power-of-two scaling keeps FP16 in range)."""
    N = 256
    g = np.random.default_rng(11)
    G = (g.normal(size=(1, N, N)) + 1j * g.normal(size=(1, N, N))).astype(np.complex64)
    for prec, pname in SPLITS:
        say(f"blink_ifft2d {pname} zero and scaled grids")
        z = ctx.blink_ifft2d(torch.zeros((1, N, N), dtype=torch.complex64, device="cuda:0"), None,
                             precision=prec).cpu().numpy()
        assert not z.any()
        base = ctx.blink_ifft2d(torch.from_numpy(G).to("cuda:0"), None, precision=prec).cpu().numpy()
        for s in (2.0 ** 60, 2.0 ** -60):
            out = ctx.blink_ifft2d(torch.from_numpy(G * np.float32(s)).to("cuda:0"), None,
                                   precision=prec).cpu().numpy()
            assert np.isfinite(out).all()
            assert rel_l2(out / s, base) <= 1e-6, (pname, s)


def test_split_close_to_fp32(torch, ctx, generated):
    """On the 1024^2 workload the split forms stay within their error budget of the FP32 form."""
    name, spec = PROBLEMS[3]
    prob, ref = generated(name, spec)
    vis, flags, uvw, freq = to_device(torch, prob)
    fp32 = ctx.blink_image_batch(vis, flags, uvw, freq, spec.grid_n, spec.pixel_scale, 0)["images"].cpu().numpy()
    for prec, pname in SPLITS:
        say(f"{pname} vs FP32 on {name}")
        img = ctx.blink_image_batch(vis, flags, uvw, freq, spec.grid_n, spec.pixel_scale, 0,
                                    precision=prec)["images"].cpu().numpy()
        for idx in np.ndindex(spec.T, spec.C, spec.P):
            e_split = rel_l2(img[idx], ref["images"][idx])
            e_fp32 = rel_l2(fp32[idx], ref["images"][idx])
            say(f"  {idx}: split {e_split:.3e}  fp32 {e_fp32:.3e}")
            assert rel_l2(img[idx], fp32[idx]) <= MIXED_TOL
