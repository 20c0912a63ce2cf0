"""GPU parity: the HIP library (called through its C ABI) against the FP64 CPU oracle.

Bars: cell indices, counts, weight sums and out-of-grid counts bit-exact; grids within a
relative L2 of 1e-6 and FP32 images within a relative L2 of 1e-5 of the FP64 oracle, per image.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2505_15204_amd import synth

pytestmark = pytest.mark.gpu

GRID_TOL = 1e-6
IMAGE_TOL = 1e-5


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


def rel_l2(a, b):
    kind = np.complex128 if (np.iscomplexobj(a) or np.iscomplexobj(b)) else np.float64
    a = np.asarray(a, kind)
    b = np.asarray(b, kind)
    nb = np.linalg.norm(b)
    if nb == 0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def small_spec(N=64, T=2, C=3, P=2, n_tiles=30, weighting=0, flag_frac=0.15, dl=4.5e-4):
    """A few tiles of the synthetic array; with dl = 4.5e-4 baselines longer than ~2.2 km fall
    outside the grid at any N, so every case has kept and dropped visibilities."""
    freqs = np.array([140.0e6, 155.5e6, 171.25e6])[:C]
    return synth.Spec(f"small-{N}", 11, n_tiles, T, P, freqs, N, dl, 3, flag_frac, weighting=weighting)


def to_device(torch, prob):
    d = "cuda:0"
    return (torch.from_numpy(prob.vis).to(d), torch.from_numpy(prob.flags).to(d),
            torch.from_numpy(prob.uvw_m).to(d), torch.from_numpy(prob.freq_hz).to(d))


def problems():
    out = [
        ("small-64-natural", small_spec()),
        ("small-64-uniform", small_spec(weighting=1)),
        ("small-8-natural", small_spec(N=8, n_tiles=12)),
        ("small-32-uniform", small_spec(N=32, n_tiles=20, weighting=1)),
        ("tiny-256", synth.spec_tiny()),
        ("vcs-1024-1x3x2", synth.spec_vcs(T=1, C=3, P=2)),
        ("phase2-2048-uniform-1x2x2", synth.spec_phase2(T=1, C=2, P=2)),
        ("precision-4096-1x1", synth.spec_precision(T=1, C=1)),
    ]
    return out


PROBLEMS = problems()


@pytest.fixture(scope="module")
def generated():
    cache = {}

    def get(name, spec):
        if name not in cache:
            cache[name] = synth.make_problem(spec, per_time_uvw_jitter=0.5 if spec.T > 1 else 0.0)
        return cache[name]
    return get


@pytest.mark.parametrize("name,spec", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_grid_parity(torch, ctx, generated, name, spec):
    prob = generated(name, spec)
    say(f"blink_grid {name} T={spec.T} C={spec.C} P={spec.P} B={spec.B} N={spec.grid_n} w={spec.weighting}")
    vis, flags, uvw, freq = to_device(torch, prob)
    res = ctx.blink_grid(vis, flags, uvw, freq, spec.grid_n, spec.pixel_scale, spec.weighting)
    torch.cuda.synchronize()
    for t in range(spec.T):
        for c in range(spec.C):
            ref = oracle.grid(prob.vis[t, c], prob.flags[t, c], prob.uvw_m[t], prob.freq_hz[c], spec.grid_n,
                              spec.pixel_scale, spec.weighting)
            assert np.array_equal(res["cell_idx"][t, c].cpu().numpy(), ref["cell_idx"])
            assert np.array_equal(res["counts"][t, c].cpu().numpy(), ref["counts"])
            assert int(res["n_out"][t, c]) == ref["n_out"]
            for p in range(spec.P):
                assert float(res["weight_sum"][t, c, p]) == ref["weight_sum"]
                g = res["grids"][t, c, p].cpu().numpy()
                assert rel_l2(g, ref["grid"][p]) <= GRID_TOL, (t, c, p, rel_l2(g, ref["grid"][p]))


@pytest.mark.parametrize("name,spec", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_image_batch_parity(torch, ctx, generated, name, spec):
    prob = generated(name, spec)
    say(f"blink_image_batch {name} T={spec.T} C={spec.C} P={spec.P} B={spec.B} N={spec.grid_n}")
    vis, flags, uvw, freq = to_device(torch, prob)
    res = ctx.blink_image_batch(vis, flags, uvw, freq, spec.grid_n, spec.pixel_scale, spec.weighting)
    torch.cuda.synchronize()
    ref = oracle.image_batch(prob.vis, prob.flags, prob.uvw_m, prob.freq_hz, spec.grid_n, spec.pixel_scale,
                             spec.weighting)
    assert np.array_equal(res["weight_sum"].cpu().numpy(), ref["weight_sum"])
    assert np.array_equal(res["n_out"].cpu().numpy(), ref["n_out"])
    img = res["images"].cpu().numpy()
    assert np.isfinite(img).all()
    for idx in np.ndindex(spec.T, spec.C, spec.P):
        e = rel_l2(img[idx], ref["images"][idx])
        assert e <= IMAGE_TOL, (idx, e)


def test_image_batch_unshifted(torch, ctx, generated):
    spec = small_spec(N=128, T=1, C=2, P=1)
    prob = generated("small-128-unshifted", spec)
    say("blink_image_batch shift=0 N=128")
    vis, flags, uvw, freq = to_device(torch, prob)
    res = ctx.blink_image_batch(vis, flags, uvw, freq, spec.grid_n, spec.pixel_scale, 0, shift=False)
    ref = oracle.image_batch(prob.vis, prob.flags, prob.uvw_m, prob.freq_hz, spec.grid_n, spec.pixel_scale,
                             0, shift=False)
    img = res["images"].cpu().numpy()
    for idx in np.ndindex(1, 2, 1):
        assert rel_l2(img[idx], ref["images"][idx]) <= IMAGE_TOL


@pytest.mark.parametrize("N", [8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
def test_ifft2d_parity_random_grids(torch, ctx, N):
    """Arbitrary (non-Hermitian) complex grids: the image is the real part of the inverse transform."""
    say(f"blink_ifft2d random grids N={N}")
    g = np.random.default_rng(N)
    n = 3 if N <= 1024 else 1
    G = (g.normal(size=(n, N, N)) + 1j * g.normal(size=(n, N, N))).astype(np.complex64)
    W = np.array([2.5, 1.0, 7.0][:n])
    dev = torch.from_numpy(G).to("cuda:0")
    for shift in (True, False):
        out = ctx.blink_ifft2d(dev, torch.from_numpy(W).to("cuda:0"), shift=shift).cpu().numpy()
        for i in range(n):
            ref, _ = oracle.ifft2d(G[i], W[i], shift=shift)
            e = rel_l2(out[i], ref)
            assert e <= IMAGE_TOL, (N, shift, i, e)


def test_ifft2d_weights(torch, ctx):
    say("blink_ifft2d weights: NULL, zero, negative")
    N = 64
    g = np.random.default_rng(5)
    G = (g.normal(size=(3, N, N)) + 1j * g.normal(size=(3, N, N))).astype(np.complex64)
    dev = torch.from_numpy(G).to("cuda:0")
    unit = ctx.blink_ifft2d(dev, None).cpu().numpy()
    for i in range(3):
        ref, _ = oracle.ifft2d(G[i], 1.0)
        assert rel_l2(unit[i], ref) <= IMAGE_TOL
    W = torch.tensor([0.0, -3.0, 4.0], dtype=torch.float64, device="cuda:0")
    out = ctx.blink_ifft2d(dev, W).cpu().numpy()
    assert not out[0].any() and not out[1].any()
    assert rel_l2(out[2], unit[2] / 4.0) <= 1e-6


def test_grid_then_ifft2d_equals_fused(torch, ctx, generated):
    spec = synth.spec_vcs(T=1, C=2, P=2)
    prob = generated("vcs-1024-1x2x2", spec)
    say("grid+ifft2d vs fused image_batch N=1024")
    vis, flags, uvw, freq = to_device(torch, prob)
    g = ctx.blink_grid(vis, flags, uvw, freq, spec.grid_n, spec.pixel_scale, 0)
    two = ctx.blink_ifft2d(g["grids"], g["weight_sum"]).cpu().numpy()
    one = ctx.blink_image_batch(vis, flags, uvw, freq, spec.grid_n, spec.pixel_scale, 0)["images"].cpu().numpy()
    for idx in np.ndindex(1, 2, 2):
        assert rel_l2(one[idx], two[idx]) <= 2e-6


def test_degenerate_inputs(torch, ctx):
    spec = small_spec(N=32, T=1, C=2, P=2, n_tiles=10, flag_frac=0.0)
    prob = synth.make_problem(spec)
    vis, flags, uvw, freq = to_device(torch, prob)
    say("degenerate: all flagged")
    allf = torch.ones_like(flags)
    r = ctx.blink_image_batch(vis, allf, uvw, freq, 32, spec.pixel_scale, 0)
    assert not r["images"].any() and not r["weight_sum"].any() and not r["n_out"].any()
    say("degenerate: all out of grid")
    r = ctx.blink_image_batch(vis, None, uvw * 1e4, freq, 32, spec.pixel_scale, 1)
    assert not r["images"].any() and not r["weight_sum"].any()
    assert (r["n_out"] == spec.B).all()
    say("degenerate: no baselines")
    r = ctx.blink_image_batch(vis[..., :0].contiguous(), flags[..., :0].contiguous(), uvw[:, :0].contiguous(),
                              freq, 32, spec.pixel_scale, 0)
    assert not r["images"].any()
    say("degenerate: empty batch")
    r = ctx.blink_image_batch(vis[:0], flags[:0], uvw[:0], freq, 32, spec.pixel_scale, 0)
    assert r["images"].numel() == 0
    say("degenerate: NaN and huge coordinates are out of grid")
    bad = uvw.clone()
    bad[0, 0, 0] = float("nan")
    bad[0, 1, 1] = 1e300
    g = ctx.blink_grid(vis, None, bad, freq, 32, spec.pixel_scale, 0)
    ref = oracle.grid(prob.vis[0, 0], None, bad[0].cpu().numpy(), prob.freq_hz[0], 32, spec.pixel_scale)
    assert np.array_equal(g["cell_idx"][0, 0].cpu().numpy(), ref["cell_idx"])
    assert int(g["cell_idx"][0, 0, 0]) == -2 and int(g["cell_idx"][0, 0, 1]) == -2


def test_chunked_workspace_matches_single_chunk(torch, ctx, generated):
    import paper_2505_15204_amd as blink
    spec = small_spec(N=64, T=2, C=3, P=2)
    prob = generated("small-64-natural", spec)
    say("chunked workspace N=64 T=2 C=3")
    vis, flags, uvw, freq = to_device(torch, prob)
    full = ctx.blink_image_batch(vis, flags, uvw, freq, 64, spec.pixel_scale, 0)
    one_pair = blink.image_batch_workspace_size(1, 1, 2, spec.B, 64)
    ws = torch.empty(one_pair, dtype=torch.uint8, device="cuda:0")
    small = ctx.blink_image_batch(vis, flags, uvw, freq, 64, spec.pixel_scale, 0, workspace=ws)
    assert torch.equal(full["weight_sum"], small["weight_sum"])
    a, b = full["images"].cpu().numpy(), small["images"].cpu().numpy()
    for idx in np.ndindex(2, 3, 2):
        assert rel_l2(a[idx], b[idx]) <= 1e-6
    # below the query for one pair the library falls back to one intermediate at a time
    tight = torch.empty(one_pair - 4096, dtype=torch.uint8, device="cuda:0")
    one = ctx.blink_image_batch(vis, flags, uvw, freq, 64, spec.pixel_scale, 0, workspace=tight)
    c = one["images"].cpu().numpy()
    for idx in np.ndindex(2, 3, 2):
        assert rel_l2(c[idx], a[idx]) <= 1e-6
    too_small = torch.empty(4096, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(blink.BlinkError) as e:
        ctx.blink_image_batch(vis, flags, uvw, freq, 64, spec.pixel_scale, 0, workspace=too_small)
    assert e.value.status == blink.BLINK_ERR_SIZE


def test_vcs_full_time_step_sampled(torch, ctx):
    """One full time step of the 1024^2 VCS workload (768 channels x 2 pols, 8128 baselines) in the
    launch configuration the benchmark times; sampled channels checked against the oracle."""
    spec = synth.spec_vcs(T=1)
    say("blink_image_batch vcs-1024 full time step 768x2 (sampled check)")
    d = synth.make_problem_device(spec, "cuda:0")
    res = ctx.blink_image_batch(d["vis"], d["flags"], d["uvw_m"], d["freq_hz"], spec.grid_n, spec.pixel_scale, 0)
    torch.cuda.synchronize()
    img = res["images"]
    assert bool(torch.isfinite(img).all())
    chans = [0, 255, 511, 767]
    vis_h = d["vis"][:, chans].cpu().numpy()
    flags_h = d["flags"][:, chans].cpu().numpy()
    uvw_h = d["uvw_m"].cpu().numpy()
    freq_h = d["freq_hz"].cpu().numpy()[chans]
    ref = oracle.image_batch(vis_h, flags_h, uvw_h, freq_h, spec.grid_n, spec.pixel_scale, 0)
    got = img[:, chans].cpu().numpy()
    assert np.array_equal(res["weight_sum"][:, chans].cpu().numpy(), ref["weight_sum"])
    assert np.array_equal(res["n_out"][:, chans].cpu().numpy(), ref["n_out"])
    for idx in np.ndindex(1, len(chans), 2):
        e = rel_l2(got[idx], ref["images"][idx])
        assert e <= IMAGE_TOL, (idx, e)
    # any-size property: a dirty image never exceeds the sum of visibility amplitudes / W per pixel
    amp = torch.abs(d["vis"][0]).to(torch.float64) * (1 - d["flags"][0].to(torch.float64))[:, None, :]
    bound = 2 * amp.sum(-1) / res["weight_sum"][0]
    assert bool((img[0].abs().amax(dim=(-1, -2)).to(torch.float64) <= bound * (1 + 1e-5)).all())
