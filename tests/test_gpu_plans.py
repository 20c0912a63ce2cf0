"""GPU parity of every compiled execution plan (strip width x row block x image group) and of
the autotuner, against the FP64 oracle. Plans only reschedule work, so every plan must meet the
same bar as the default one."""
import numpy as np
import pytest

import oracle
from paper_2505_15204_amd import synth

pytestmark = pytest.mark.gpu

IMAGE_TOL = 1e-5


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


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
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def restore(ctx, N, weighting, plan, precision=0):
    ctx.set_plan(N, weighting, plan["col_strip"], plan["row_block"], plan["group"], precision=precision,
                 col_loop=plan["col_loop"])


def make(torch, N, weighting, C, P):
    spec = synth.Spec(f"plans-{N}", 21, 128, 1, P, synth.vcs_channels()[:C * 97:97], N, synth.ARCMIN * 1024 / N,
                      20, 0.1, weighting=weighting)
    prob = synth.make_problem(spec)
    ref = oracle.image_batch(prob.vis, prob.flags, prob.uvw_m, prob.freq_hz, N, spec.pixel_scale, weighting)
    d = "cuda:0"
    dev = (torch.from_numpy(prob.vis).to(d), torch.from_numpy(prob.flags).to(d), torch.from_numpy(prob.uvw_m).to(d),
           torch.from_numpy(prob.freq_hz).to(d))
    return spec, dev, ref


CASES = [(256, 0, 3, 2), (256, 1, 3, 2), (512, 0, 2, 2), (1024, 0, 3, 2), (1024, 1, 2, 2), (2048, 0, 1, 2),
         (2048, 1, 1, 2), (4096, 0, 1, 2)]


@pytest.mark.parametrize("N,weighting,C,P", CASES, ids=[f"N{c[0]}-w{c[1]}" for c in CASES])
def test_every_plan_matches_oracle(torch, ctx, N, weighting, C, P):
    import paper_2505_15204_amd as blink
    spec, (vis, flags, uvw, freq), ref = make(torch, N, weighting, C, P)
    cols, rows = blink.plan_options(N, weighting)
    n_img = C * P
    groups = sorted({0, 1, max(1, n_img - 1)})
    default = ctx.get_plan(N, weighting)

    def check(col, row, grp, loop):
        say(f"plan N={N} w={weighting} col_strip={col} row_block={row} group={grp} col_loop={loop}")
        ctx.set_plan(N, weighting, col, row, grp, col_loop=loop)
        res = ctx.blink_image_batch(vis, flags, uvw, freq, N, spec.pixel_scale, weighting)
        assert np.array_equal(res["weight_sum"].cpu().numpy(), ref["weight_sum"])
        img = res["images"].cpu().numpy()
        for idx in np.ndindex(1, C, P):
            e = rel_l2(img[idx], ref["images"][idx])
            assert e <= IMAGE_TOL, (col, row, grp, loop, idx, e)
    try:
        for col in cols:
            for row in rows:
                for grp in groups:
                    check(col, row, grp, 1)
            # strips per column workgroup: a power of two, one that does not divide the strip
            # count, and more than there are strips (one workgroup per image)
            for loop in (4, 3, 64):
                check(col, rows[0], 0, loop)
    finally:
        restore(ctx, N, weighting, default)


def test_set_plan_rejects_uncompiled_options(torch, ctx):
    import paper_2505_15204_amd as blink
    with pytest.raises(blink.BlinkError):
        ctx.set_plan(1024, 0, 3, 4, 0)
    with pytest.raises(blink.BlinkError):
        ctx.set_plan(1024, 0, 16, 5, 0)
    with pytest.raises(blink.BlinkError):
        ctx.set_plan(1024, 0, 16, 4, -1)
    for loop in (0, 65):
        with pytest.raises(blink.BlinkError):
            ctx.set_plan(1024, 0, 16, 4, 0, col_loop=loop)


def test_autotuner_picks_a_compiled_plan_and_leaves_valid_images(torch, ctx, tmp_path):
    import paper_2505_15204_amd as blink
    spec, (vis, flags, uvw, freq), ref = make(torch, 1024, 0, 3, 2)
    say("autotune N=1024 natural, 6 images")
    default = ctx.get_plan(1024, 0)
    try:
        out = torch.empty((1, 3, 2, 1024, 1024), dtype=torch.float32, device="cuda:0")
        plan, ms = ctx.autotune_image_batch(vis, flags, uvw, freq, 1024, spec.pixel_scale, 0, out=out)
        cols, rows = blink.plan_options(1024, 0)
        assert plan["col_strip"] in cols and plan["row_block"] in rows and plan["group"] > 0 and ms > 0
        assert plan["col_loop"] in (1, 2, 4, 8, 16)
        assert ctx.get_plan(1024, 0) == plan
        img = out.cpu().numpy()
        for idx in np.ndindex(1, 3, 2):
            assert rel_l2(img[idx], ref["images"][idx]) <= IMAGE_TOL
        path = tmp_path / "plans.json"
        ctx.save_plans(str(path))
        restore(ctx, 1024, 0, default)
        ctx.load_plans(str(path))
        assert ctx.get_plan(1024, 0) == plan
    finally:
        restore(ctx, 1024, 0, default)


@pytest.mark.parametrize("precision", [0, 1, 2], ids=["fp32", "split-f16", "split-bf16"])
def test_benched_plan_full_time_step(torch, ctx, precision):
    """One full time step of the 1024^2 VCS workload (768 channels x 2 pols, 8128 baselines, 10%
    flags) under the committed tuned plans, i.e. the launch configuration the benchmark times for
    each precision form. Sampled channels are checked against the FP64 oracle: weight sums and
    out-of-grid counts bit-exact; images within 1e-5 (FP32) or, for the split forms, within 1e-3
    relative L2 and peak error with the same 6-sigma detections."""
    import paper_2505_15204_amd as blink
    from image_checks import peak_error, recovery
    spec = synth.spec_vcs(T=1)
    with blink.Context(0) as c2:                     # the loaded plans stay in this context
        c2.load_plans(blink.PLANS_PATH)
        plan = c2.get_plan(1024, 0, precision)
        say(f"benched plan, vcs-1024 full time step, precision={precision}: {plan}")
        assert plan["group"] > 0
        d = synth.make_problem_device(spec, "cuda:0")
        res = c2.blink_image_batch(d["vis"], d["flags"], d["uvw_m"], d["freq_hz"], spec.grid_n, spec.pixel_scale,
                                   0, precision=precision)
        torch.cuda.synchronize()
    img = res["images"]
    assert bool(torch.isfinite(img).all())
    chans = [0, 1, 23, 24, 383, 766, 767]           # first/last images of the tuned groups of 48
    ref = oracle.image_batch(d["vis"][:, chans].cpu().numpy(), d["flags"][:, chans].cpu().numpy(),
                             d["uvw_m"].cpu().numpy(), d["freq_hz"].cpu().numpy()[chans], spec.grid_n,
                             spec.pixel_scale, 0)
    assert np.array_equal(res["weight_sum"][:, chans].cpu().numpy(), ref["weight_sum"])
    assert np.array_equal(res["n_out"][:, chans].cpu().numpy(), ref["n_out"])
    got = img[:, chans].cpu().numpy()
    for idx in np.ndindex(1, len(chans), 2):
        e = rel_l2(got[idx], ref["images"][idx])
        if precision == 0:
            assert e <= IMAGE_TOL, (idx, e)
        else:
            pk = peak_error(got[idx], ref["images"][idx])
            missing, spurious = recovery(got[idx], ref["images"][idx])
            say(f"  {idx}: rel_l2={e:.3e} peak={pk:.3e} missing={len(missing)} spurious={len(spurious)}")
            assert e <= 1e-3 and pk <= 1e-3 and not missing and not spurious, (idx, e, pk)
    # every image of the step: natural W = 2 x (unflagged - out of grid), bit-exact
    kept = (1 - d["flags"][0].to(torch.int64)).sum(-1) - res["n_out"][0].to(torch.int64)
    assert torch.equal(res["weight_sum"][0], (2 * kept).to(torch.float64)[:, None].expand(-1, 2))
