"""GPU parity at the Phase II shape (144 tiles, 10296 cross baselines, 3072 x 10 kHz channels from
185 MHz, 2 pols, 2048^2 at 0.75 arcmin, uniform weighting), in the launch configuration the
benchmark times: the committed execution plans, one time step imaged in four calls of 768
channels. Sampled channels of each call are checked against the FP64 oracle one by one: weight
sums (occupied cells) and out-of-grid counts bit-exact, images within a relative L2 of 1e-5.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2505_15204_amd import synth

pytestmark = pytest.mark.gpu

IMAGE_TOL = 1e-5
CALL_CHANNELS = 768


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
    c.load_plans(blink.PLANS_PATH)
    yield c
    c.close()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_phase2_time_step_sampled(torch, ctx):
    spec = synth.spec_phase2(T=1)
    N, P, B = spec.grid_n, spec.P, spec.B
    assert (B, N, spec.C, spec.weighting) == (10296, 2048, 3072, 1)
    say(f"Phase II time step: C={spec.C} P={P} B={B} N={N}, uniform, calls of {CALL_CHANNELS} channels")
    d = synth.make_problem_device(spec, "cuda:0")
    uvw_h = d["uvw_m"].cpu().numpy()
    freq_all = d["freq_hz"].cpu().numpy()
    images = torch.empty((1, CALL_CHANNELS, P, N, N), dtype=torch.float32, device="cuda:0")
    picks = (0, 767)        # first and last channel of each call
    for c0 in range(0, spec.C, CALL_CHANNELS):
        say(f"  channels {c0} .. {c0 + CALL_CHANNELS - 1}")
        sl = slice(c0, c0 + CALL_CHANNELS)
        res = ctx.blink_image_batch(d["vis"][:, sl], d["flags"][:, sl], d["uvw_m"], d["freq_hz"][sl], N,
                                    spec.pixel_scale, 1, out=images)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(images).all())
        chans = [c0 + j for j in picks]
        ref = oracle.image_batch(d["vis"][:, chans].cpu().numpy(), d["flags"][:, chans].cpu().numpy(), uvw_h,
                                 freq_all[chans], N, spec.pixel_scale, 1)
        assert np.array_equal(res["weight_sum"][:, list(picks)].cpu().numpy(), ref["weight_sum"])
        assert np.array_equal(res["n_out"][:, list(picks)].cpu().numpy(), ref["n_out"])
        got = images[:, list(picks)].cpu().numpy()
        for idx in np.ndindex(1, len(picks), P):
            e = rel_l2(got[idx], ref["images"][idx])
            say(f"    channel {chans[idx[1]]} pol {idx[2]}: W={ref['weight_sum'][idx]:.0f} rel_l2={e:.2e}")
            assert e <= IMAGE_TOL, (chans[idx[1]], idx, e)
        # any-size property on the whole call: uniform weighting averages placements per cell, so
        # |I| <= (sum over occupied cells of the largest |V| there) / W <= max|V| * W / W
        vmax = (torch.abs(d["vis"][0, sl]) * (1 - d["flags"][0, sl].to(torch.float32))[:, None, :]).amax(-1)
        peak = images[0].abs().amax(dim=(-1, -2))
        assert bool((peak.to(torch.float64) <= vmax.to(torch.float64) * (1 + 1e-5)).all())
