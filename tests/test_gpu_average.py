"""GPU parity of the image averages (blink_image_average) against the FP64 oracle: every
combination of averaged axes on random images, and Stokes I / band averages of imaged data."""
import sys

import numpy as np
import pytest

import oracle
from image_checks import rel_l2
from paper_2505_15204_amd import synth

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


@pytest.mark.parametrize("axes", range(8))
def test_average_axes(torch, ctx, axes):
    say(f"blink_image_average axes={axes}")
    g = np.random.default_rng(50 + axes)
    imgs = g.normal(size=(3, 5, 2, 32, 32)).astype(np.float32)
    out = ctx.blink_image_average(torch.from_numpy(imgs).to("cuda:0"), axes).cpu().numpy()
    ref = oracle.image_average(imgs, axes)
    assert out.shape == ref.shape
    assert np.abs(out - ref).max() <= 1e-6 * np.abs(ref).max()


def test_stokes_i_and_band_average_of_images(torch, ctx):
    """Stokes I and the band average of one time step of 1024^2 images made by the library."""
    import paper_2505_15204_amd as blink
    spec = synth.spec_vcs(T=1, C=16, P=2)
    say("blink_image_batch vcs-1024 1x16x2 then Stokes I and band average")
    d = synth.make_problem_device(spec, "cuda:0")
    imgs = ctx.blink_image_batch(d["vis"], d["flags"], d["uvw_m"], d["freq_hz"], 1024, spec.pixel_scale, 0)["images"]
    torch.cuda.synchronize()
    host = imgs.cpu().numpy()
    for axes in (blink.AVG_POL, blink.AVG_CHANNEL | blink.AVG_POL):
        out = ctx.blink_image_average(imgs, axes).cpu().numpy()
        ref = oracle.image_average(host, axes)
        for idx in np.ndindex(out.shape[:3]):
            assert rel_l2(out[idx], ref[idx]) <= 1e-6
    with pytest.raises(blink.BlinkError):
        ctx.blink_image_average(imgs, 9)
