"""blink_image_batch_noalloc (no workspace: the library's static scratch array) against
blink_image_batch (caller's workspace) on the same inputs, through the C ABI.

Bar (the same as for the oracle comparisons of the FP32 path): weight sums and out-of-grid counts
bit-exact, images within a relative L2 of 1e-5 per image (the two calls add a cell's placements in
different atomic orders). Two calls in a row, the second with a smaller problem, so the second
call runs on the scratch contents the first one left; then a problem whose single (t, c) pair does
not fit the scratch is rejected before anything is written.
"""
import sys

import numpy as np
import pytest

from paper_2505_15204_amd import synth

pytestmark = pytest.mark.gpu

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
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def device_problem(torch, spec):
    prob = synth.make_problem(spec)
    d = "cuda:0"
    return (torch.from_numpy(prob.vis).to(d), torch.from_numpy(prob.flags).to(d),
            torch.from_numpy(prob.uvw_m).to(d), torch.from_numpy(prob.freq_hz).to(d))


def compare(torch, ctx, spec, weighting):
    vis, flags, uvw, freq = device_problem(torch, spec)
    T, C, P, B = vis.shape
    N = spec.grid_n
    d = "cuda:0"
    ref = ctx.blink_image_batch(vis, flags, uvw, freq, N, spec.pixel_scale, weighting)
    torch.cuda.synchronize()
    out = torch.full((T, C, P, N, N), float("nan"), dtype=torch.float32, device=d)
    wsum = torch.full((T, C, P), -1.0, dtype=torch.float64, device=d)
    nout = torch.full((T, C), -1, dtype=torch.int32, device=d)
    before = torch.cuda.memory_allocated(d)
    ctx.blink_image_batch_noalloc(vis, flags, uvw, freq, N, spec.pixel_scale, weighting, out=out,
                                  weight_sum=wsum, n_out=nout)
    assert torch.cuda.memory_allocated(d) == before     # the binding allocated nothing either
    torch.cuda.synchronize()
    assert np.array_equal(wsum.cpu().numpy(), ref["weight_sum"].cpu().numpy())
    assert np.array_equal(nout.cpu().numpy(), ref["n_out"].cpu().numpy())
    a, r = out.cpu().numpy(), ref["images"].cpu().numpy()
    assert np.isfinite(a).all()
    worst = max(rel_l2(a[idx], r[idx]) for idx in np.ndindex(T, C, P))
    say(f"  {T * C * P} images of {N}^2: worst relative L2 against blink_image_batch {worst:.2e}")
    assert worst <= IMAGE_TOL


def test_noalloc_matches_workspace_entry_point(torch, ctx):
    import paper_2505_15204_amd as blink
    # First call: the VCS shape, 24 channels x 2 pols of 1024^2 (48 images; the 64 MiB scratch holds
    # 15 half-spectrum intermediates, so the call runs several image groups).
    spec1 = synth.spec_vcs(T=1, C=24, P=2)
    say(f"noalloc call 1: {spec1.name} T=1 C=24 P=2 B={spec1.B} N={spec1.grid_n}, natural")
    compare(torch, ctx, spec1, blink.WEIGHT_NATURAL)
    # Second call, smaller: 2 time steps x 3 channels x 2 pols of 256^2, uniform weighting, on the
    # scratch contents the first call left.
    spec2 = synth.Spec("noalloc-256", 12, 64, 2, 2, np.array([150.0e6, 160.0e6, 170.0e6]), 256, synth.ARCMIN * 4,
                       5, 0.1, weighting=1)
    say(f"noalloc call 2: {spec2.name} T=2 C=3 P=2 B={spec2.B} N=256, uniform")
    compare(torch, ctx, spec2, blink.WEIGHT_UNIFORM)


def test_noalloc_rejects_pairs_beyond_the_scratch(torch, ctx):
    import paper_2505_15204_amd as blink
    # One (t, c) pair at 4096^2 needs a 64 MiB half spectrum plus its placements: more than the scratch.
    spec = synth.Spec("noalloc-4096", 13, 16, 1, 1, np.array([150.0e6]), 4096, synth.ARCMIN, 2, 0.0)
    vis, flags, uvw, freq = device_problem(torch, spec)
    out = torch.full((1, 1, 1, 4096, 4096), 7.0, dtype=torch.float32, device="cuda:0")
    say("noalloc call at 4096^2 (must be rejected)")
    with pytest.raises(blink.BlinkError) as ei:
        ctx.blink_image_batch_noalloc(vis, flags, uvw, freq, 4096, spec.pixel_scale, 0, out=out)
    assert ei.value.status == blink.BLINK_ERR_SIZE
    assert "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())          # nothing was written
    # the context stays usable
    spec2 = synth.Spec("noalloc-64", 14, 16, 1, 1, np.array([150.0e6]), 64, synth.ARCMIN * 16, 2, 0.0)
    compare(torch, ctx, spec2, blink.WEIGHT_NATURAL)
