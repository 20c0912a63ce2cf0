"""Entry points called on a stream other than torch's current one: the binding allocates the
call's workspace and outputs on that stream, so memory the caller allocates on the current stream
right after the call never lands on a workspace that the queued kernels still use."""
import sys

import numpy as np
import pytest

import oracle
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


def test_side_stream_then_allocation_on_current_stream(torch, ctx):
    import paper_2505_15204_amd as blink
    spec = synth.spec_vcs(T=1, C=48, P=2)
    d = synth.make_problem_device(spec, "cuda:0")
    say("blink_image_batch on a side stream, then garbage allocations on the current stream")
    ref = ctx.blink_image_batch(d["vis"], d["flags"], d["uvw_m"], d["freq_hz"], spec.grid_n, spec.pixel_scale, 0)
    torch.cuda.synchronize()
    ws_bytes = blink.image_batch_workspace_size(1, 48, 2, spec.B, spec.grid_n)
    side = torch.cuda.Stream()                      # default priority
    side.wait_stream(torch.cuda.current_stream())
    for rep in range(3):
        res = ctx.blink_image_batch(d["vis"], d["flags"], d["uvw_m"], d["freq_hz"], spec.grid_n, spec.pixel_scale,
                                    0, stream=side)
        # the workspace of the call is free on return; allocate and overwrite as much on the
        # current stream while the side stream's kernels still run
        junk = [torch.full((ws_bytes // 4,), float("nan"), device="cuda:0") for _ in range(2)]
        side.synchronize()
        torch.cuda.synchronize()
        del junk
        assert torch.equal(res["weight_sum"], ref["weight_sum"])
        diff = (res["images"] - ref["images"]).abs().max().item()
        assert diff <= 1e-6 * ref["images"].abs().max().item(), (rep, diff)
    # and the result is the oracle's for a sampled channel
    chans = [5]
    o = oracle.image_batch(d["vis"][:, chans].cpu().numpy(), d["flags"][:, chans].cpu().numpy(),
                           d["uvw_m"].cpu().numpy(), d["freq_hz"].cpu().numpy()[chans], spec.grid_n,
                           spec.pixel_scale, 0)
    got = res["images"][:, chans].cpu().numpy()
    for idx in np.ndindex(1, 1, 2):
        e = np.linalg.norm(got[idx] - o["images"][idx]) / np.linalg.norm(o["images"][idx])
        assert e <= 1e-5
