"""GPU parity of the incoherent de-dispersion (blink_dedisperse) against the FP64 oracle.

Both sum in FP64 in channel order and divide by C once, so every output pixel is the oracle's
value rounded to float: the comparison is exact."""
import sys

import numpy as np
import pytest

import oracle

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


CASES = [
    # name, T, C, N, dt, DMs, channel spacing (Hz)
    ("N32-C16", 20, 16, 32, 0.05, [0.0, 1.0, 2.5, 4.0], 1.0e6),
    ("N256-C64", 24, 64, 256, 0.05, [0.0, 0.7, 3.0], 0.4e6),
    ("N8-C3-one-dm", 6, 3, 8, 0.1, [10.0], 5.0e6),
]


@pytest.mark.parametrize("name,T,C,N,dt,dms,df", CASES, ids=[c[0] for c in CASES])
def test_dedisperse_matches_oracle(torch, ctx, name, T, C, N, dt, dms, df):
    import paper_2505_15204_amd as blink
    freq = 140.0e6 + df * np.arange(C)
    delays = blink.dispersion_delays(freq, dt, dms)
    assert np.array_equal(delays, oracle.dispersion_delays(freq, dt, dms))
    t_out = T - int(delays.max())
    imgs = np.random.default_rng(90).normal(size=(T, C, N, N)).astype(np.float32)
    say(f"blink_dedisperse {name}: T={T} C={C} N={N} n_dm={len(dms)} t_out={t_out} max delay={delays.max()}")
    out = ctx.blink_dedisperse(torch.from_numpy(imgs).to("cuda:0"), delays, t_out).cpu().numpy()
    ref = oracle.dedisperse(imgs, delays, t_out)
    assert np.array_equal(out, ref.astype(np.float32))


def test_dedisperse_recovers_dispersed_pulse(torch, ctx):
    import paper_2505_15204_amd as blink
    T, C, N = 48, 32, 64
    freq = 139.0e6 + 40.0e3 * 24 * np.arange(C)
    dms = [0.0, 1.0, 2.0, 3.0, 4.0]
    delays = blink.dispersion_delays(freq, 0.02, dms)
    t0, y, x = 5, 40, 17
    imgs = np.zeros((T, C, N, N), dtype=np.float32)
    for c in range(C):
        imgs[t0 + delays[3, c], c, y, x] = 2.0
    t_out = T - int(delays.max())
    say(f"dispersed pulse at DM 3, max delay {delays.max()}")
    out = ctx.blink_dedisperse(torch.from_numpy(imgs).to("cuda:0"), delays, t_out).cpu().numpy()
    assert out[3, t0, y, x] == 2.0 and np.count_nonzero(out[3]) == 1
    assert all(out[k].max() < 2.0 for k in (0, 1, 2, 4))


def test_dedisperse_argument_errors(torch, ctx):
    import paper_2505_15204_amd as blink
    imgs = torch.zeros((6, 4, 8, 8), dtype=torch.float32, device="cuda:0")
    delays = np.array([[0, 1, 2, 3]], dtype=np.int32)
    with pytest.raises(blink.BlinkError):
        ctx.blink_dedisperse(imgs, delays, 4)          # 4 + 3 > 6
    with pytest.raises(blink.BlinkError):
        ctx.blink_dedisperse(imgs, -delays, 3)
    with pytest.raises(blink.BlinkError):
        ctx.blink_dedisperse(imgs, delays, 7)
    out = ctx.blink_dedisperse(imgs, delays, 3)
    assert out.shape == (1, 3, 8, 8) and not out.any()
