"""GPU parity of the correlator (blink_correlate, Eq. 3 / Section 6.2.2) against the oracle.

The sums are integers, exact on both sides (int32 on the matrix cores, int64 in the oracle), and
both divide in FP64 and round once, so visibilities and autocorrelations are compared bit for
bit. Cases cover ragged input tiles (2A not a multiple of 32), a K that is not a multiple of the
64-value staging chunk, the largest array (256 antennas, 80 KB of LDS), the int32 bound
(K = 65535 of -128 values), both polarisation layouts, and a plane wave correlated and imaged.
"""
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


CASES = [
    # name, S, F, A, n_int, n_favg, pol_mode, seed
    ("A4-K8", 8, 4, 4, 4, 2, 4, 1),
    ("A12-ragged-tile", 6, 3, 12, 3, 1, 4, 2),
    ("A36-three-slabs", 10, 4, 36, 5, 2, 2, 3),
    ("A128-K800", 200, 8, 128, 200, 4, 4, 4),
    ("A128-K800-xx-yy", 200, 8, 128, 200, 4, 2, 5),
    ("A256-max", 64, 2, 256, 32, 2, 4, 6),
    ("A8-K1", 3, 5, 8, 1, 1, 4, 7),
]


@pytest.mark.parametrize("name,S,F,A,n_int,n_favg,mode,seed", CASES, ids=[c[0] for c in CASES])
def test_correlate_bit_exact(torch, ctx, name, S, F, A, n_int, n_favg, mode, seed):
    g = np.random.default_rng(seed)
    volt = g.integers(-128, 128, size=(S, F, A, 2, 2)).astype(np.int8)
    say(f"blink_correlate {name}: S={S} F={F} A={A} n_int={n_int} n_favg={n_favg} pol_mode={mode}")
    res = ctx.blink_correlate(torch.from_numpy(volt).to("cuda:0"), n_int, n_favg, mode, autos=True)
    ref = oracle.correlate(volt, n_int, n_favg, mode)
    assert np.array_equal(res["vis"].cpu().numpy(), ref["vis"])
    assert np.array_equal(res["autos"].cpu().numpy(), ref["autos"])


def test_correlate_int32_bound(torch, ctx):
    """K = 65535 samples of -128 - 128i: every real sum is 2 x 16384 x 65535, just below 2^31."""
    S, F, A = 65535, 1, 4
    volt = np.full((S, F, A, 2, 2), -128, dtype=np.int8)
    say("blink_correlate K=65535 of -128")
    res = ctx.blink_correlate(torch.from_numpy(volt).to("cuda:0"), S, 1, 4, autos=True)
    ref = oracle.correlate(volt, S, 1, 4)
    assert np.array_equal(res["vis"].cpu().numpy(), ref["vis"])
    assert np.array_equal(res["autos"].cpu().numpy(), ref["autos"])
    assert (res["vis"].cpu().numpy().real == 32768.0).all()


def test_correlate_then_image_plane_wave(torch, ctx):
    """A plane wave from (l, m) = (5, -3) pixels, quantised to int8 voltages, correlated and
    imaged with blink_image_batch (XX, YY), peaks at pixel (N/2 - 3, N/2 + 5) in both pols."""
    A, S, F, N = 32, 16, 2, 128
    pos = synth.tile_positions(A, np.random.default_rng(70))
    uvw = synth.baseline_uvw(pos)[None]                                    # [1][B][3]
    freq = np.array([150.0e6, 150.04e6])
    dl = 8.0e-3
    l, m = 5 * dl, -3 * dl
    volt = np.zeros((S, F, A, 2, 2), dtype=np.int8)
    g = np.random.default_rng(71)
    for f, fr in enumerate(freq):
        ph = np.exp(-2j * np.pi * (fr / synth.C_LIGHT) * (pos[:, 0] * l + pos[:, 1] * m))
        for s in range(S):
            x = 60.0 * ph * np.exp(2j * np.pi * g.random())                # common random phase per sample
            for p in range(2):
                volt[s, f, :, p, 0] = np.rint(x.real)
                volt[s, f, :, p, 1] = np.rint(x.imag)
    say("correlate -> image, plane wave, A=32 N=128")
    vis = ctx.blink_correlate(torch.from_numpy(volt).to("cuda:0"), S, 1, 2)["vis"]     # [1][F][2][B]
    img = ctx.blink_image_batch(vis, None, torch.from_numpy(uvw).to("cuda:0"), torch.from_numpy(freq).to("cuda:0"),
                                N, dl, 0)["images"].cpu().numpy()
    for f, p in np.ndindex(F, 2):
        y, x = np.unravel_index(np.argmax(img[0, f, p]), (N, N))
        assert (y, x) == (N // 2 - 3, N // 2 + 5), (f, p, y, x)


def test_correlate_argument_errors(torch, ctx):
    import paper_2505_15204_amd as blink
    volt = torch.zeros((4, 2, 6, 2, 2), dtype=torch.int8, device="cuda:0")
    with pytest.raises(blink.BlinkError):
        ctx.blink_correlate(volt, 2, 1)                       # A = 6 is not a multiple of 4
    volt = torch.zeros((4, 2, 8, 2, 2), dtype=torch.int8, device="cuda:0")
    with pytest.raises(blink.BlinkError):
        ctx.blink_correlate(volt, 3, 1)                       # 3 does not divide S = 4
    with pytest.raises(blink.BlinkError):
        ctx.blink_correlate(volt, 2, 1, pol_mode=3)
    flat = torch.zeros(4 * 2 * 8 * 4 + 16, dtype=torch.int8, device="cuda:0")
    with pytest.raises(blink.BlinkError):
        ctx.blink_correlate(flat[2:2 + 4 * 2 * 8 * 4].view(4, 2, 8, 2, 2), 2, 1)   # not 16-byte aligned


def test_correlate_rounds_exact_midpoint_to_even(torch, ctx):
    """A mean that is exactly halfway between two floats: XX of baseline (1, 0) sums to
    3 (2^24 + 1) over K = 6144 terms, so V = 16777217 / 2048 = 8192 + 2^-11, the midpoint of
    8192 and 8192 + 2^-10; rounded to even it is 8192 on both sides."""
    S, F, A, n_int, n_favg = 2048, 3, 4, 2048, 3
    volt = np.zeros((S, F, A, 2, 2), dtype=np.int8)
    volt[:, :, 0, 0] = (64, 64)
    volt[:, :, 1, 0] = (64, 64)
    for s in range(3):                        # three terms of 64 * 62 + 65 * 65 = 8193
        volt[s, 0, 0, 0] = (64, 65)
        volt[s, 0, 1, 0] = (62, 65)
    say("blink_correlate exact rounding midpoint, K=6144")
    res = ctx.blink_correlate(torch.from_numpy(volt).to("cuda:0"), n_int, n_favg, 4, autos=True)
    ref = oracle.correlate(volt, n_int, n_favg, 4)
    assert ref["vis"][0, 0, 0, 0].real == np.float32(8192.0)
    assert np.array_equal(res["vis"].cpu().numpy(), ref["vis"])
    assert np.array_equal(res["autos"].cpu().numpy(), ref["autos"])
