"""CPU tests: the FP64 oracle against its pins (no GPU needed)."""
import numpy as np
import pytest

import oracle
import oracle_pins


@pytest.fixture(scope="module")
def O():
    oracle.build(force=False)
    return oracle.default()


@pytest.mark.parametrize("pin", oracle_pins.PINS + oracle_pins.EXTRA_PINS, ids=lambda p: p.__name__)
def test_pin(O, pin):
    pin(O)


def test_batch_matches_per_image(O):
    """The threaded batch driver gives the same images as gridding and imaging one at a time."""
    g = np.random.default_rng(21)
    T, C, P, B, N = 2, 3, 2, 120, 32
    uvw = np.zeros((T, B, 3))
    uvw[:, :, :2] = g.uniform(-300, 300, size=(T, B, 2))
    freq = np.array([140e6, 150e6, 160e6])
    vis = (g.normal(size=(T, C, P, B)) + 1j * g.normal(size=(T, C, P, B))).astype(np.complex64)
    flags = (g.random((T, C, B)) < 0.2).astype(np.uint8)
    dl = 1.0 / 200.0
    for weighting in (0, 1):
        res = O.image_batch(vis, flags, uvw, freq, N, dl, weighting=weighting, n_threads=4,
                            want_counts=True)
        for t in range(T):
            for c in range(C):
                one = O.grid(vis[t, c], flags[t, c], uvw[t], freq[c], N, dl, weighting=weighting)
                assert np.array_equal(res["cell_idx"][t, c], one["cell_idx"])
                assert np.array_equal(res["counts"][t, c], one["counts"])
                assert res["n_out"][t, c] == one["n_out"]
                for p in range(P):
                    img, _ = O.ifft2d(one["grid"][p], one["weight_sum"], shift=True)
                    assert np.array_equal(res["images"][t, c, p], img)
                    assert res["weight_sum"][t, c, p] == one["weight_sum"]


def test_rejects_bad_arguments(O):
    with pytest.raises(ValueError):
        O.grid(np.ones((1, 4), np.complex64), None, np.zeros((4, 3)), 150e6, 12, 0.01)
    with pytest.raises(ValueError):
        O.ifft2d(np.ones((6, 6)), 1.0)
