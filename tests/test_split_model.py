"""CPU tests of the split-precision numerical model (tests/split_model.py): it reproduces the
exact transform when no rounding is applied, and predicts that split FP16/BF16 meet a relative
L2 of 1e-3 against FP64 while unsplit BF16 does not (the negative control)."""
import numpy as np
import pytest

import split_model as sm


def grid(N, seed=0):
    g = np.random.default_rng(seed)
    return g.normal(size=(N, N)) + 1j * g.normal(size=(N, N))


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_real_embedding_is_the_inverse_dft16():
    M = sm.dft16_real()
    x = np.random.default_rng(3).normal(size=16) + 1j * np.random.default_rng(4).normal(size=16)
    xr = np.empty(32)
    xr[0::2], xr[1::2] = x.real, x.imag
    y = M @ xr
    ref = np.fft.ifft(x) * 16
    assert np.abs(y[0::2] + 1j * y[1::2] - ref).max() < 1e-6


def test_bf16_rounding_is_nearest_even():
    assert sm.round_bf16(1.0 + 2.0 ** -8) == 1.0                  # tie -> even (1.0)
    assert sm.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6   # tie -> even (upper)
    assert sm.round_bf16(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7       # representable
    assert sm.round_bf16(-3.0) == -3.0


@pytest.mark.parametrize("N", [256, 4096])
def test_model_stages_without_rounding_are_exact(N, monkeypatch):
    monkeypatch.setitem(sm.ROUND, "f16", lambda x: np.asarray(x, np.float64))
    x = grid(N)[:4] if N == 4096 else grid(N)
    got = sm.fft_rows(x, "f16", split=True)
    ref = np.fft.ifft(x, axis=1) * N
    assert rel(got, ref) < 1e-6              # FP32 twiddles and stage outputs only


def test_split_forms_meet_the_target_and_unsplit_bf16_does_not():
    N = 256
    G = grid(N, seed=7)
    ref = np.fft.ifft2(G) * N * N
    err = {(k, s): rel(sm.ifft2_model(G, k, s), ref) for k in ("f16", "bf16") for s in (True, False)}
    assert err[("f16", True)] < 1e-5
    assert err[("bf16", True)] < 1e-4
    assert err[("bf16", False)] > 1e-3      # negative control
    assert err[("f16", True)] < err[("f16", False)] and err[("bf16", True)] < err[("bf16", False)]


def test_three_stage_rows_4096():
    x = grid(4096, seed=9)[:8]
    ref = np.fft.ifft(x, axis=1) * 4096
    assert rel(sm.fft_rows(x, "f16", True), ref) < 1e-5
    assert rel(sm.fft_rows(x, "bf16", True), ref) < 1e-4
    assert rel(sm.fft_rows(x, "bf16", False), ref) > 1e-3
