"""Numerical model (plain numpy, CPU) of the split-precision radix-16 FFT stages.

It predicts the error of the matrix-core precision forms before any kernel runs, and serves as
the negative control: the same stages with unsplit BF16 operands miss a relative L2 of 1e-3.
The model follows the kernels' arithmetic, not their code: each radix-16 stage multiplies by
FP32 twiddles, rounds every operand of the real 32 x 32 DFT matrix and of the data to the 16-bit
type (hi) and, when split, rounds the remainder again (lo), forms lo*hi + hi*lo + hi*hi (or hi*hi
alone) exactly and rounds the sum to FP32. FP16 data are first scaled by a power of two so that
the largest part lies in [32, 64).
"""
import numpy as np


def round_f16(x):
    return np.asarray(x, np.float64).astype(np.float16).astype(np.float64)


def round_bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


ROUND = {"f16": round_f16, "bf16": round_bf16}


def dft16_real():
    """Real 32 x 32 matrix of the 16-point inverse DFT on interleaved (re, im) vectors."""
    j = np.arange(16)
    a = 2.0 * np.pi * ((j[:, None] * j[None, :]) % 16) / 16.0
    c, s = np.cos(a).astype(np.float32).astype(np.float64), np.sin(a).astype(np.float32).astype(np.float64)
    M = np.zeros((32, 32))
    M[0::2, 0::2] = c
    M[0::2, 1::2] = -s
    M[1::2, 0::2] = s
    M[1::2, 1::2] = c
    return M


def _product(X, M, kind, split):
    """X: (n, 32) real rows; returns X @ M.T under the operand model, rounded to FP32."""
    r = ROUND[kind]
    Mh = r(M)
    Xh = r(X)
    if split:
        Ml = r(M - Mh)
        Xl = r(X - Xh)
        Y = Xh @ Ml.T + Xl @ Mh.T + Xh @ Mh.T
    else:
        Y = Xh @ Mh.T
    return Y.astype(np.float32).astype(np.float64)


def fft_rows(x, kind, split):
    """Inverse FFT (+ sign, unnormalised) of every row of x (length 16^k) with the model stages."""
    x = np.asarray(x, np.complex128)
    n_rows, N = x.shape
    k = int(round(np.log(N) / np.log(16)))
    assert 16 ** k == N, "the model covers powers of 16"
    scale = 1.0
    if kind == "f16":
        mx = max(np.abs(x.real).max(), np.abs(x.imag).max())
        if mx > 0:
            scale = 2.0 ** (6 - np.frexp(mx)[1])
    x = (x * scale).astype(np.complex64).astype(np.complex128)
    M = dft16_real()
    tw = np.exp(2j * np.pi * np.arange(N) / N).astype(np.complex64)
    NB = N // 16
    b = np.arange(NB)
    m = np.arange(16)
    ns = 1
    for _ in range(k):
        kk = b & (ns - 1)
        stride = N // (ns * 16)
        X = x[:, b[:, None] + m[None, :] * NB].astype(np.complex64)
        X = (X * tw[(kk[:, None] * m[None, :] * stride) % N][None]).astype(np.complex128)
        Xr = np.empty(X.shape[:2] + (32,))
        Xr[..., 0::2] = X.real
        Xr[..., 1::2] = X.imag
        Y = _product(Xr.reshape(-1, 32), M, kind, split).reshape(n_rows, NB, 32)
        Yc = Y[..., 0::2] + 1j * Y[..., 1::2]
        out = np.empty_like(x)
        idx = (b - kk)[:, None] * 16 + kk[:, None] + m[None, :] * ns
        out[:, idx] = Yc
        x = out
        ns *= 16
    return x / scale


def ifft2_model(G, kind, split):
    """2D inverse FFT (+ sign, unnormalised): rows (u) then columns (v), FP32 between passes."""
    A = fft_rows(G, kind, split).astype(np.complex64)
    return fft_rows(A.T, kind, split).T
