"""ctypes wrapper of the FP64 CPU oracle (``libblink_ref.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the package smoke check and the
benchmark's CPU-baseline leg. The product path never imports this module.
Arguments are NumPy arrays on the host; see ``blink_ref.h`` for definitions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libblink_ref.so")
SRC = os.path.join(HERE, "blink_ref.c")

_lib = None


def compile_library(src: str, out: str) -> str:
    """gcc -O2 -fopenmp -ffp-contract=off (no fast-math) of one oracle source into a shared object."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-D_GNU_SOURCE", "-fPIC", "-shared", "-Wall", "-Wextra", "-I", HERE, "-o", tmp, src,
           "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile libblink_ref.so next to its source."""
    if force or not os.path.exists(LIB_PATH):
        compile_library(SRC, LIB_PATH)
    return LIB_PATH


def load(path: str):
    """Load an oracle shared object and declare its signatures."""
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, f64 = ctypes.c_int, ctypes.c_double
    L.blink_ref_cells_per_metre.restype = f64
    L.blink_ref_cells_per_metre.argtypes = [f64, i32, f64]
    L.blink_ref_grid.restype = i32
    L.blink_ref_grid.argtypes = [P, P, P, i32, i32, f64, i32, f64, i32, P, P, P, P, P]
    L.blink_ref_ifft1d.restype = i32
    L.blink_ref_ifft1d.argtypes = [P, i32]
    L.blink_ref_ifft2d.restype = i32
    L.blink_ref_ifft2d.argtypes = [P, i32, f64, i32, P, P]
    L.blink_ref_image_batch.restype = i32
    L.blink_ref_image_batch.argtypes = [P, P, P, P, i32, i32, i32, i32, i32, f64, i32, i32,
                                        P, P, P, P, P, i32]
    L.blink_ref_image_batch_c128.restype = i32
    L.blink_ref_image_batch_c128.argtypes = [P, P, P, P, i32, i32, i32, i32, i32, f64, i32, i32,
                                             P, P, P, P, P, i32]
    L.blink_ref_dft.restype = i32
    L.blink_ref_dft.argtypes = [P, P, P, i32, i32, f64, i32, f64, i32, i32, P, P, P]
    L.blink_ref_correct_vis.restype = i32
    L.blink_ref_correct_vis.argtypes = [P, P, P, i32, i32, i32, i32, P, i32, f64, f64, P]
    L.blink_ref_correlate.restype = i32
    L.blink_ref_correlate.argtypes = [P, i32, i32, i32, i32, i32, i32, P, P]
    L.blink_ref_dispersion_delays.restype = i32
    L.blink_ref_dispersion_delays.argtypes = [P, i32, f64, P, i32, P]
    L.blink_ref_dedisperse.restype = i32
    L.blink_ref_dedisperse.argtypes = [P, i32, i32, i32, P, i32, i32, P]
    L.blink_ref_max_threads.restype = i32
    L.blink_ref_max_threads.argtypes = []
    L.blink_ref_es_kernel.restype = f64
    L.blink_ref_es_kernel.argtypes = [f64, f64]
    L.blink_ref_es_transform.restype = f64
    L.blink_ref_es_transform.argtypes = [f64, i32, f64]
    L.blink_ref_grid_conv.restype = i32
    L.blink_ref_grid_conv.argtypes = [P, P, P, i32, i32, f64, i32, f64, i32, f64, P, P, P]
    L.blink_ref_conv_correction.restype = i32
    L.blink_ref_conv_correction.argtypes = [i32, i32, f64, i32, P]
    L.blink_ref_image_average.restype = i32
    L.blink_ref_image_average.argtypes = [P, i32, i32, i32, i32, i32, P]
    L.blink_ref_image_batch_conv.restype = i32
    L.blink_ref_image_batch_conv.argtypes = [P, P, P, P, i32, i32, i32, i32, i32, f64, i32, f64, i32, P, P, P,
                                             i32]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        _lib = load(LIB_PATH)
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Oracle:
    """The oracle's entry points bound to one loaded copy of the library."""

    def __init__(self, L):
        self.L = L

    def cells_per_metre(self, freq_hz: float, grid_n: int, pixel_scale: float) -> float:
        return self.L.blink_ref_cells_per_metre(float(freq_hz), int(grid_n), float(pixel_scale))

    def grid(self, vis, flags, uvw, freq_hz, grid_n, pixel_scale, weighting=0):
        """Grid one (t,c): vis complex [P][B] (or [B]), flags [B] or None, uvw [B][3].

        Returns dict(grid complex128 [P][N][N], counts int32 [N][N], cell_idx int32 [B],
        weight_sum float, n_out int)."""
        vis = np.asarray(vis)
        if vis.ndim == 1:
            vis = vis[None]
        P, B = vis.shape
        v = _c(vis, np.complex64)
        f = None if flags is None else _c(flags, np.uint8)
        u = _c(uvw, np.float64)
        N = int(grid_n)
        g = np.empty((P, N, N), dtype=np.complex128)
        counts = np.empty((N, N), dtype=np.int32)
        cell = np.empty(B, dtype=np.int32)
        W = ctypes.c_double()
        nout = ctypes.c_int32()
        rc = self.L.blink_ref_grid(_ptr(v), _ptr(f), _ptr(u), P, B, float(freq_hz), N, float(pixel_scale),
                                  int(weighting), _ptr(g), _ptr(counts), _ptr(cell), ctypes.byref(W),
                                  ctypes.byref(nout))
        if rc != 0:
            raise ValueError(f"blink_ref_grid failed with code {rc}")
        return {"grid": g, "counts": counts, "cell_idx": cell, "weight_sum": W.value,
                "n_out": nout.value}

    def dft(self, vis, flags, uvw, freq_hz, grid_n, pixel_scale, snap=False, shift=True):
        """Direct transform of one (t,c): vis complex [P][B] (or [B]), flags [B] or None, uvw [B][3];
        natural weighting; nearest cells with snap, exact positions without. Returns
        dict(images float64 [P][N][N], weight_sum float, n_out int)."""
        vis = np.asarray(vis)
        if vis.ndim == 1:
            vis = vis[None]
        P, B = vis.shape
        v = _c(vis, np.complex64)
        f = None if flags is None else _c(flags, np.uint8)
        u = _c(uvw, np.float64)
        N = int(grid_n)
        img = np.empty((P, N, N), dtype=np.float64)
        W = ctypes.c_double()
        nout = ctypes.c_int32()
        rc = self.L.blink_ref_dft(_ptr(v), _ptr(f), _ptr(u), P, B, float(freq_hz), N, float(pixel_scale),
                                 int(bool(snap)), int(bool(shift)), _ptr(img), ctypes.byref(W), ctypes.byref(nout))
        if rc != 0:
            raise ValueError(f"blink_ref_dft failed with code {rc}")
        return {"images": img, "weight_sum": W.value, "n_out": nout.value}

    def ifft1d(self, x):
        a = _c(x, np.complex128).copy()
        rc = self.L.blink_ref_ifft1d(_ptr(a), a.shape[0])
        if rc != 0:
            raise ValueError(f"blink_ref_ifft1d failed with code {rc}")
        return a

    def ifft2d(self, grid_, weight_sum=1.0, shift=True):
        """Dirty image of one complex grid [N][N]. Returns (image float64 [N][N], imag_max)."""
        g = _c(grid_, np.complex128)
        N = g.shape[0]
        img = np.empty((N, N), dtype=np.float64)
        im = ctypes.c_double()
        rc = self.L.blink_ref_ifft2d(_ptr(g), N, float(weight_sum), int(bool(shift)), _ptr(img),
                                    ctypes.byref(im))
        if rc != 0:
            raise ValueError(f"blink_ref_ifft2d failed with code {rc}")
        return img, im.value

    def image_batch(self, vis, flags, uvw, freq_hz, grid_n, pixel_scale, weighting=0, shift=True,
                    n_threads=0, want_counts=False):
        """Whole path over vis [T][C][P][B]. Returns dict(images [T][C][P][N][N] float64,
        weight_sum [T][C][P], n_out [T][C], cell_idx [T][C][B], counts [T][C][N][N] or None)."""
        v = _c(vis, np.complex64)
        T, C, P, B = v.shape
        f = None if flags is None else _c(flags, np.uint8)
        u = _c(uvw, np.float64)
        fr = _c(freq_hz, np.float64)
        N = int(grid_n)
        images = np.empty((T, C, P, N, N), dtype=np.float64)
        W = np.empty((T, C, P), dtype=np.float64)
        nout = np.empty((T, C), dtype=np.int32)
        cell = np.empty((T, C, B), dtype=np.int32)
        counts = np.empty((T, C, N, N), dtype=np.int32) if want_counts else None
        rc = self.L.blink_ref_image_batch(_ptr(v), _ptr(f), _ptr(u), _ptr(fr), T, C, P, B, N,
                                         float(pixel_scale), int(weighting), int(bool(shift)),
                                         _ptr(images), _ptr(W), _ptr(nout), _ptr(cell), _ptr(counts),
                                         int(n_threads))
        if rc != 0:
            raise ValueError(f"blink_ref_image_batch failed with code {rc}")
        return {"images": images, "weight_sum": W, "n_out": nout, "cell_idx": cell, "counts": counts}

    def image_batch_c128(self, vis, flags, uvw, freq_hz, grid_n, pixel_scale, weighting=0, shift=True,
                         n_threads=0):
        """image_batch on complex double visibilities [T][C][P][B] (no rounding to complex64)."""
        v = _c(vis, np.complex128)
        T, C, P, B = v.shape
        f = None if flags is None else _c(flags, np.uint8)
        u = _c(uvw, np.float64)
        fr = _c(freq_hz, np.float64)
        N = int(grid_n)
        images = np.empty((T, C, P, N, N), dtype=np.float64)
        W = np.empty((T, C, P), dtype=np.float64)
        nout = np.empty((T, C), dtype=np.int32)
        rc = self.L.blink_ref_image_batch_c128(_ptr(v), _ptr(f), _ptr(u), _ptr(fr), T, C, P, B, N,
                                              float(pixel_scale), int(weighting), int(bool(shift)),
                                              _ptr(images), _ptr(W), _ptr(nout), None, None, int(n_threads))
        if rc != 0:
            raise ValueError(f"blink_ref_image_batch_c128 failed with code {rc}")
        return {"images": images, "weight_sum": W, "n_out": nout}

    def correct_vis(self, vis, uvw, freq_hz, gains=None, l0=0.0, m0=0.0):
        """Corrected visibilities (complex128 [T][C][P][B]): per-antenna factors gains
        [C][P][A] (complex64, or None) and the phase-centre rotation to (l0, m0)."""
        v = _c(vis, np.complex64)
        T, C, P, B = v.shape
        u = _c(uvw, np.float64)
        fr = _c(freq_hz, np.float64)
        g = None if gains is None else _c(gains, np.complex64)
        A = 0 if g is None else g.shape[-1]
        out = np.empty((T, C, P, B), dtype=np.complex128)
        rc = self.L.blink_ref_correct_vis(_ptr(v), _ptr(u), _ptr(fr), T, C, P, B, _ptr(g), int(A), float(l0),
                                         float(m0), _ptr(out))
        if rc != 0:
            raise ValueError(f"blink_ref_correct_vis failed with code {rc}")
        return out

    def image_batch_corrected(self, vis, flags, uvw, freq_hz, grid_n, pixel_scale, weighting=0, gains=None,
                              l0=0.0, m0=0.0, shift=True, n_threads=0):
        """Corrections, then the whole path on the complex double corrected visibilities."""
        vc = self.correct_vis(vis, uvw, freq_hz, gains, l0, m0)
        return self.image_batch_c128(vc, flags, uvw, freq_hz, grid_n, pixel_scale, weighting, shift, n_threads)

    def correlate(self, volt, n_int, n_favg, pol_mode=4):
        """Visibilities of int8 voltages [S][F][A][2][2] (re, im): dict(vis complex64 [T][C][P][B],
        autos complex64 [T][C][A][4])."""
        v = _c(volt, np.int8)
        S, F, A = v.shape[:3]
        assert v.shape[3:] == (2, 2)
        T, C = S // n_int, F // n_favg
        B = A * (A - 1) // 2
        vis = np.empty((T, C, pol_mode, B), dtype=np.complex64)
        autos = np.empty((T, C, A, 4), dtype=np.complex64)
        rc = self.L.blink_ref_correlate(_ptr(v), S, F, A, int(n_int), int(n_favg), int(pol_mode), _ptr(vis),
                                       _ptr(autos))
        if rc != 0:
            raise ValueError(f"blink_ref_correlate failed with code {rc}")
        return {"vis": vis, "autos": autos}

    def dispersion_delays(self, freq_hz, dt_s, dms):
        """Integer delays [n_dm][C] (samples of dt_s) of dispersion measures dms at channels freq_hz."""
        fr = _c(freq_hz, np.float64)
        d = _c(np.atleast_1d(dms), np.float64)
        out = np.empty((d.shape[0], fr.shape[0]), dtype=np.int32)
        rc = self.L.blink_ref_dispersion_delays(_ptr(fr), fr.shape[0], float(dt_s), _ptr(d), d.shape[0], _ptr(out))
        if rc != 0:
            raise ValueError(f"blink_ref_dispersion_delays failed with code {rc}")
        return out

    def dedisperse(self, images, delays, t_out):
        """De-dispersed images [n_dm][t_out][N][N] (float64) of images [T][C][N][N] (float32)."""
        a = _c(images, np.float32)
        T, C, N, _ = a.shape
        dl = _c(delays, np.int32)
        out = np.empty((dl.shape[0], int(t_out), N, N), dtype=np.float64)
        rc = self.L.blink_ref_dedisperse(_ptr(a), T, C, N, _ptr(dl), dl.shape[0], int(t_out), _ptr(out))
        if rc != 0:
            raise ValueError(f"blink_ref_dedisperse failed with code {rc}")
        return out

    def max_threads(self) -> int:
        return int(self.L.blink_ref_max_threads())

    def image_average(self, images, axes):
        """Average float images [T][C][P][N][N] over the axes in `axes` (1 time, 2 channel,
        4 polarisation); returns float64 [T'][C'][P'][N][N]."""
        a = _c(images, np.float32)
        T, C, P, N, _ = a.shape
        shape = (1 if axes & 1 else T, 1 if axes & 2 else C, 1 if axes & 4 else P, N, N)
        out = np.empty(shape, dtype=np.float64)
        rc = self.L.blink_ref_image_average(_ptr(a), T, C, P, N, int(axes), _ptr(out))
        if rc != 0:
            raise ValueError(f"blink_ref_image_average failed with code {rc}")
        return out

    # -- convolutional gridding (exponential-of-semicircle kernel, grid correction)
    def es_kernel(self, z: float, beta: float) -> float:
        return self.L.blink_ref_es_kernel(float(z), float(beta))

    def es_transform(self, nu: float, width: int, beta: float) -> float:
        return self.L.blink_ref_es_transform(float(nu), int(width), float(beta))

    def grid_conv(self, vis, flags, uvw, freq_hz, grid_n, pixel_scale, width, beta):
        """Convolutional gridding of one (t,c): vis complex [P][B] (or [B]). Returns dict(grid
        complex128 [P][N][N], weight_sum, n_out)."""
        vis = np.asarray(vis)
        if vis.ndim == 1:
            vis = vis[None]
        P, B = vis.shape
        v = _c(vis, np.complex64)
        f = None if flags is None else _c(flags, np.uint8)
        u = _c(uvw, np.float64)
        N = int(grid_n)
        g = np.empty((P, N, N), dtype=np.complex128)
        W = ctypes.c_double()
        nout = ctypes.c_int32()
        rc = self.L.blink_ref_grid_conv(_ptr(v), _ptr(f), _ptr(u), P, B, float(freq_hz), N, float(pixel_scale),
                                       int(width), float(beta), _ptr(g), ctypes.byref(W), ctypes.byref(nout))
        if rc != 0:
            raise ValueError(f"blink_ref_grid_conv failed with code {rc}")
        return {"grid": g, "weight_sum": W.value, "n_out": nout.value}

    def conv_correction(self, grid_n, width, beta, shift=True):
        corr = np.empty(int(grid_n), dtype=np.float64)
        rc = self.L.blink_ref_conv_correction(int(grid_n), int(width), float(beta), int(bool(shift)), _ptr(corr))
        if rc != 0:
            raise ValueError(f"blink_ref_conv_correction failed with code {rc}")
        return corr

    def image_batch_conv(self, vis, flags, uvw, freq_hz, grid_n, pixel_scale, width, beta, shift=True,
                         n_threads=0):
        """Convolutional path over vis [T][C][P][B]: dict(images, weight_sum, n_out)."""
        v = _c(vis, np.complex64)
        T, C, P, B = v.shape
        f = None if flags is None else _c(flags, np.uint8)
        u = _c(uvw, np.float64)
        fr = _c(freq_hz, np.float64)
        N = int(grid_n)
        images = np.empty((T, C, P, N, N), dtype=np.float64)
        W = np.empty((T, C, P), dtype=np.float64)
        nout = np.empty((T, C), dtype=np.int32)
        rc = self.L.blink_ref_image_batch_conv(_ptr(v), _ptr(f), _ptr(u), _ptr(fr), T, C, P, B, N,
                                              float(pixel_scale), int(width), float(beta), int(bool(shift)),
                                              _ptr(images), _ptr(W), _ptr(nout), int(n_threads))
        if rc != 0:
            raise ValueError(f"blink_ref_image_batch_conv failed with code {rc}")
        return {"images": images, "weight_sum": W, "n_out": nout}


def default() -> Oracle:
    return Oracle(lib())


def cells_per_metre(*a, **k):
    return default().cells_per_metre(*a, **k)


def grid(*a, **k):
    return default().grid(*a, **k)


def dft(*a, **k):
    return default().dft(*a, **k)


def ifft1d(*a, **k):
    return default().ifft1d(*a, **k)


def ifft2d(*a, **k):
    return default().ifft2d(*a, **k)


def image_batch(*a, **k):
    return default().image_batch(*a, **k)


def image_batch_c128(*a, **k):
    return default().image_batch_c128(*a, **k)


def correct_vis(*a, **k):
    return default().correct_vis(*a, **k)


def image_batch_corrected(*a, **k):
    return default().image_batch_corrected(*a, **k)


def correlate(*a, **k):
    return default().correlate(*a, **k)


def dispersion_delays(*a, **k):
    return default().dispersion_delays(*a, **k)


def dedisperse(*a, **k):
    return default().dedisperse(*a, **k)


def max_threads() -> int:
    return default().max_threads()


def image_average(*a, **k):
    return default().image_average(*a, **k)


def es_kernel(*a, **k):
    return default().es_kernel(*a, **k)


def es_transform(*a, **k):
    return default().es_transform(*a, **k)


def grid_conv(*a, **k):
    return default().grid_conv(*a, **k)


def conv_correction(*a, **k):
    return default().conv_correction(*a, **k)


def image_batch_conv(*a, **k):
    return default().image_batch_conv(*a, **k)
