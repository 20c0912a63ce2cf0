"""MI355X batched dirty imaging (BLINK's gridding + inverse 2D FFT hot path).

Thin ctypes binding of ``libblink.so`` (declared in ``include/blink.h``). The functions
take torch tensors that already live on the GPU and pass their device pointers and the
current HIP stream to the library; every step of the computation runs in the library's
HIP kernels. PyTorch is used only to allocate device memory (outputs, workspace) and for
streams. There is no CPU fallback: if the library is missing, calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libblink.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "blink.h")
PLANS_PATH = os.path.join(PKG, "plans_gfx950.json")     # autotuned execution plans (blink_set_plan)

BLINK_OK, BLINK_ERR_ARG, BLINK_ERR_SIZE, BLINK_ERR_NOMEM, BLINK_ERR_HIP, BLINK_ERR_STATE = range(6)
WEIGHT_NATURAL, WEIGHT_UNIFORM = 0, 1
KERNELS = ("bin", "grid", "grid_colfft", "dense_colfft", "weights", "row_fft", "desc_prep", "persistent",
           "conv_correction", "average", "correct", "correlate", "dedisperse")
AVG_TIME, AVG_CHANNEL, AVG_POL = 1, 2, 4   # BLINK_KERNEL_* ids
DESC_BAD = 1
DESC_PERSISTENT, DESC_STAGED = 0, 1   # BLINK_DESC_PERSISTENT / BLINK_DESC_STAGED: forms of the uneven-batch path

# blink_image_desc as a NumPy structured dtype (64 bytes, C layout)
import numpy as _np  # noqa: E402

DESC_DTYPE = _np.dtype([("vis_offset", "<i8"), ("uvw_offset", "<i8"), ("flag_offset", "<i8"),
                        ("image_offset", "<i8"), ("freq_hz", "<f8"), ("pixel_scale", "<f8"),
                        ("n_baselines", "<i4"), ("grid_n", "<i4"), ("reserved", "<i4", (2,))])
assert DESC_DTYPE.itemsize == 64
STATIC_SCRATCH_BYTES = 64 << 20   # BLINK_STATIC_SCRATCH_BYTES (blink_image_batch_noalloc)
PREC_FP32 = 0            # BLINK_PREC_FP32: FP32 radix-16 butterflies
PREC_SPLIT_F16 = 1       # BLINK_PREC_SPLIT_F16: matrix-core radix-16 stages, FP16 hi + lo operands
PREC_SPLIT_BF16 = 2      # BLINK_PREC_SPLIT_BF16: the same with BF16 operands
PRECISIONS = (PREC_FP32, PREC_SPLIT_F16, PREC_SPLIT_BF16)

_lib = None


class BlinkError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


class Problem(ctypes.Structure):
    """blink_problem: one entry point's problem for the single workspace query."""
    _fields_ = [(n, ctypes.c_int) for n in ("entry", "T", "C", "P", "B", "n_img", "grid_n", "weighting", "precision",
                                            "kernel_width", "max_baselines", "workgroups", "n_dm")]


ENTRY_GRID, ENTRY_IFFT2D, ENTRY_IMAGE_BATCH, ENTRY_IMAGE_BATCH_CORRECTED, ENTRY_IMAGE_BATCH_CONV, \
    ENTRY_IMAGE_BATCH_DESC, ENTRY_DEDISPERSE = range(7)


class Corrections(ctypes.Structure):
    """blink_corrections: per-antenna factors (device pointer or None), antennas, phase centre."""
    _fields_ = [("gains", ctypes.c_void_p), ("n_ant", ctypes.c_int), ("l0", ctypes.c_double),
                ("m0", ctypes.c_double)]


def header_functions() -> list:
    """Names of the functions declared in include/blink.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(blink_[a-z0-9_]+)\s*\(", text)))


def lib() -> ctypes.CDLL:
    """Load libblink.so and declare its signatures. Raises if the library was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2505_15204_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, f64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    L.blink_version.restype = i32
    L.blink_status_string.restype = ctypes.c_char_p
    L.blink_status_string.argtypes = [i32]
    L.blink_create.restype = i32
    L.blink_create.argtypes = [ctypes.POINTER(P), i32]
    L.blink_destroy.restype = i32
    L.blink_destroy.argtypes = [P]
    L.blink_last_error.restype = ctypes.c_char_p
    L.blink_last_error.argtypes = [P]
    L.blink_grid_workspace_size.restype = i32
    L.blink_workspace_size.restype = i32
    L.blink_workspace_size.argtypes = [P, ctypes.POINTER(Problem), ctypes.POINTER(sz)]
    L.blink_grid_workspace_size.argtypes = [i32, i32, i32, i32, ctypes.POINTER(sz)]
    L.blink_ifft2d_workspace_size.restype = i32
    L.blink_ifft2d_workspace_size.argtypes = [i32, i32, i32, ctypes.POINTER(sz)]
    L.blink_image_batch_workspace_size.restype = i32
    L.blink_image_batch_workspace_size.argtypes = [i32, i32, i32, i32, i32, i32, i32, ctypes.POINTER(sz)]
    L.blink_grid.restype = i32
    L.blink_grid.argtypes = [P, P, P, P, P, i32, i32, i32, i32, i32, f64, i32, P, P, P, P, P, P, sz, P]
    L.blink_ifft2d.restype = i32
    L.blink_ifft2d.argtypes = [P, P, P, i32, i32, i32, i32, P, P, sz, P]
    L.blink_image_batch.restype = i32
    L.blink_image_batch.argtypes = [P, P, P, P, P, i32, i32, i32, i32, i32, f64, i32, i32, i32, P, P, P,
                                    P, sz, P]
    L.blink_image_batch_corrected_workspace_size.restype = i32
    L.blink_image_batch_noalloc.argtypes = [P, P, P, P, P, i32, i32, i32, i32, i32, f64, i32, i32, i32, P, P, P, P]
    L.blink_image_batch_noalloc.restype = i32
    L.blink_image_batch_corrected_workspace_size.argtypes = [i32, i32, i32, i32, i32, i32, i32, ctypes.POINTER(sz)]
    L.blink_image_batch_corrected.restype = i32
    L.blink_image_batch_corrected.argtypes = [P, P, P, P, P, i32, i32, i32, i32, i32, f64, i32, i32, i32,
                                              ctypes.POINTER(Corrections), P, P, P, P, sz, P]
    L.blink_correlate.restype = i32
    L.blink_correlate.argtypes = [P, P, i32, i32, i32, i32, i32, i32, P, P, P]
    L.blink_dispersion_delays.restype = i32
    L.blink_dispersion_delays.argtypes = [P, i32, f64, P, i32, P]
    L.blink_dedisperse_workspace_size.restype = i32
    L.blink_dedisperse_workspace_size.argtypes = [i32, i32, ctypes.POINTER(sz)]
    L.blink_dedisperse.restype = i32
    L.blink_dedisperse.argtypes = [P, P, i32, i32, i32, P, i32, i32, P, P, sz, P]
    L.blink_plan_options.restype = i32
    L.blink_plan_options.argtypes = [i32, i32, P, P, P, P]
    L.blink_get_plan.restype = i32
    L.blink_get_plan.argtypes = [P, i32, i32, i32, P, P, P, P]
    L.blink_set_plan.restype = i32
    L.blink_set_plan.argtypes = [P, i32, i32, i32, i32, i32, i32, i32]
    L.blink_image_batch_conv_workspace_size.restype = i32
    L.blink_image_batch_conv_workspace_size.argtypes = [i32, i32, i32, i32, i32, i32, i32, ctypes.POINTER(sz)]
    L.blink_image_batch_conv.restype = i32
    L.blink_image_batch_conv.argtypes = [P, P, P, P, P, i32, i32, i32, i32, i32, f64, i32, f64, i32, i32, P, P, P,
                                         P, sz, P]
    L.blink_image_average.restype = i32
    L.blink_image_average.argtypes = [P, P, i32, i32, i32, i32, i32, P, P]
    L.blink_autotune_image_batch.restype = i32
    L.blink_autotune_image_batch.argtypes = [P, P, P, P, P, i32, i32, i32, i32, i32, f64, i32, i32, i32, P, P,
                                             P, P, sz, P, P, P, P, P, P]
    i64 = ctypes.c_int64
    desc_args = [P, P, i32, P, i64, P, i64, P, i64, i32, i32, i32, i32, i32, P, i64, P, P, P, P, sz]
    L.blink_desc_workspace_size.restype = i32
    L.blink_desc_workspace_size.argtypes = [i32, i32, i32, i32, ctypes.POINTER(sz)]
    L.blink_image_batch_desc.restype = i32
    L.blink_image_batch_desc.argtypes = desc_args + [P]
    L.blink_get_desc_plan.restype = i32
    L.blink_get_desc_plan.argtypes = [P, P, P]
    L.blink_set_desc_plan.restype = i32
    L.blink_set_desc_plan.argtypes = [P, i32, i32]
    L.blink_get_desc_form.restype = i32
    L.blink_get_desc_form.argtypes = [P, P]
    L.blink_set_desc_form.restype = i32
    L.blink_set_desc_form.argtypes = [P, i32]
    L.blink_autotune_desc.restype = i32
    L.blink_autotune_desc.argtypes = desc_args + [P, P, P, P]
    L.blink_graph_create_desc.restype = i32
    L.blink_graph_create_desc.argtypes = desc_args + [ctypes.POINTER(P)]
    L.blink_graph_launch.restype = i32
    L.blink_graph_launch.argtypes = [P, P]
    L.blink_graph_destroy.restype = i32
    L.blink_graph_destroy.argtypes = [P]
    L.blink_profile_enable.restype = i32
    L.blink_profile_enable.argtypes = [P, i32]
    L.blink_profile_read.restype = i32
    L.blink_profile_read.argtypes = [P, i32, ctypes.POINTER(f64), ctypes.POINTER(ctypes.c_int64)]
    _lib = L
    return L


def status_string(st: int) -> str:
    return lib().blink_status_string(st).decode()


def _check(st: int, ctx=None, what: str = ""):
    if st != BLINK_OK:
        detail = lib().blink_last_error(ctx).decode() if ctx else ""
        raise BlinkError(st, f"{what}: {status_string(st)}" + (f" ({detail})" if detail else ""))


def workspace_size(entry: int, **fields) -> int:
    """Workspace bytes of an entry point (ENTRY_*) for the problem given by blink_problem's fields."""
    p = Problem(entry=entry, **fields)
    n = ctypes.c_size_t()
    _check(lib().blink_workspace_size(None, ctypes.byref(p), ctypes.byref(n)), None, what="blink_workspace_size")
    return n.value


def grid_workspace_size(T: int, C: int, B: int, grid_n: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().blink_grid_workspace_size(T, C, B, grid_n, ctypes.byref(n)), what="blink_grid_workspace_size")
    return n.value


def ifft2d_workspace_size(n_img: int, grid_n: int, precision: int = PREC_FP32) -> int:
    n = ctypes.c_size_t()
    _check(lib().blink_ifft2d_workspace_size(n_img, grid_n, precision, ctypes.byref(n)),
           what="blink_ifft2d_workspace_size")
    return n.value


def image_batch_workspace_size(T: int, C: int, P: int, B: int, grid_n: int, weighting: int = 0,
                               precision: int = PREC_FP32) -> int:
    n = ctypes.c_size_t()
    _check(lib().blink_image_batch_workspace_size(T, C, P, B, grid_n, weighting, precision, ctypes.byref(n)),
           what="blink_image_batch_workspace_size")
    return n.value


def image_batch_corrected_workspace_size(T: int, C: int, P: int, B: int, grid_n: int, weighting: int = 0,
                                         precision: int = PREC_FP32) -> int:
    n = ctypes.c_size_t()
    _check(lib().blink_image_batch_corrected_workspace_size(T, C, P, B, grid_n, weighting, precision,
                                                            ctypes.byref(n)),
           what="blink_image_batch_corrected_workspace_size")
    return n.value


def dispersion_delays(freq_hz, dt_s: float, dms):
    """Integer delays [n_dm][C] (int32 NumPy, steps of dt_s) of the trial DMs at channel frequencies
    freq_hz (host arrays; blink_dispersion_delays)."""
    import numpy as np
    fr = np.ascontiguousarray(freq_hz, dtype=np.float64)
    dm = np.ascontiguousarray(np.atleast_1d(dms), dtype=np.float64)
    out = np.empty((dm.shape[0], fr.shape[0]), dtype=np.int32)
    _check(lib().blink_dispersion_delays(fr.ctypes.data_as(ctypes.c_void_p), fr.shape[0], float(dt_s),
                                         dm.ctypes.data_as(ctypes.c_void_p), dm.shape[0],
                                         out.ctypes.data_as(ctypes.c_void_p)), what="blink_dispersion_delays")
    return out


def dedisperse_workspace_size(C: int, n_dm: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().blink_dedisperse_workspace_size(C, n_dm, ctypes.byref(n)), what="blink_dedisperse_workspace_size")
    return n.value


def image_batch_conv_workspace_size(T: int, C: int, P: int, B: int, grid_n: int, kernel_width: int,
                                    precision: int = PREC_FP32) -> int:
    n = ctypes.c_size_t()
    _check(lib().blink_image_batch_conv_workspace_size(T, C, P, B, grid_n, kernel_width, precision, ctypes.byref(n)),
           what="blink_image_batch_conv_workspace_size")
    return n.value


def plan_options(grid_n: int, weighting: int = 0):
    """Compiled (col_strip, row_block) options for a grid size: two lists, largest first."""
    col = (ctypes.c_int * 4)()
    row = (ctypes.c_int * 4)()
    nc, nr = ctypes.c_int(), ctypes.c_int()
    _check(lib().blink_plan_options(grid_n, weighting, col, ctypes.byref(nc), row, ctypes.byref(nr)),
           what="blink_plan_options")
    return list(col)[:nc.value], list(row)[:nr.value]


def desc_workspace_size(n_img: int, max_baselines: int, max_grid_n: int, workgroups: int = 512) -> int:
    n = ctypes.c_size_t()
    _check(lib().blink_desc_workspace_size(n_img, max_baselines, max_grid_n, workgroups, ctypes.byref(n)),
           what="blink_desc_workspace_size")
    return n.value


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _on_stream(method):
    """Run an entry method with the caller's `stream` as torch's current stream, so that every
    tensor the binding allocates for the call (workspace, outputs) belongs to the stream the
    kernels run on: torch's caching allocator then reuses the workspace, which is freed when the
    method returns, only behind the work queued on that stream."""
    import functools

    @functools.wraps(method)
    def wrapper(self, *args, **kwargs):
        stream = kwargs.get("stream")
        if stream is None:
            return method(self, *args, **kwargs)
        import torch
        with torch.cuda.device(self.device), torch.cuda.stream(stream):
            return method(self, *args, **kwargs)
    return wrapper


class Context:
    """One library context (device tables and error state) on a HIP device."""

    def __init__(self, device: int = 0):
        import torch  # noqa: F401  (device memory and streams come from torch)

        self.device = device
        h = ctypes.c_void_p()
        st = lib().blink_create(ctypes.byref(h), device)
        _check(st, None, f"blink_create(device={device})")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().blink_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- kernel timing (hipEvents around every launch while enabled)
    def profile_enable(self, enable: bool = True):
        _check(lib().blink_profile_enable(self.handle, int(bool(enable))), self.handle, "blink_profile_enable")

    def profile_read(self) -> dict:
        """{kernel name: (total ms, launches)} for every kernel id; waits for the recorded events."""
        out = {}
        for k, name in enumerate(KERNELS):
            ms = ctypes.c_double()
            n = ctypes.c_int64()
            _check(lib().blink_profile_read(self.handle, k, ctypes.byref(ms), ctypes.byref(n)), self.handle,
                   "blink_profile_read")
            out[name] = (ms.value, n.value)
        return out

    # -- execution plans (scheduling only; results are the same up to rounding order)
    def get_plan(self, grid_n: int, weighting: int = 0, precision: int = PREC_FP32) -> dict:
        c, r, g, lp = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().blink_get_plan(self.handle, grid_n, weighting, precision, ctypes.byref(c), ctypes.byref(r),
                                    ctypes.byref(g), ctypes.byref(lp)), self.handle, "blink_get_plan")
        return {"col_strip": c.value, "row_block": r.value, "group": g.value, "col_loop": lp.value}

    def set_plan(self, grid_n: int, weighting: int = 0, col_strip: int = 0, row_block: int = 0, group: int = 0,
                 precision: int = PREC_FP32, col_loop: int = 1):
        _check(lib().blink_set_plan(self.handle, grid_n, weighting, precision, col_strip, row_block, group, col_loop),
               self.handle, "blink_set_plan")

    def save_plans(self, path: str, sizes=(256, 512, 1024, 2048, 4096), precisions=PRECISIONS):
        """Write the context's plans as JSON keyed by device name, grid size, weighting and precision."""
        import json
        torch = self._torch()
        name = torch.cuda.get_device_properties(self.device).gcnArchName
        rec = {f"{name}/{n}/{w}/{p}": self.get_plan(n, w, p) for n in sizes for w in (0, 1) for p in precisions}
        with open(path, "w") as fh:
            json.dump(rec, fh, indent=1, sort_keys=True)

    def load_plans(self, path: str):
        """Apply the plans of this device from a file written by save_plans (keys without a
        precision field are FP32 plans; plans without col_loop take one strip per workgroup)."""
        import json
        torch = self._torch()
        name = torch.cuda.get_device_properties(self.device).gcnArchName
        for key, p in json.load(open(path)).items():
            parts = key.split("/")
            if parts[-1].isdigit() and parts[-2].isdigit() and parts[-3].isdigit():
                dev, n, w, prec = "/".join(parts[:-3]), parts[-3], parts[-2], parts[-1]
            else:
                dev, n, w, prec = "/".join(parts[:-2]), parts[-2], parts[-1], str(PREC_FP32)
            if dev == name:
                self.set_plan(int(n), int(w), p["col_strip"], p["row_block"], p["group"], precision=int(prec),
                              col_loop=p.get("col_loop", 1))

    @_on_stream
    def autotune_image_batch(self, vis, flags, uvw_m, freq_hz, grid_n: int, pixel_scale: float, weighting: int = 0,
                             precision: int = PREC_FP32, shift: bool = True, out=None, workspace=None, stream=None):
        """Time every compiled plan on this problem and keep the fastest; returns (plan dict, best ms)."""
        torch = self._torch()
        T, C, P, B = vis.shape
        N = int(grid_n)
        self._require("vis", vis, torch.complex64)
        self._require("uvw_m", uvw_m, torch.float64, (T, B, 3))
        self._require("freq_hz", freq_hz, torch.float64, (C,))
        if flags is not None:
            self._require("flags", flags, torch.uint8, (T, C, B))
        dev = vis.device
        if out is None:
            out = torch.empty((T, C, P, N, N), dtype=torch.float32, device=dev)
        self._require("out", out, torch.float32, (T, C, P, N, N))
        wsum = torch.empty((T, C, P), dtype=torch.float64, device=dev)
        nout = torch.empty((T, C), dtype=torch.int32, device=dev)
        ws = self._workspace(image_batch_workspace_size(T, C, P, B, N, weighting, precision), workspace)
        c, r, g, lp, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        st = lib().blink_autotune_image_batch(self.handle, _ptr(vis), _ptr(flags), _ptr(uvw_m), _ptr(freq_hz), T, C,
                                              P, B, N, float(pixel_scale), int(weighting), int(precision),
                                              int(bool(shift)), _ptr(out), _ptr(wsum), _ptr(nout), _ptr(ws),
                                              ws.numel(), self._stream(stream), ctypes.byref(c), ctypes.byref(r),
                                              ctypes.byref(g), ctypes.byref(lp), ctypes.byref(ms))
        _check(st, self.handle, "blink_autotune_image_batch")
        return {"col_strip": c.value, "row_block": r.value, "group": g.value, "col_loop": lp.value}, ms.value

    # -- uneven batches (one descriptor per image)
    def _desc_args(self, desc, vis, uvw_m, flags, images, weighting, precision, shift, weight_sum, n_out, status,
                   max_baselines, max_grid_n, workspace, workgroups_for_size=512):
        torch = self._torch()
        self._require("desc", desc, torch.uint8)
        if desc.numel() % 64:
            raise ValueError("desc must hold 64-byte blink_image_desc records (uint8 tensor)")
        n_img = desc.numel() // 64
        self._require("vis", vis, torch.complex64)
        self._require("uvw_m", uvw_m, torch.float64)
        if flags is not None:
            self._require("flags", flags, torch.uint8)
        self._require("images", images, torch.float32)
        for name, t, dt in (("weight_sum", weight_sum, torch.float64), ("n_out", n_out, torch.int32),
                            ("status", status, torch.int32)):
            if t is not None:
                self._require(name, t, dt)
        ws = self._workspace(desc_workspace_size(n_img, max_baselines, max_grid_n, workgroups_for_size), workspace)
        return [self.handle, _ptr(desc), n_img, _ptr(vis), vis.numel(), _ptr(uvw_m), uvw_m.numel() // 3,
                _ptr(flags), 0 if flags is None else flags.numel(), int(max_baselines), int(max_grid_n),
                int(weighting), int(precision), int(bool(shift)), _ptr(images), images.numel(), _ptr(weight_sum),
                _ptr(n_out), _ptr(status), _ptr(ws), ws.numel()], ws

    @_on_stream
    def blink_image_batch_desc(self, desc, vis, uvw_m, flags, images, max_baselines: int, max_grid_n: int,
                               weighting: int = 0, precision: int = PREC_FP32, shift: bool = True, weight_sum=None,
                               n_out=None, status=None, workspace=None, stream=None):
        """Uneven batch: desc is a uint8 device tensor of blink_image_desc records (DESC_DTYPE);
        vis complex64, uvw_m float64 [..][3], flags uint8 or None and images float32 are flat
        device arrays addressed by the descriptors' offsets."""
        args, ws = self._desc_args(desc, vis, uvw_m, flags, images, weighting, precision, shift, weight_sum, n_out,
                                   status, max_baselines, max_grid_n, workspace)
        st = lib().blink_image_batch_desc(*args, self._stream(stream))
        _check(st, self.handle, "blink_image_batch_desc")
        return images

    def get_desc_plan(self) -> dict:
        b, w, f = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().blink_get_desc_plan(self.handle, ctypes.byref(b), ctypes.byref(w)), self.handle,
               "blink_get_desc_plan")
        _check(lib().blink_get_desc_form(self.handle, ctypes.byref(f)), self.handle, "blink_get_desc_form")
        return {"block_threads": b.value, "workgroups": w.value, "form": f.value}

    def set_desc_plan(self, block_threads: int = 512, workgroups: int = 0, form=None):
        _check(lib().blink_set_desc_plan(self.handle, block_threads, workgroups), self.handle, "blink_set_desc_plan")
        if form is not None:
            _check(lib().blink_set_desc_form(self.handle, int(form)), self.handle, "blink_set_desc_form")

    @_on_stream
    def autotune_desc(self, desc, vis, uvw_m, flags, images, max_baselines: int, max_grid_n: int, weighting: int = 0,
                      precision: int = PREC_FP32, shift: bool = True, workspace=None, stream=None):
        args, ws = self._desc_args(desc, vis, uvw_m, flags, images, weighting, precision, shift, None, None, None,
                                   max_baselines, max_grid_n, workspace)
        b, w, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        st = lib().blink_autotune_desc(*args, self._stream(stream), ctypes.byref(b), ctypes.byref(w), ctypes.byref(ms))
        _check(st, self.handle, "blink_autotune_desc")
        return self.get_desc_plan(), ms.value

    def graph_desc(self, desc, vis, uvw_m, flags, images, max_baselines: int, max_grid_n: int, weighting: int = 0,
                   precision: int = PREC_FP32, shift: bool = True, weight_sum=None, n_out=None, status=None,
                   workspace=None):
        """Capture one blink_image_batch_desc call (these buffers) into a hipGraph; returns a Graph."""
        args, ws = self._desc_args(desc, vis, uvw_m, flags, images, weighting, precision, shift, weight_sum, n_out,
                                   status, max_baselines, max_grid_n, workspace)
        h = ctypes.c_void_p()
        st = lib().blink_graph_create_desc(*args, ctypes.byref(h))
        _check(st, self.handle, "blink_graph_create_desc")
        return Graph(self, h, keep=(ws, desc, vis, uvw_m, flags, images, weight_sum, n_out, status))

    # -- helpers
    def _torch(self):
        import torch
        return torch

    def _stream(self, stream):
        torch = self._torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(s.cuda_stream)

    def _require(self, name, t, dtype, shape=None):
        torch = self._torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.device.type != "cuda":
            raise ValueError(f"{name} must be on the GPU, got {t.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def _workspace(self, nbytes, workspace):
        torch = self._torch()
        if workspace is None:
            workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        self._require("workspace", workspace, torch.uint8)
        return workspace

    # -- entry points (same names as the C ABI)
    @_on_stream
    def blink_grid(self, vis, flags, uvw_m, freq_hz, grid_n: int, pixel_scale: float, weighting: int = 0,
                   want_counts: bool = True, want_cell_idx: bool = True, workspace=None, stream=None):
        """Nearest-cell gridding. vis complex64 [T][C][P][B]; flags uint8 [T][C][B] or None;
        uvw_m float64 [T][B][3]; freq_hz float64 [C]. Returns a dict of device tensors:
        grids complex64 [T][C][P][N][N], counts int32 [T][C][N][N], weight_sum float64 [T][C][P],
        cell_idx int32 [T][C][B], n_out int32 [T][C]."""
        torch = self._torch()
        T, C, P, B = vis.shape
        N = int(grid_n)
        self._require("vis", vis, torch.complex64)
        if flags is not None:
            self._require("flags", flags, torch.uint8, (T, C, B))
        self._require("uvw_m", uvw_m, torch.float64, (T, B, 3))
        self._require("freq_hz", freq_hz, torch.float64, (C,))
        dev = vis.device
        grids = torch.empty((T, C, P, N, N), dtype=torch.complex64, device=dev)
        counts = torch.empty((T, C, N, N), dtype=torch.int32, device=dev) if want_counts else None
        wsum = torch.empty((T, C, P), dtype=torch.float64, device=dev)
        cell = torch.empty((T, C, B), dtype=torch.int32, device=dev) if want_cell_idx else None
        nout = torch.empty((T, C), dtype=torch.int32, device=dev)
        ws = self._workspace(grid_workspace_size(T, C, B, N), workspace)
        st = lib().blink_grid(self.handle, _ptr(vis), _ptr(flags), _ptr(uvw_m), _ptr(freq_hz), T, C, P, B, N,
                              float(pixel_scale), int(weighting), _ptr(grids), _ptr(counts), _ptr(wsum),
                              _ptr(cell), _ptr(nout), _ptr(ws), ws.numel(), self._stream(stream))
        _check(st, self.handle, "blink_grid")
        return {"grids": grids, "counts": counts, "weight_sum": wsum, "cell_idx": cell, "n_out": nout}

    @_on_stream
    def blink_ifft2d(self, grids, weight_sum=None, shift: bool = True, precision: int = PREC_FP32,
                     out=None, workspace=None, stream=None):
        """Dirty images Re(IDFT2(G))/W of complex64 grids [..., N, N]; returns float32 [..., N, N]."""
        torch = self._torch()
        self._require("grids", grids, torch.complex64)
        N = int(grids.shape[-1])
        if grids.shape[-2] != N:
            raise ValueError("grids must be square")
        n_img = grids.numel() // (N * N)
        if weight_sum is not None:
            self._require("weight_sum", weight_sum, torch.float64)
            if weight_sum.numel() != n_img:
                raise ValueError("weight_sum must hold one value per grid")
        if out is None:
            out = torch.empty(grids.shape, dtype=torch.float32, device=grids.device)
        self._require("out", out, torch.float32, grids.shape)
        ws = self._workspace(ifft2d_workspace_size(n_img, N, precision), workspace)
        st = lib().blink_ifft2d(self.handle, _ptr(grids), _ptr(weight_sum), n_img, N, int(precision),
                                int(bool(shift)), _ptr(out), _ptr(ws), ws.numel(), self._stream(stream))
        _check(st, self.handle, "blink_ifft2d")
        return out

    @_on_stream
    def blink_image_batch(self, vis, flags, uvw_m, freq_hz, grid_n: int, pixel_scale: float,
                          weighting: int = 0, precision: int = PREC_FP32, shift: bool = True, out=None,
                          weight_sum=None, n_out=None, workspace=None, stream=None):
        """Fused gridding + inverse 2D FFT. Returns dict(images float32 [T][C][P][N][N],
        weight_sum float64 [T][C][P], n_out int32 [T][C]) of device tensors."""
        torch = self._torch()
        T, C, P, B = vis.shape
        N = int(grid_n)
        self._require("vis", vis, torch.complex64)
        if flags is not None:
            self._require("flags", flags, torch.uint8, (T, C, B))
        self._require("uvw_m", uvw_m, torch.float64, (T, B, 3))
        self._require("freq_hz", freq_hz, torch.float64, (C,))
        dev = vis.device
        if out is None:
            out = torch.empty((T, C, P, N, N), dtype=torch.float32, device=dev)
        self._require("out", out, torch.float32, (T, C, P, N, N))
        if weight_sum is None:
            weight_sum = torch.empty((T, C, P), dtype=torch.float64, device=dev)
        if n_out is None:
            n_out = torch.empty((T, C), dtype=torch.int32, device=dev)
        ws = self._workspace(image_batch_workspace_size(T, C, P, B, N, weighting, precision), workspace)
        st = lib().blink_image_batch(self.handle, _ptr(vis), _ptr(flags), _ptr(uvw_m), _ptr(freq_hz), T, C, P,
                                     B, N, float(pixel_scale), int(weighting), int(precision), int(bool(shift)),
                                     _ptr(out), _ptr(weight_sum), _ptr(n_out), _ptr(ws), ws.numel(),
                                     self._stream(stream))
        _check(st, self.handle, "blink_image_batch")
        return {"images": out, "weight_sum": weight_sum, "n_out": n_out}

    def blink_image_batch_noalloc(self, vis, flags, uvw_m, freq_hz, grid_n: int, pixel_scale: float,
                                  weighting: int = 0, precision: int = PREC_FP32, shift: bool = True, *, out,
                                  weight_sum=None, n_out=None, stream=None):
        """blink_image_batch without a workspace: the library's static scratch array serves instead,
        so the call allocates no device memory (the caller passes every output, `out` included;
        weight_sum and n_out may be None). Calls that overlap on one GPU race on that array."""
        torch = self._torch()
        T, C, P, B = vis.shape
        N = int(grid_n)
        self._require("vis", vis, torch.complex64)
        if flags is not None:
            self._require("flags", flags, torch.uint8, (T, C, B))
        self._require("uvw_m", uvw_m, torch.float64, (T, B, 3))
        self._require("freq_hz", freq_hz, torch.float64, (C,))
        self._require("out", out, torch.float32, (T, C, P, N, N))
        if weight_sum is not None:
            self._require("weight_sum", weight_sum, torch.float64, (T, C, P))
        if n_out is not None:
            self._require("n_out", n_out, torch.int32, (T, C))
        st = lib().blink_image_batch_noalloc(self.handle, _ptr(vis), _ptr(flags), _ptr(uvw_m), _ptr(freq_hz), T, C,
                                             P, B, N, float(pixel_scale), int(weighting), int(precision),
                                             int(bool(shift)), _ptr(out), _ptr(weight_sum), _ptr(n_out),
                                             self._stream(stream))
        _check(st, self.handle, "blink_image_batch_noalloc")
        return {"images": out, "weight_sum": weight_sum, "n_out": n_out}

    @_on_stream
    def blink_image_batch_corrected(self, vis, flags, uvw_m, freq_hz, grid_n: int, pixel_scale: float,
                                    weighting: int = 0, gains=None, l0: float = 0.0, m0: float = 0.0,
                                    precision: int = PREC_FP32, shift: bool = True, out=None, weight_sum=None,
                                    n_out=None, workspace=None, stream=None):
        """blink_image_batch on visibilities corrected by per-antenna factors gains (complex64
        device tensor [C][P][n_ant], or None) and moved to the phase centre (l0, m0)."""
        torch = self._torch()
        T, C, P, B = vis.shape
        N = int(grid_n)
        self._require("vis", vis, torch.complex64)
        if flags is not None:
            self._require("flags", flags, torch.uint8, (T, C, B))
        self._require("uvw_m", uvw_m, torch.float64, (T, B, 3))
        self._require("freq_hz", freq_hz, torch.float64, (C,))
        n_ant = 0
        if gains is not None:
            self._require("gains", gains, torch.complex64)
            if gains.dim() != 3 or tuple(gains.shape[:2]) != (C, P):
                raise ValueError(f"gains must be [C][P][n_ant] = [{C}][{P}][n_ant], got {tuple(gains.shape)}")
            n_ant = int(gains.shape[2])
        dev = vis.device
        if out is None:
            out = torch.empty((T, C, P, N, N), dtype=torch.float32, device=dev)
        self._require("out", out, torch.float32, (T, C, P, N, N))
        if weight_sum is None:
            weight_sum = torch.empty((T, C, P), dtype=torch.float64, device=dev)
        if n_out is None:
            n_out = torch.empty((T, C), dtype=torch.int32, device=dev)
        ws = self._workspace(image_batch_corrected_workspace_size(T, C, P, B, N, weighting, precision), workspace)
        corr = Corrections(_ptr(gains), n_ant, float(l0), float(m0))
        st = lib().blink_image_batch_corrected(self.handle, _ptr(vis), _ptr(flags), _ptr(uvw_m), _ptr(freq_hz), T, C,
                                               P, B, N, float(pixel_scale), int(weighting), int(precision),
                                               int(bool(shift)), ctypes.byref(corr), _ptr(out), _ptr(weight_sum),
                                               _ptr(n_out), _ptr(ws), ws.numel(), self._stream(stream))
        _check(st, self.handle, "blink_image_batch_corrected")
        return {"images": out, "weight_sum": weight_sum, "n_out": n_out}

    @_on_stream
    def blink_correlate(self, volt, n_int: int, n_favg: int = 1, pol_mode: int = 4, autos: bool = False, out=None,
                        autos_out=None, stream=None):
        """Correlator: volt int8 device tensor [S][F][A][2][2] (re, im). Returns dict(vis complex64
        [T][C][pol_mode][B], autos complex64 [T][C][A][4] or None)."""
        torch = self._torch()
        self._require("volt", volt, torch.int8)
        if volt.dim() != 5 or tuple(volt.shape[3:]) != (2, 2):
            raise ValueError(f"volt must be [S][F][A][2][2], got {tuple(volt.shape)}")
        S, F, A = (int(x) for x in volt.shape[:3])
        T, C, B = S // int(n_int), F // int(n_favg), A * (A - 1) // 2
        dev = volt.device
        if out is None:
            out = torch.empty((T, C, pol_mode, B), dtype=torch.complex64, device=dev)
        self._require("out", out, torch.complex64, (T, C, pol_mode, B))
        if autos and autos_out is None:
            autos_out = torch.empty((T, C, A, 4), dtype=torch.complex64, device=dev)
        if autos_out is not None:
            self._require("autos_out", autos_out, torch.complex64, (T, C, A, 4))
        st = lib().blink_correlate(self.handle, _ptr(volt), S, F, A, int(n_int), int(n_favg), int(pol_mode), _ptr(out),
                                   _ptr(autos_out), self._stream(stream))
        _check(st, self.handle, "blink_correlate")
        return {"vis": out, "autos": autos_out}

    @_on_stream
    def blink_dedisperse(self, images, delays, t_out: int, out=None, workspace=None, stream=None):
        """De-disperse images float32 device [T][C][N][N] with the host delay table delays int32
        [n_dm][C]; returns out float32 [n_dm][t_out][N][N]."""
        import numpy as np
        torch = self._torch()
        self._require("images", images, torch.float32)
        if images.dim() != 4 or images.shape[2] != images.shape[3]:
            raise ValueError(f"images must be [T][C][N][N], got {tuple(images.shape)}")
        T, C, N = int(images.shape[0]), int(images.shape[1]), int(images.shape[2])
        dl = np.ascontiguousarray(delays, dtype=np.int32)
        if dl.ndim != 2 or dl.shape[1] != C:
            raise ValueError(f"delays must be [n_dm][{C}], got {dl.shape}")
        n_dm = dl.shape[0]
        if out is None:
            out = torch.empty((n_dm, int(t_out), N, N), dtype=torch.float32, device=images.device)
        self._require("out", out, torch.float32, (n_dm, int(t_out), N, N))
        ws = self._workspace(dedisperse_workspace_size(C, n_dm), workspace)
        st = lib().blink_dedisperse(self.handle, _ptr(images), T, C, N, dl.ctypes.data_as(ctypes.c_void_p), n_dm,
                                    int(t_out), _ptr(out), _ptr(ws), ws.numel(), self._stream(stream))
        _check(st, self.handle, "blink_dedisperse")
        return out

    @_on_stream
    def blink_image_average(self, images, axes: int, out=None, stream=None):
        """Average float32 images [T][C][P][N][N] over the axes in `axes` (AVG_TIME | AVG_CHANNEL |
        AVG_POL); returns float32 [T'][C'][P'][N][N] (averaged axes have extent 1)."""
        torch = self._torch()
        self._require("images", images, torch.float32)
        T, C, P, N, N2 = images.shape
        if N != N2:
            raise ValueError("images must be square")
        shape = (1 if axes & AVG_TIME else T, 1 if axes & AVG_CHANNEL else C, 1 if axes & AVG_POL else P, N, N)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=images.device)
        self._require("out", out, torch.float32, shape)
        st = lib().blink_image_average(self.handle, _ptr(images), T, C, P, N, int(axes), _ptr(out),
                                       self._stream(stream))
        _check(st, self.handle, "blink_image_average")
        return out

    @_on_stream
    def blink_image_batch_conv(self, vis, flags, uvw_m, freq_hz, grid_n: int, pixel_scale: float,
                               kernel_width: int = 8, kernel_beta: float = 18.4, precision: int = PREC_FP32,
                               shift: bool = True, out=None, weight_sum=None, n_out=None, workspace=None,
                               stream=None):
        """Convolutional gridding (exponential-of-semicircle kernel of kernel_width cells) + inverse
        2D FFT + grid correction, natural weighting. Same arguments and outputs as blink_image_batch."""
        torch = self._torch()
        T, C, P, B = vis.shape
        N = int(grid_n)
        self._require("vis", vis, torch.complex64)
        if flags is not None:
            self._require("flags", flags, torch.uint8, (T, C, B))
        self._require("uvw_m", uvw_m, torch.float64, (T, B, 3))
        self._require("freq_hz", freq_hz, torch.float64, (C,))
        dev = vis.device
        if out is None:
            out = torch.empty((T, C, P, N, N), dtype=torch.float32, device=dev)
        self._require("out", out, torch.float32, (T, C, P, N, N))
        if weight_sum is None:
            weight_sum = torch.empty((T, C, P), dtype=torch.float64, device=dev)
        if n_out is None:
            n_out = torch.empty((T, C), dtype=torch.int32, device=dev)
        ws = self._workspace(image_batch_conv_workspace_size(T, C, P, B, N, kernel_width, precision), workspace)
        st = lib().blink_image_batch_conv(self.handle, _ptr(vis), _ptr(flags), _ptr(uvw_m), _ptr(freq_hz), T, C, P,
                                          B, N, float(pixel_scale), int(kernel_width), float(kernel_beta),
                                          int(precision), int(bool(shift)), _ptr(out), _ptr(weight_sum),
                                          _ptr(n_out), _ptr(ws), ws.numel(), self._stream(stream))
        _check(st, self.handle, "blink_image_batch_conv")
        return {"images": out, "weight_sum": weight_sum, "n_out": n_out}


class Graph:
    """A captured hipGraph of one uneven-batch call; launch() replays it on the current stream."""

    def __init__(self, ctx: Context, handle, keep=()):
        self.ctx = ctx
        self.handle = handle
        self._keep = keep          # the captured buffers must outlive the graph

    def launch(self, stream=None):
        _check(lib().blink_graph_launch(self.handle, self.ctx._stream(stream)), self.ctx.handle, "blink_graph_launch")
        if stream is not None and self._keep:
            # the workspace (allocated at capture on another stream) is in use on `stream` now
            self._keep[0].record_stream(stream)

    def close(self):
        if getattr(self, "handle", None):
            lib().blink_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
