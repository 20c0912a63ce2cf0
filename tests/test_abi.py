"""CPU tests of the C ABI: the library loads, exports every declared entry point, and rejects bad
arguments on the host before touching a GPU. No compute call is made here."""
import ctypes
import os

import pytest

import paper_2505_15204_amd as blink
from paper_2505_15204_amd import build as blink_build


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(blink.LIB_PATH):
        blink_build.build()
    return blink.lib()


def test_exports_every_declared_function(L):
    names = blink.header_functions()
    assert {"blink_grid", "blink_ifft2d", "blink_image_batch", "blink_create"} <= set(names)
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/blink.h but not exported"


def test_status_strings(L):
    for st in range(6):
        assert blink.status_string(st)
    assert L.blink_version() >= 100


def test_create_without_gpu_reports_hip_error(L):
    h = ctypes.c_void_p()
    st = L.blink_create(ctypes.byref(h), 0)
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if not has_gpu:
        assert st == blink.BLINK_ERR_HIP and not h.value
    elif st == blink.BLINK_OK:
        L.blink_destroy(h)
    assert L.blink_create(None, 0) == blink.BLINK_ERR_ARG
    assert L.blink_destroy(None) == blink.BLINK_OK
    assert L.blink_last_error(None) == b"no context"


def _image_batch(L, T=1, C=1, P=1, B=10, N=64, dl=1e-3, weighting=0, precision=0, ctx=None, ws=1 << 20):
    dummy = ctypes.c_void_p(0x1000)                    # never dereferenced: validation fails first
    return L.blink_image_batch(ctx, dummy, None, dummy, dummy, T, C, P, B, N, dl, weighting, precision, 1,
                               dummy, None, None, ctypes.c_void_p(0x10000), ws, None)


def test_argument_errors_precede_any_device_work(L):
    E = blink
    assert _image_batch(L, N=100) == E.BLINK_ERR_SIZE        # not a power of two
    assert _image_batch(L, N=4) == E.BLINK_ERR_SIZE          # below 8
    assert _image_batch(L, N=8192) == E.BLINK_ERR_SIZE       # above 4096
    assert _image_batch(L, T=-1) == E.BLINK_ERR_ARG
    assert _image_batch(L, P=0) == E.BLINK_ERR_ARG
    assert _image_batch(L, B=-5) == E.BLINK_ERR_ARG
    assert _image_batch(L, weighting=7) == E.BLINK_ERR_ARG
    assert _image_batch(L, dl=0.0) == E.BLINK_ERR_ARG
    assert _image_batch(L, dl=float("nan")) == E.BLINK_ERR_ARG
    assert _image_batch(L) == E.BLINK_ERR_ARG                # NULL context
    dummy = ctypes.c_void_p(0x1000)
    assert L.blink_ifft2d(None, dummy, None, 1, 24, 0, 1, dummy, dummy, 1 << 20, None) == E.BLINK_ERR_SIZE
    assert L.blink_ifft2d(None, dummy, None, -1, 64, 0, 1, dummy, dummy, 1 << 20, None) == E.BLINK_ERR_ARG
    assert L.blink_ifft2d(None, dummy, None, 1, 64, 9, 1, dummy, dummy, 1 << 20, None) == E.BLINK_ERR_ARG
    assert L.blink_grid(None, dummy, None, dummy, dummy, 1, 1, 1, 10, 48, 1e-3, 0, dummy, None, None, None,
                        None, dummy, 1 << 20, None) == E.BLINK_ERR_SIZE


def test_workspace_sizes(L):
    s1 = blink.image_batch_workspace_size(1, 1, 2, 8128, 1024)
    s2 = blink.image_batch_workspace_size(1, 2, 2, 8128, 1024)
    # one (t,c) pair holds at least its two half-spectrum intermediates (N x N/2 complex64 each)
    assert s1 >= 2 * 1024 * 512 * 8
    assert s2 > s1 and s2 <= 2 * s1 + 4096
    assert blink.image_batch_workspace_size(0, 0, 1, 10, 64) == 0
    assert blink.ifft2d_workspace_size(3, 256) >= 3 * 256 * 128 * 8
    assert blink.grid_workspace_size(2, 3, 100, 64) >= 6 * 2 * 100 * 8
    for fn, args in ((blink.image_batch_workspace_size, (1, 1, 1, 10, 96)),
                     (blink.ifft2d_workspace_size, (1, 96)),
                     (blink.grid_workspace_size, (1, 1, 10, 96))):
        with pytest.raises(blink.BlinkError) as e:
            fn(*args)
        assert e.value.status == blink.BLINK_ERR_SIZE
    with pytest.raises(blink.BlinkError):
        blink.image_batch_workspace_size(1, 1, 1, 10, 64, precision=5)


def test_single_workspace_query_matches_each_entry(L):
    assert blink.workspace_size(blink.ENTRY_GRID, T=2, C=3, B=100, grid_n=64) == blink.grid_workspace_size(2, 3, 100, 64)
    assert blink.workspace_size(blink.ENTRY_IFFT2D, n_img=5, grid_n=256, precision=1) == \
        blink.ifft2d_workspace_size(5, 256, 1)
    for w in (0, 1):
        for prec in (0, 2):
            kw = dict(T=1, C=4, P=2, B=8128, grid_n=1024, weighting=w, precision=prec)
            assert blink.workspace_size(blink.ENTRY_IMAGE_BATCH, **kw) == \
                blink.image_batch_workspace_size(1, 4, 2, 8128, 1024, w, prec)
            assert blink.workspace_size(blink.ENTRY_IMAGE_BATCH_CORRECTED, **kw) == \
                blink.image_batch_corrected_workspace_size(1, 4, 2, 8128, 1024, w, prec)
    assert blink.workspace_size(blink.ENTRY_IMAGE_BATCH_CONV, T=1, C=2, P=2, B=8128, grid_n=1024, kernel_width=8) == \
        blink.image_batch_conv_workspace_size(1, 2, 2, 8128, 1024, 8)
    assert blink.workspace_size(blink.ENTRY_IMAGE_BATCH_DESC, n_img=10, max_baselines=100, grid_n=256,
                                workgroups=4) == blink.desc_workspace_size(10, 100, 256, 4)
    assert blink.workspace_size(blink.ENTRY_DEDISPERSE, C=768, n_dm=4) == blink.dedisperse_workspace_size(768, 4)
    with pytest.raises(blink.BlinkError) as ei:
        blink.workspace_size(99, T=1)
    assert ei.value.status == blink.BLINK_ERR_ARG
    with pytest.raises(blink.BlinkError) as ei:
        blink.workspace_size(blink.ENTRY_IMAGE_BATCH, T=1, C=1, P=1, B=10, grid_n=96)
    assert ei.value.status == blink.BLINK_ERR_SIZE


def test_desc_workspace_and_validation(L):
    s = blink.desc_workspace_size(10, 100, 256, 4)
    # enough for the persistent form's 4 slots and for the staged form (every image's placements,
    # and a chunk buffer of at most the batch's half spectra)
    assert s >= 4 * 2 * 100 * 8 + 4 * 256 * 128 * 8
    assert s >= 10 * 2 * 100 * 8 + 10 * 256 * 128 * 8
    assert blink.desc_workspace_size(10, 100, 256, 8) >= s
    assert blink.desc_workspace_size(10, 100, 256, 64) == blink.desc_workspace_size(10, 100, 256, 10)
    # many workgroups: the persistent slots (256 KiB each) outgrow the staged form's 256 MiB buffer
    assert blink.desc_workspace_size(2000, 100, 256, 2000) > blink.desc_workspace_size(2000, 100, 256, 1500)
    with pytest.raises(blink.BlinkError):
        blink.desc_workspace_size(10, 100, 300, 4)
    dummy = ctypes.c_void_p(0x1000)
    # bad max_grid_n, negative n_img, unknown weighting, NULL context: rejected before any device work
    args = lambda n_img=1, max_n=256, w=0, prec=0: [None, dummy, n_img, dummy, 10, dummy, 10, None, 0, 10, max_n, w,
                                                  prec, 1, dummy, 1 << 20, None, None, None, ctypes.c_void_p(0x10000),
                                                  1 << 24, None]
    assert L.blink_image_batch_desc(*args(max_n=300)) == blink.BLINK_ERR_SIZE
    assert L.blink_image_batch_desc(*args(n_img=-1)) == blink.BLINK_ERR_ARG
    assert L.blink_image_batch_desc(*args(w=3)) == blink.BLINK_ERR_ARG
    assert L.blink_image_batch_desc(*args(prec=4)) == blink.BLINK_ERR_ARG
    assert L.blink_image_batch_desc(*args()) == blink.BLINK_ERR_ARG
    assert L.blink_set_desc_plan(None, 512, 0) == blink.BLINK_ERR_ARG
    assert L.blink_set_desc_form(None, blink.DESC_STAGED) == blink.BLINK_ERR_ARG
    assert L.blink_get_desc_form(None, None) == blink.BLINK_ERR_ARG
    assert L.blink_graph_launch(None, None) == blink.BLINK_ERR_ARG
    assert L.blink_graph_destroy(None) == blink.BLINK_OK


def test_conv_argument_checks(L):
    dummy = ctypes.c_void_p(0x1000)

    def call(N=64, width=8, beta=18.4, prec=0, T=1, ctx=None):
        return L.blink_image_batch_conv(ctx, dummy, None, dummy, dummy, T, 1, 1, 10, N, 1e-3, width, beta, prec, 1,
                                        dummy, None, None, ctypes.c_void_p(0x10000), 1 << 20, None)
    assert call(N=100) == blink.BLINK_ERR_SIZE
    assert call(T=-1) == blink.BLINK_ERR_ARG
    assert call() == blink.BLINK_ERR_ARG                      # NULL context
    s = blink.image_batch_conv_workspace_size(1, 2, 2, 8128, 1024, 8)
    assert s > blink.image_batch_workspace_size(1, 2, 2, 8128, 1024)
    for bad in ((1, 1, 1, 10, 64, 0), (1, 1, 1, 10, 64, 32), (1, 1, 1, 10, 64, 17), (1, 1, 1, 10, 16, 8)):
        with pytest.raises(blink.BlinkError):
            blink.image_batch_conv_workspace_size(*bad)


def test_corrections_argument_checks(L):
    """blink_image_batch_corrected: the blink_corrections layout, and its argument errors on the
    host (phase centre off the unit disc, antennas that do not give B) before any device work."""
    assert ctypes.sizeof(blink.Corrections) == 32 and blink.Corrections.l0.offset == 16
    dummy = ctypes.c_void_p(0x1000)

    def call(corr, B=21, N=64, T=1, ctx=None):
        return L.blink_image_batch_corrected(ctx, dummy, None, dummy, dummy, T, 1, 1, B, N, 1e-3, 0, 0, 1,
                                             ctypes.byref(corr) if corr is not None else None, dummy, None, None,
                                             ctypes.c_void_p(0x10000), 1 << 20, None)
    ok = blink.Corrections(None, 0, 0.01, -0.02)
    assert call(ok) == blink.BLINK_ERR_ARG                    # NULL context
    assert call(None) == blink.BLINK_ERR_ARG                  # NULL context, no corrections
    assert call(ok, N=100) == blink.BLINK_ERR_SIZE
    assert call(blink.Corrections(None, 0, 0.8, 0.7)) == blink.BLINK_ERR_ARG
    assert call(blink.Corrections(None, 0, float("nan"), 0.0)) == blink.BLINK_ERR_ARG
    assert call(blink.Corrections(dummy, 6, 0.0, 0.0)) == blink.BLINK_ERR_ARG     # 6 antennas: 15 baselines
    assert call(blink.Corrections(dummy, 1, 0.0, 0.0), B=0) == blink.BLINK_ERR_ARG
    s = blink.image_batch_corrected_workspace_size(1, 2, 2, 8128, 1024)
    assert s >= blink.image_batch_workspace_size(1, 2, 2, 8128, 1024) + 2 * 2 * 8128 * 8


def test_dispersion_delays_on_the_host(L):
    """blink_dispersion_delays runs on the host and matches the oracle's table; bad arguments fail."""
    import numpy as np

    import oracle
    f = 139.0e6 + 40.0e3 * (np.arange(768) + 0.5)
    dms = [0.0, 2.97, 100.0, 600.0]
    assert np.array_equal(blink.dispersion_delays(f, 0.02, dms), oracle.dispersion_delays(f, 0.02, dms))
    for bad in ((f, 0.0, dms), (f, 0.02, [-1.0]), (-f, 0.02, dms)):
        with pytest.raises(blink.BlinkError):
            blink.dispersion_delays(*bad)
    assert blink.dedisperse_workspace_size(768, 4) >= 768 * 4 * 4
    dummy = ctypes.c_void_p(0x1000)
    d = np.zeros((1, 4), dtype=np.int32)
    assert L.blink_dedisperse(None, dummy, 4, 4, 64, d.ctypes.data_as(ctypes.c_void_p), 1, 2, dummy, dummy, 1 << 20,
                              None) == blink.BLINK_ERR_ARG
