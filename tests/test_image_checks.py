"""CPU tests of the image comparison measures used for the reduced-precision forms."""
import numpy as np

from image_checks import local_maxima, peak_error, recovery, rel_l2, robust_sigma


def blobs(shape=(64, 64), centres=((10, 12), (40, 50), (30, 20)), amp=(9.0, 7.0, 8.0), seed=0):
    y, x = np.mgrid[:shape[0], :shape[1]]
    img = np.random.default_rng(seed).normal(0.0, 1.0, shape)
    for (cy, cx), a in zip(centres, amp):
        img += a * np.exp(-((y - cy) ** 2 + (x - cx) ** 2) / 4.0) * 2.0
    return img


def test_robust_sigma_of_normal_noise():
    x = np.random.default_rng(1).normal(0.0, 3.0, 200000)
    assert abs(robust_sigma(x) - 3.0) < 0.03
    assert robust_sigma(np.ones(10)) == 0.0


def test_local_maxima_finds_blobs_and_edges():
    img = np.zeros((8, 8))
    img[0, 0] = 5.0          # corner maximum (neighbours outside the image do not count)
    img[4, 4] = 3.0
    img[4, 5] = 3.0          # a two-pixel plateau: both are >= their neighbours
    img[6, 1] = 0.5          # below the threshold
    assert local_maxima(img, 1.0) == {(0, 0), (4, 4), (4, 5)}
    assert local_maxima(-img, 1.0) == set()


def test_recovery_detects_missing_and_spurious_sources():
    ref = blobs()
    thr_pixels = local_maxima(ref, 6 * robust_sigma(ref))
    assert {(10, 12), (40, 50), (30, 20)} <= thr_pixels
    assert recovery(ref + 1e-9, ref) == (set(), set())
    lost = ref.copy()
    lost[35:46, 45:56] = 0.0                     # a source vanishes
    missing, spurious = recovery(lost, ref)
    assert (40, 50) in missing and not spurious
    extra = ref.copy()
    extra[55, 5] = 50.0                          # a source appears
    missing, spurious = recovery(extra, ref)
    assert (55, 5) in spurious and not missing


def test_rel_l2_and_peak_error():
    ref = blobs()
    got = ref * (1 + 1e-4)
    assert abs(rel_l2(got, ref) - 1e-4) < 1e-9
    assert abs(peak_error(got, ref) - 1e-4) < 1e-9
    assert rel_l2(np.zeros(3), np.zeros(3)) == 0.0
