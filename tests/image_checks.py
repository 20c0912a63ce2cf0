"""Image comparison measures for the reduced-precision FFT forms (plain numpy, CPU).

* rel_l2            ||a - b|| / ||b||
* peak_error        relative error at the reference image's largest-magnitude pixel
* robust_sigma      1.4826 * median absolute deviation from the median (the normal-noise sigma)
* local_maxima      pixels strictly above a threshold that are >= all eight neighbours
* recovery          the 6-sigma detection check: the local maxima above 6 sigma (sigma from the
                    reference) must be the same pixels in both images
"""
import numpy as np


def rel_l2(a, b):
    kind = np.complex128 if (np.iscomplexobj(a) or np.iscomplexobj(b)) else np.float64
    a = np.asarray(a, kind)
    b = np.asarray(b, kind)
    nb = np.linalg.norm(b)
    if nb == 0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def peak_error(got, ref):
    ref = np.asarray(ref, np.float64)
    i = np.unravel_index(np.argmax(np.abs(ref)), ref.shape)
    return float(abs(float(got[i]) - ref[i]) / abs(ref[i])) if ref[i] != 0 else float(abs(float(got[i])))


def robust_sigma(img):
    x = np.asarray(img, np.float64).ravel()
    return float(1.4826 * np.median(np.abs(x - np.median(x))))


def local_maxima(img, threshold):
    """Set of (y, x) with img > threshold and img >= each of its (up to) eight neighbours."""
    a = np.asarray(img, np.float64)
    p = np.pad(a, 1, mode="constant", constant_values=-np.inf)
    ok = a > threshold
    H, W = a.shape
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy or dx:
                ok &= a >= p[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
    return set(zip(*np.nonzero(ok)))


def recovery(got, ref, nsigma=6.0):
    """(missing, spurious): reference maxima above nsigma*sigma absent from `got`, and maxima of
    `got` above that threshold absent from the reference. sigma is the reference's robust sigma."""
    thr = nsigma * robust_sigma(ref)
    r = local_maxima(ref, thr)
    g = local_maxima(got, thr)
    return r - g, g - r
