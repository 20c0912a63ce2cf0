"""Pins of the FP64 oracle against facts fixed by the paper and by the mathematics.

Every pin takes an ``oracle.Oracle`` (so the same checks can be run against a copy of
the oracle built with a planted mistake) and raises AssertionError on failure.
None of them re-types the oracle's arithmetic: they compare it with hand-worked golden
values, brute-force definitions evaluated a different way (direct sums instead of FFTs,
sums over baselines instead of over cells), an independent library FFT, closed forms
and invariants.
"""
from __future__ import annotations

import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
C_LIGHT = 299792458.0


# ----------------------------------------------------------------------------- fixtures

def read_cell_fixture():
    rows = []
    with open(os.path.join(GOLDEN, "cell_index_worked.txt")) as fh:
        for ln in fh:
            ln = ln.strip()
            if not ln or ln.startswith("#"):
                continue
            f, n, dl, u, v, iu, iv, cell = ln.split()
            rows.append((float(f), int(n), float(dl), float(u), float(v), int(iu), int(iv),
                         int(cell)))
    return rows


def read_tiny_fixture():
    sections = {}
    cur = None
    with open(os.path.join(GOLDEN, "tiny_grid_n8.txt")) as fh:
        for ln in fh:
            ln = ln.strip()
            if not ln or ln.startswith("#"):
                continue
            if ln.startswith("["):
                cur = ln.strip("[]")
                sections[cur] = []
                continue
            if cur is not None:
                sections[cur].append(ln.split())
    return sections


def small_problem(seed, B=300, N=64, P=1, flag_frac=0.1, extent=0.45, n_src=4):
    """Random baselines inside the grid (mostly), point-source visibilities plus noise."""
    g = np.random.default_rng(seed)
    f = 150.0e6
    dl = 1.0 / 300.0
    k = (f / C_LIGHT) * (N * dl)
    rmax = extent * N / k                           # metres reaching `extent` of the grid
    uvw = np.zeros((B, 3))
    uvw[:, :2] = g.uniform(-rmax, rmax, size=(B, 2))
    src = [(g.uniform(1, 5), g.uniform(-0.05, 0.05), g.uniform(-0.05, 0.05)) for _ in range(n_src)]
    vis = np.zeros((P, B), np.complex128)
    for s, l, m in src:
        vis += s * np.exp(-2j * np.pi * (uvw[:, 0] * l + uvw[:, 1] * m) * f / C_LIGHT)
    vis += g.normal(0, 0.3, (P, B)) + 1j * g.normal(0, 0.3, (P, B))
    flags = (g.random(B) < flag_frac).astype(np.uint8)
    return vis.astype(np.complex64), flags, uvw, f, N, dl


def direct_image_from_grid(G, W, shift):
    """Brute-force definition: I[y][x] = Re(sum_{kv,ku} G[kv][ku] e^{+2 pi i (ku X + kv Y)/N})/W."""
    N = G.shape[0]
    pos = np.arange(N) - (N // 2 if shift else 0)
    ang = 2.0 * np.pi * np.outer(np.arange(N), pos) / N            # [k][pixel]
    E = np.exp(1j * ang)
    full = E.T @ G @ E                                              # [y][x]
    return full.real / W, np.abs(full.imag).max() / W


def snapped_sum_image(vis, flags, uvw, f, N, dl, shift=True):
    """Whole path as a sum over baselines at their snapped cells (natural weighting):
    I = (1/W) sum_b 2 Re(V_b exp(+2 pi i (iu X + iv Y)/N))."""
    k = (f / C_LIGHT) * (N * dl)
    ru = np.rint(uvw[:, 0] * k)
    rv = np.rint(uvw[:, 1] * k)
    keep = (flags == 0) & (np.abs(ru) < N // 2) & (np.abs(rv) < N // 2)
    W = 2.0 * keep.sum()
    pos = np.arange(N) - (N // 2 if shift else 0)
    Ex = np.exp(2j * np.pi * np.outer(ru[keep], pos) / N)          # [b][x]
    Ey = np.exp(2j * np.pi * np.outer(rv[keep], pos) / N)          # [b][y]
    v = vis[keep].astype(np.complex128)
    img = 2.0 * np.real(np.einsum("b,by,bx->yx", v, Ey, Ex)) / W
    return img, keep, W


def ungridded_image(vis, keep, uvw, f, N, dl, W):
    """Direct transform of the unsnapped visibilities at every pixel."""
    k = (f / C_LIGHT) * (N * dl)
    pos = np.arange(N) - N // 2
    xu = uvw[keep, 0] * k
    xv = uvw[keep, 1] * k
    Ex = np.exp(2j * np.pi * np.outer(xu, pos) / N)
    Ey = np.exp(2j * np.pi * np.outer(xv, pos) / N)
    v = vis[keep].astype(np.complex128)
    return 2.0 * np.real(np.einsum("b,by,bx->yx", v, Ey, Ex)) / W


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ----------------------------------------------------------------------------- pins

def pin_cell_worked(O):
    """Hand-worked k and cell indices, including ties (round half to even) and the strict edge."""
    rows = read_cell_fixture()
    kA = O.cells_per_metre(150.0e6, 256, math.pi / 10800.0)
    assert abs(kA - 0.03725946705691879) <= 1e-17, kA
    assert O.cells_per_metre(C_LIGHT, 8, 1.0 / 64.0) == 0.125
    for f, n, dl, u, v, iu, iv, cell in rows:
        out = O.grid(np.array([[1 + 0j]], np.complex64), None, np.array([[u, v, 0.0]]), f, n, dl)
        assert int(out["cell_idx"][0]) == cell, (f, n, u, v, cell, out["cell_idx"][0])
        assert out["n_out"] == (1 if cell == -2 else 0)


def pin_tiny_grid(O):
    """Hand-enumerated 7-baseline grid, counts, weights and closed-form image pixels."""
    fx = read_tiny_fixture()
    bl = np.array([[float(x) for x in r] for r in fx["baselines"]])
    uvw = np.zeros((bl.shape[0], 3))
    uvw[:, :2] = bl[:, 0:2]
    flags = bl[:, 2].astype(np.uint8)
    vis = (bl[:, 3] + 1j * bl[:, 4]).astype(np.complex64)
    expect_cells = [int(x) for x in fx["cell_idx"][0]]
    weights = {r[0]: float(r[1]) for r in fx["weights"]}
    for wname, wcode in (("natural", 0), ("uniform", 1)):
        out = O.grid(vis, flags, uvw, C_LIGHT, 8, 1.0 / 64.0, weighting=wcode)
        assert list(out["cell_idx"]) == expect_cells, out["cell_idx"]
        assert out["n_out"] == int(weights["n_out"])
        assert out["weight_sum"] == weights[wname], out["weight_sum"]
        g = out["grid"][0].reshape(-1)
        expect = np.zeros(64, np.complex128)
        counts = np.zeros(64, np.int32)
        for cell, re, im, cnt in fx[f"{wname}_grid"]:
            expect[int(cell)] = float(re) + 1j * float(im)
            counts[int(cell)] = int(cnt)
        assert np.array_equal(g, expect), (wname, g)
        assert np.array_equal(out["counts"].reshape(-1), counts)
        img, _ = O.ifft2d(out["grid"][0], out["weight_sum"], shift=True)
        for w, x, y, val in fx["pixels"]:
            if w == wname:
                assert abs(img[int(y), int(x)] - float(val)) < 1e-14, (w, x, y, img[int(y), int(x)])
        # unshifted: the phase-centre value sits at the corner
        img0, _ = O.ifft2d(out["grid"][0], out["weight_sum"], shift=False)
        assert abs(img0[0, 0] - img[4, 4]) < 1e-14


def pin_ifft1d_bruteforce(O):
    """Radix-2 FFT against the O(n^2) definition and against numpy's FFT."""
    g = np.random.default_rng(1)
    for n in (1, 2, 4, 8, 16, 32, 64, 256):
        x = g.normal(size=n) + 1j * g.normal(size=n)
        y = O.ifft1d(x)
        j = np.arange(n)
        direct = np.exp(2j * np.pi * np.outer(j, j) / n) @ x
        assert np.abs(y - direct).max() <= 1e-12 * max(1.0, np.abs(direct).max()), n
        assert np.abs(y - np.fft.ifft(x) * n).max() <= 1e-12 * max(1.0, np.abs(direct).max()), n


def pin_ifft2d_bruteforce(O):
    """2D image of a random (non-Hermitian) grid against the direct O(N^4) definition."""
    g = np.random.default_rng(2)
    for N in (2, 4, 8, 16):
        G = g.normal(size=(N, N)) + 1j * g.normal(size=(N, N))
        for shift in (True, False):
            img, im = O.ifft2d(G, 3.5, shift=shift)
            ref, ref_im = direct_image_from_grid(G, 3.5, shift)
            assert np.abs(img - ref).max() <= 1e-12 * np.abs(ref).max(), (N, shift)
            assert abs(im - ref_im) <= 1e-12 * ref_im, (N, shift)


def pin_ifft2d_library(O):
    """2D image against numpy.fft.ifft2 (+ sign, 1/N^2) followed by fftshift."""
    g = np.random.default_rng(3)
    for N in (32, 128):
        G = g.normal(size=(N, N)) + 1j * g.normal(size=(N, N))
        img, _ = O.ifft2d(G, 2.0, shift=True)
        ref = np.fft.fftshift(np.fft.ifft2(G) * N * N).real / 2.0
        assert np.abs(img - ref).max() <= 1e-11 * np.abs(ref).max(), N
        img0, _ = O.ifft2d(G, 2.0, shift=False)
        ref0 = (np.fft.ifft2(G) * N * N).real / 2.0
        assert np.abs(img0 - ref0).max() <= 1e-11 * np.abs(ref0).max(), N


def pin_closed_forms(O):
    """Flat grid -> centred delta of height N^2/W; one unit cell -> a cosine plane wave."""
    for N in (8, 64):
        img, _ = O.ifft2d(np.ones((N, N), np.complex128), 4.0, shift=True)
        delta = np.zeros((N, N))
        delta[N // 2, N // 2] = N * N / 4.0
        assert np.abs(img - delta).max() <= 1e-12 * N * N, N
        a, b = 3, N - 2                                     # ku = 3, kv = -2
        G = np.zeros((N, N), np.complex128)
        G[b, a] = 1.0
        img, im = O.ifft2d(G, 1.0, shift=True)
        X = np.arange(N) - N // 2
        ref = np.cos(2 * np.pi * (a * X[None, :] + b * X[:, None]) / N)
        assert np.abs(img - ref).max() <= 1e-12, N
        assert abs(im - 1.0) <= 1e-12                     # |sin| reaches 1 on this grid


def pin_parseval_and_sum(O):
    """Parseval and the sum rule on a Hermitian grid produced by gridding."""
    vis, flags, uvw, f, N, dl = small_problem(4, B=400, N=64)
    out = O.grid(vis, flags, uvw, f, N, dl)
    G, W = out["grid"][0], out["weight_sum"]
    img, _ = O.ifft2d(G, W, shift=True)
    lhs = float((img ** 2).sum())
    rhs = N * N / W ** 2 * float((np.abs(G) ** 2).sum())
    assert abs(lhs - rhs) <= 1e-11 * rhs, (lhs, rhs)
    assert abs(img.sum() - N * N * G[0, 0].real / W) <= 1e-10 * abs(img).sum()


def pin_snapped_dft(O):
    """Grid + FFT + shift + 1/W equals the direct sum over baselines at their snapped cells."""
    for seed, N in ((5, 32), (6, 64)):
        vis, flags, uvw, f, N, dl = small_problem(seed, B=300, N=N, extent=0.6)
        res = O.image_batch(vis[None, None], flags[None, None], uvw[None], np.array([f]), N, dl)
        img = res["images"][0, 0, 0]
        ref, keep, W = snapped_sum_image(vis[0], flags, uvw, f, N, dl)
        assert res["weight_sum"][0, 0, 0] == W
        assert res["n_out"][0, 0] == int(((flags == 0) & ~keep).sum())
        assert np.abs(img - ref).max() <= 1e-12 * np.abs(ref).max(), seed


def pin_ungridded_bound(O):
    """Against the direct transform of the unsnapped visibilities: equal at the phase centre,
    and within (2/W) sum |V| pi (|X|+|Y|)/N everywhere (snapping moves a sample <= half a cell)."""
    vis, flags, uvw, f, N, dl = small_problem(7, B=250, N=64, extent=0.4)
    res = O.image_batch(vis[None, None], flags[None, None], uvw[None], np.array([f]), N, dl)
    img = res["images"][0, 0, 0]
    k = (f / C_LIGHT) * (N * dl)
    keep = (flags == 0) & (np.abs(np.rint(uvw[:, 0] * k)) < N // 2) & (np.abs(np.rint(uvw[:, 1] * k)) < N // 2)
    W = res["weight_sum"][0, 0, 0]
    Id = ungridded_image(vis[0], keep, uvw, f, N, dl, W)
    X = np.abs(np.arange(N) - N // 2)
    bound = (2.0 / W) * np.abs(vis[0][keep]).astype(np.float64).sum() * np.pi * (X[None, :] + X[:, None]) / N
    assert abs(img[N // 2, N // 2] - Id[N // 2, N // 2]) <= 1e-12 * abs(Id[N // 2, N // 2])
    assert np.all(np.abs(img - Id) <= bound + 1e-12)
    # the bound must not be vacuous: snapping error is far below it on average
    assert np.abs(img - Id).max() < 0.5 * bound.max()


def pin_direct_dft(O):
    """The oracle's direct transform (a sum over baselines, no grid, no FFT): at the snapped cells it
    equals the gridded image (grid + FFT + shift + 1/W) to rounding; at the exact positions it equals
    it at the phase centre and stays within the half-cell bound elsewhere; a point source placed on
    a pixel centre images to exactly its flux there when nothing is snapped."""
    for seed, N, shift in ((11, 32, True), (12, 64, True), (13, 32, False)):
        vis, flags, uvw, f, N, dl = small_problem(seed, B=200, N=N, P=2, extent=0.6)
        res = O.image_batch(vis[None, None], flags[None, None], uvw[None], np.array([f]), N, dl, shift=shift)
        d = O.dft(vis, flags, uvw, f, N, dl, snap=True, shift=shift)
        assert d["weight_sum"] == res["weight_sum"][0, 0, 0] and d["n_out"] == res["n_out"][0, 0]
        for p in range(2):
            img = res["images"][0, 0, p]
            assert np.abs(d["images"][p] - img).max() <= 1e-12 * np.abs(img).max(), (seed, p)
    vis, flags, uvw, f, N, dl = small_problem(14, B=250, N=64, extent=0.4)
    img = O.image_batch(vis[None, None], flags[None, None], uvw[None], np.array([f]), N, dl)["images"][0, 0, 0]
    d = O.dft(vis, flags, uvw, f, N, dl, snap=False)
    Id, W = d["images"][0], d["weight_sum"]
    k = (f / C_LIGHT) * (N * dl)
    keep = (flags == 0) & (np.abs(np.rint(uvw[:, 0] * k)) < N // 2) & (np.abs(np.rint(uvw[:, 1] * k)) < N // 2)
    X = np.abs(np.arange(N) - N // 2)
    bound = (2.0 / W) * np.abs(vis[0][keep]).astype(np.float64).sum() * np.pi * (X[None, :] + X[:, None]) / N
    c = N // 2
    assert abs(img[c, c] - Id[c, c]) <= 1e-12 * abs(Id[c, c])
    assert np.all(np.abs(img - Id) <= bound + 1e-12)
    assert np.abs(img - Id).max() > 1e-6          # snapping is visible away from the centre
    # a 3 Jy source at (l, m) = (5 dl, -3 dl), unsnapped: exactly 3 at pixel (N/2 + 5, N/2 - 3)
    l0, m0, S = 5 * dl, -3 * dl, 3.0
    src = (S * np.exp(-2j * np.pi * (uvw[:, 0] * l0 + uvw[:, 1] * m0) * f / C_LIGHT)).astype(np.complex64)
    src64 = S * np.exp(-2j * np.pi * (uvw[:, 0] * l0 + uvw[:, 1] * m0) * f / C_LIGHT)
    d = O.dft(src, flags, uvw, f, N, dl, snap=False)["images"][0]
    err = (2.0 / W) * np.abs(src.astype(np.complex128) - src64)[keep].sum()   # complex64 rounding of V
    assert abs(d[c - 3, c + 5] - S) <= err + 1e-12
    assert np.unravel_index(np.argmax(d), d.shape) == (c - 3, c + 5)


def pin_point_source_centre(O):
    """V = 1 (a unit source at the phase centre): the dirty beam, 1 at the centre, <= 1, even."""
    vis, flags, uvw, f, N, dl = small_problem(8, B=300, N=64)
    ones = np.ones_like(vis)
    for weighting in (0, 1):
        res = O.image_batch(ones[None, None], flags[None, None], uvw[None], np.array([f]), N, dl,
                            weighting=weighting)
        img = res["images"][0, 0, 0]
        c = N // 2
        assert abs(img[c, c] - 1.0) <= 1e-12
        assert np.abs(img).max() <= 1.0 + 1e-12
        inner = img[1:, 1:]                                   # X, Y in [-N/2+1, N/2-1]
        assert np.abs(inner - inner[::-1, ::-1]).max() <= 1e-12


def pin_shift_theorem(O):
    """A point source at (l, m) = (p dl, q dl) through Eq. 4 images as the dirty beam rolled by
    (+p, +q): +l is +x (column), +m is +y (row), and the transform sign is the inverse one."""
    N, f, dl = 32, C_LIGHT, 1.0 / 256.0                    # k = 0.125: 8 m per cell
    g = np.random.default_rng(9)
    cells = g.integers(-12, 13, size=(120, 2))
    uvw = np.zeros((120, 3))
    uvw[:, :2] = cells * 8.0
    flags = np.zeros(120, np.uint8)
    beam = O.image_batch(np.ones((1, 1, 1, 120), np.complex64), flags[None, None], uvw[None],
                         np.array([f]), N, dl)["images"][0, 0, 0]
    for p, q in ((3, 0), (0, 5), (-4, 2)):
        l, m = p * dl, q * dl
        vis = np.exp(-2j * np.pi * (uvw[:, 0] * l + uvw[:, 1] * m) * f / C_LIGHT)
        img = O.image_batch(vis.astype(np.complex64)[None, None, None], flags[None, None], uvw[None],
                            np.array([f]), N, dl)["images"][0, 0, 0]
        rolled = np.roll(np.roll(beam, q, axis=0), p, axis=1)
        assert np.abs(img - rolled).max() <= 2e-7, (p, q)       # complex64 rounding of V
        y, x = np.unravel_index(np.argmax(img), img.shape)
        assert (x, y) == (N // 2 + p, N // 2 + q), (p, q, x, y)


def pin_realness(O):
    """The Hermitian-completed grid transforms to a real image (imaginary part at rounding level)."""
    vis, flags, uvw, f, N, dl = small_problem(10, B=400, N=128)
    out = O.grid(vis, flags, uvw, f, N, dl)
    img, im = O.ifft2d(out["grid"][0], out["weight_sum"], shift=True)
    assert im <= 1e-12 * np.abs(img).max(), im


def pin_invariants(O):
    """Count, weight and symmetry invariants of gridding (natural and uniform)."""
    vis, flags, uvw, f, N, dl = small_problem(11, B=500, N=32, extent=0.7, P=2)
    nat = O.grid(vis, flags, uvw, f, N, dl, weighting=0)
    uni = O.grid(vis, flags, uvw, f, N, dl, weighting=1)
    cell = nat["cell_idx"]
    kept = int((cell >= 0).sum())
    assert np.array_equal(cell == -1, flags == 1)
    assert nat["n_out"] == int((cell == -2).sum()) and nat["n_out"] > 0
    cnt = nat["counts"]
    assert int(cnt.sum()) == 2 * kept
    mirror = np.roll(np.roll(cnt[::-1, ::-1], 1, axis=0), 1, axis=1)   # counts[-kv][-ku]
    assert np.array_equal(cnt, mirror)
    assert nat["weight_sum"] == 2 * kept
    assert uni["weight_sum"] == int((cnt > 0).sum())
    assert np.array_equal(uni["counts"], cnt) and np.array_equal(uni["cell_idx"], cell)
    vmax = np.abs(vis.astype(np.complex128)).max()
    assert np.abs(uni["grid"]).max() <= vmax * (1 + 1e-12)
    occupied = cnt > 0
    assert np.all(uni["grid"][:, ~occupied] == 0) and np.all(nat["grid"][:, ~occupied] == 0)
    # the natural cell sum is the uniform cell mean times the count
    assert np.allclose(nat["grid"], uni["grid"] * cnt[None], rtol=1e-12, atol=1e-12)
    # Hermitian grid
    G = nat["grid"][0]
    Gm = np.conj(np.roll(np.roll(G[::-1, ::-1], 1, axis=0), 1, axis=1))
    assert np.abs(G - Gm).max() <= 1e-12 * np.abs(G).max()


def pin_degenerate(O):
    """All flagged, or all outside the grid: W = 0 and an all-zero image; empty baseline list."""
    vis, flags, uvw, f, N, dl = small_problem(12, B=50, N=16)
    allf = np.ones_like(flags)
    res = O.image_batch(vis[None, None], allf[None, None], uvw[None], np.array([f]), N, dl)
    assert res["weight_sum"][0, 0, 0] == 0 and not res["images"].any()
    assert np.all(res["cell_idx"] == -1) and res["n_out"][0, 0] == 0
    far = uvw * 1000.0
    res = O.image_batch(vis[None, None], None, far[None], np.array([f]), N, dl)
    assert res["weight_sum"][0, 0, 0] == 0 and not res["images"].any()
    assert res["n_out"][0, 0] == 50
    res = O.image_batch(np.zeros((1, 1, 1, 0), np.complex64), None, np.zeros((1, 0, 3)),
                        np.array([f]), N, dl)
    assert res["weight_sum"][0, 0, 0] == 0 and not res["images"].any()


def pin_pols_share_flags(O):
    """Polarisations are independent images that share cells and flags."""
    vis, flags, uvw, f, N, dl = small_problem(13, B=200, N=32, P=2)
    both = O.image_batch(vis[None, None], flags[None, None], uvw[None], np.array([f]), N, dl)
    for p in range(2):
        one = O.image_batch(vis[None, None, p:p + 1], flags[None, None], uvw[None], np.array([f]), N, dl)
        assert np.array_equal(both["images"][0, 0, p], one["images"][0, 0, 0])
    assert not np.allclose(both["images"][0, 0, 0], both["images"][0, 0, 1])


# ----------------------------------------------------------------------------- convolutional gridding pins

def pin_es_kernel_values(O):
    """Worked values of phi(z) = exp(beta (sqrt(1 - z^2) - 1)): sqrt(1 - 0.36) = 0.8 exactly."""
    assert O.es_kernel(0.0, 7.0) == 1.0
    assert abs(O.es_kernel(0.6, 2.0) - math.exp(-0.4)) <= 1e-15
    assert abs(O.es_kernel(-0.6, 2.0) - math.exp(-0.4)) <= 1e-15
    assert O.es_kernel(1.0, 3.0) == 0.0 and O.es_kernel(-1.5, 3.0) == 0.0
    assert O.es_kernel(0.3, 0.0) == 1.0


def pin_es_transform(O):
    """c(nu) against the closed form for beta = 0 (sin(pi W nu)/(pi nu), W at nu = 0) and against
    SciPy's adaptive quadrature of the untransformed integral for beta > 0."""
    from scipy import integrate
    for W in (1, 4, 8):
        assert abs(O.es_transform(0.0, W, 0.0) - W) <= 1e-12 * W
        for nu in (0.05, 0.21, 0.5):
            ref = math.sin(math.pi * W * nu) / (math.pi * nu)
            assert abs(O.es_transform(nu, W, 0.0) - ref) <= 1e-11 * W, (W, nu)
    for W, beta in ((6, 13.8), (8, 18.4), (4, 5.0)):
        for nu in (0.0, 0.125, 0.3, 0.49):
            f = lambda d: math.exp(beta * (math.sqrt(max(0.0, 1.0 - (2 * d / W) ** 2)) - 1.0)) * math.cos(2 * math.pi * nu * d)
            ref = 2.0 * integrate.quad(f, 0.0, W / 2.0, epsabs=1e-14, epsrel=1e-13, limit=400)[0]
            assert abs(O.es_transform(nu, W, beta) - ref) <= 1e-9 * abs(ref) + 1e-13, (W, beta, nu)


def pin_conv_width1_is_nearest_cell(O):
    """With W = 1 and beta = 0 the kernel covers exactly the nearest cell with weight 1, so the
    convolutional grid is the (independently pinned) nearest-cell natural grid."""
    vis, flags, uvw, f, N, dl = small_problem(31, B=400, N=32, P=2, extent=0.6)
    k = (f / C_LIGHT) * (N * dl)
    frac = np.abs(np.abs(uvw[:, :2] * k) % 1.0 - 0.5)
    assert frac.min() > 1e-6                        # no half-integer ties in this draw
    a = O.grid(vis, flags, uvw, f, N, dl, 0)
    b = O.grid_conv(vis, flags, uvw, f, N, dl, 1, 0.0)
    assert a["weight_sum"] == b["weight_sum"] and a["n_out"] == b["n_out"] and a["n_out"] > 0
    assert np.abs(a["grid"] - b["grid"]).max() <= 1e-12


def pin_conv_hermitian(O):
    vis, flags, uvw, f, N, dl = small_problem(32, B=200, N=32, P=1, extent=0.5)
    G = O.grid_conv(vis, flags, uvw, f, N, dl, 6, 13.8)["grid"][0]
    idx = (-np.arange(N)) % N
    M = np.conj(G[np.ix_(idx, idx)])
    assert np.abs(G - M).max() <= 1e-12 * np.abs(G).max()


def pin_conv_matches_direct_transform(O):
    """Gridding with the kernel and dividing by its transform reproduces the direct transform of the
    unsnapped visibilities in the central half of the image (aliasing suppressed), where
    nearest-cell gridding is off by about 10 percent. Pins positions, mirror, normalisation and
    the correction's axis and sign."""
    vis, flags, uvw, f, N, dl = small_problem(33, B=250, N=64, P=1, extent=0.42, n_src=3)
    vis = vis[0]
    out = O.image_batch_conv(vis[None, None, None, :], flags[None, None, :], uvw[None], np.array([f]), N, dl, 8, 18.4)
    img = out["images"][0, 0, 0]
    k = (f / C_LIGHT) * (N * dl)
    keep = (flags == 0) & (np.abs(np.rint(uvw[:, 0] * k)) < N // 2) & (np.abs(np.rint(uvw[:, 1] * k)) < N // 2)
    W = 2.0 * keep.sum()
    assert out["weight_sum"][0, 0, 0] == W
    ref = ungridded_image(vis, keep, uvw, f, N, dl, W)
    c = slice(N // 4, 3 * N // 4)
    scale = np.abs(ref).max()
    assert np.abs(img - ref)[c, c].max() <= 1e-6 * scale
    near = O.image_batch(vis[None, None, None, :], flags[None, None, :], uvw[None], np.array([f]), N, dl, 0)
    assert np.abs(near["images"][0, 0, 0] - ref)[c, c].max() > 1e-2 * scale


def pin_conv_batch_consistency(O):
    """The batch driver is gridding, the inverse transform, then division by c(X/N) c(Y/N)."""
    vis, flags, uvw, f, N, dl = small_problem(34, B=150, N=32, P=2, extent=0.5)
    for shift in (True, False):
        out = O.image_batch_conv(vis[None, None], flags[None, None], uvw[None], np.array([f]), N, dl, 4, 9.2,
                                 shift=shift)
        g = O.grid_conv(vis, flags, uvw, f, N, dl, 4, 9.2)
        corr = O.conv_correction(N, 4, 9.2, shift)
        X = np.arange(N) - N // 2 if shift else np.where(np.arange(N) < N // 2, np.arange(N), np.arange(N) - N)
        assert np.abs(corr - np.array([O.es_transform(x / N, 4, 9.2) for x in X])).max() <= 1e-15 * 4
        for p in range(2):
            base, _ = O.ifft2d(g["grid"][p], g["weight_sum"], shift)
            want = base / np.outer(corr, corr)
            assert np.abs(out["images"][0, 0, p] - want).max() <= 1e-12 * np.abs(want).max()


def pin_image_average(O):
    """Averages against numpy's mean over the same axes; Stokes I of identical pols is that pol."""
    g = np.random.default_rng(35)
    imgs = g.normal(size=(3, 4, 2, 8, 8)).astype(np.float32)
    for axes in range(8):
        ax = tuple(i for i, bit in enumerate((1, 2, 4)) if axes & bit)
        ref = imgs.astype(np.float64).mean(axis=ax, keepdims=True) if ax else imgs.astype(np.float64)
        got = O.image_average(imgs, axes)
        assert got.shape == ref.shape and np.abs(got - ref).max() <= 1e-12, axes
    same = np.repeat(imgs[:, :, :1], 2, axis=2)
    assert np.array_equal(O.image_average(same, 4)[:, :, 0], imgs[:, :, 0].astype(np.float64))


# ----------------------------------------------------------------------------- corrections

def correction_problem(seed, n_ant=7, T=2, C=3, P=2):
    """Random visibilities and non-coplanar baselines (w != 0) of n_ant antennas."""
    g = np.random.default_rng(seed)
    B = n_ant * (n_ant - 1) // 2
    pos = g.uniform(-400.0, 400.0, size=(n_ant, 3))
    pos[:, 2] = g.uniform(-40.0, 40.0, size=n_ant)
    rows, cols = np.tril_indices(n_ant, k=-1)          # (1,0), (2,0), (2,1), ...: b = i(i-1)/2 + j
    uvw = np.repeat((pos[rows] - pos[cols])[None], T, axis=0)
    uvw[1:] += g.normal(scale=0.5, size=uvw[1:].shape)  # the baselines move a little in time
    freq = 150.0e6 + 1.28e6 * np.arange(C)
    vis = (g.normal(size=(T, C, P, B)) + 1j * g.normal(size=(T, C, P, B))).astype(np.complex64)
    return vis, uvw, freq, rows, cols


def pin_corrections_identity(O):
    """Unit gains and no phase-centre offset leave the visibilities, and the images, unchanged."""
    vis, uvw, freq, _, _ = correction_problem(40)
    T, C, P, B = vis.shape
    ones = np.ones((C, P, 7), dtype=np.complex64)
    for gains in (None, ones):
        vc = O.correct_vis(vis, uvw, freq, gains, 0.0, 0.0)
        assert np.array_equal(vc, vis.astype(np.complex128))
    a = O.image_batch(vis, None, uvw, freq, 32, 2.0e-3, 0)
    b = O.image_batch_corrected(vis, None, uvw, freq, 32, 2.0e-3, 0, ones, 0.0, 0.0)
    assert np.array_equal(a["images"], b["images"]) and np.array_equal(a["weight_sum"], b["weight_sum"])


def pin_corrections_undo_gains(O):
    """Visibilities corrupted by per-antenna gains, built as diag(g) M diag(g)^H on the full
    correlation matrix M, are restored by the solutions 1/g."""
    vis, uvw, freq, rows, cols = correction_problem(41)
    T, C, P, B = vis.shape
    A = 7
    g = np.random.default_rng(42)
    gains = (g.uniform(0.5, 1.5, size=(C, P, A)) * np.exp(2j * np.pi * g.uniform(size=(C, P, A))))
    obs = np.empty((T, C, P, B), dtype=np.complex128)
    for t, c, p in np.ndindex(T, C, P):
        M = np.zeros((A, A), dtype=np.complex128)
        M[rows, cols] = vis[t, c, p]
        M[cols, rows] = np.conj(vis[t, c, p])
        D = np.diag(gains[c, p])
        obs[t, c, p] = (D @ M @ D.conj().T)[rows, cols]
    sol = (1.0 / gains).astype(np.complex64)
    back = O.correct_vis(obs.astype(np.complex64), uvw, freq, sol, 0.0, 0.0)
    assert np.abs(back - vis).max() <= 1e-5 * np.abs(vis).max()


def pin_corrections_phase_centre(O):
    """A point source at (l0, m0), with the w term of Eq. 4 (non-coplanar baselines), has the
    same visibility S on every baseline after the phase centre moves to (l0, m0), so the
    naturally weighted image has S at the centre pixel."""
    vis, uvw, freq, _, _ = correction_problem(43, P=1)
    T, C, P, B = vis.shape
    l0, m0, S = 0.031, -0.047, 2.5
    n0 = math.sqrt(1.0 - l0 * l0 - m0 * m0)
    src = np.empty((T, C, 1, B), dtype=np.complex128)
    for c in range(C):
        lam = C_LIGHT / freq[c]
        src[:, c, 0] = S * np.exp(-2j * np.pi * (uvw[..., 0] * l0 + uvw[..., 1] * m0 + uvw[..., 2] * (n0 - 1.0)) / lam)
    vc = O.correct_vis(src.astype(np.complex64), uvw, freq, None, l0, m0)
    assert np.abs(vc - S).max() <= 1e-6 * S
    N = 32
    res = O.image_batch_corrected(src.astype(np.complex64), None, uvw, freq, N, 2.0e-3, 0, None, l0, m0)
    for t, c in np.ndindex(T, C):
        assert abs(res["images"][t, c, 0, N // 2, N // 2] - S) <= 1e-6 * S
    # without the correction the source sits off the phase centre: the centre pixel is lower
    plain = O.image_batch(src.astype(np.complex64), None, uvw, freq, N, 2.0e-3, 0)
    assert (plain["images"][:, :, 0, N // 2, N // 2] < 0.9 * S).all()


# ----------------------------------------------------------------------------- correlation

def numpy_correlate(volt, n_int, n_favg, pol_mode):
    """Eq. 3 as a complex matrix product X X^H per (interval, output channel), numpy complex128."""
    x = volt[..., 0].astype(np.float64) + 1j * volt[..., 1].astype(np.float64)     # [S][F][A][2]
    S, F, A, _ = x.shape
    T, C = S // n_int, F // n_favg
    x = x.reshape(T, n_int, C, n_favg, A * 2).transpose(0, 2, 4, 1, 3).reshape(T, C, A * 2, n_int * n_favg)
    R = x @ np.conj(x).transpose(0, 1, 3, 2) / (n_int * n_favg)                    # [T][C][2A][2A]
    rows, cols = np.tril_indices(A, k=-1)
    prods = [(0, 0), (0, 1), (1, 0), (1, 1)] if pol_mode == 4 else [(0, 0), (1, 1)]
    vis = np.stack([R[:, :, 2 * rows + p, 2 * cols + q] for p, q in prods], axis=2)
    autos = np.stack([R[:, :, 2 * np.arange(A) + p, 2 * np.arange(A) + q] for p, q in
                      [(0, 0), (0, 1), (1, 0), (1, 1)]], axis=3)
    return vis.astype(np.complex64), autos.astype(np.complex64)


def pin_correlate_matrix_product(O):
    """The correlator equals X X^H computed by numpy, exactly (integer sums, one rounding)."""
    g = np.random.default_rng(60)
    volt = g.integers(-128, 128, size=(12, 6, 5, 2, 2)).astype(np.int8)
    for n_int, n_favg in ((3, 2), (12, 1), (1, 6)):
        for mode in (4, 2):
            got = O.correlate(volt, n_int, n_favg, mode)
            vis, autos = numpy_correlate(volt, n_int, n_favg, mode)
            assert np.array_equal(got["vis"], vis), (n_int, n_favg, mode)
            assert np.array_equal(got["autos"], autos), (n_int, n_favg, mode)


def pin_correlate_quarter_turns(O):
    """Antenna voltages 100 i^m (X) and 50 i^n (Y), with m, n fixed per antenna and channel: every
    product is exact, e.g. XY of (i, j) = 5000 i^(m_i - n_j), and the autocorrelations are real
    powers 10000 and 2500."""
    g = np.random.default_rng(61)
    S, F, A = 4, 2, 6
    m = g.integers(0, 4, size=(F, A))
    n = g.integers(0, 4, size=(F, A))
    unit = {0: (1, 0), 1: (0, 1), 2: (-1, 0), 3: (0, -1)}
    volt = np.zeros((S, F, A, 2, 2), dtype=np.int8)
    for f, a in np.ndindex(F, A):
        volt[:, f, a, 0] = [100 * unit[m[f, a]][0], 100 * unit[m[f, a]][1]]
        volt[:, f, a, 1] = [50 * unit[n[f, a]][0], 50 * unit[n[f, a]][1]]
    res = O.correlate(volt, S, 1, 4)
    ph = lambda k: 1j ** (k % 4)
    b = 0
    for i in range(1, A):
        for j in range(i):
            for f in range(F):
                want = [10000 * ph(m[f, i] - m[f, j]), 5000 * ph(m[f, i] - n[f, j]),
                        5000 * ph(n[f, i] - m[f, j]), 2500 * ph(n[f, i] - n[f, j])]
                assert np.allclose(res["vis"][0, f, :, b], want, rtol=0, atol=0), (i, j, f)
            b += 1
    assert np.array_equal(res["autos"][0, :, :, 0], np.full((F, A), 10000, np.complex64))
    assert np.array_equal(res["autos"][0, :, :, 3], np.full((F, A), 2500, np.complex64))


def pin_correlate_averaging_groups(O):
    """A real X voltage a(s, f) common to all antennas: every XX visibility is the mean of a^2
    over its own block of n_int samples and n_favg channels (numpy's mean over the blocks)."""
    S, F, A, n_int, n_favg = 6, 8, 3, 3, 4
    a = (np.arange(S)[:, None] + 1) + 7 * np.arange(F)[None, :]
    a = (a % 127).astype(np.int8)
    volt = np.zeros((S, F, A, 2, 2), dtype=np.int8)
    volt[:, :, :, 0, 0] = a[:, :, None]
    res = O.correlate(volt, n_int, n_favg, 2)
    power = (a.astype(np.float64) ** 2).reshape(S // n_int, n_int, F // n_favg, n_favg).mean(axis=(1, 3))
    for b in range(A * (A - 1) // 2):
        assert np.array_equal(res["vis"][:, :, 0, b], power.astype(np.complex64))
        assert not res["vis"][:, :, 1, b].any()


# ----------------------------------------------------------------------------- de-dispersion

def pin_dispersion_delays_worked(O):
    """Delays against the hand-worked values of tests/golden/dispersion_delays.txt."""
    for ln in open(os.path.join(GOLDEN, "dispersion_delays.txt")):
        ln = ln.strip()
        if not ln or ln.startswith("#"):
            continue
        f, fr, dm, dt, want = ln.split()
        got = O.dispersion_delays(np.array([float(f), float(fr)]), float(dt), [float(dm)])
        assert got[0, 0] == int(want) and got[0, 1] == 0, (ln, got)


def pin_dedisperse_dm0_is_channel_mean(O):
    """At DM 0 every delay is 0 and de-dispersion is the channel average (numpy's mean)."""
    g = np.random.default_rng(80)
    imgs = g.normal(size=(5, 6, 4, 4)).astype(np.float32)
    d = O.dispersion_delays(150e6 + 1e6 * np.arange(6), 0.05, [0.0])
    assert not d.any()
    out = O.dedisperse(imgs, d, 5)
    assert np.abs(out[0] - imgs.astype(np.float64).mean(axis=1)).max() <= 1e-12


def pin_dedisperse_recovers_pulse(O):
    """A pulse of amplitude 3 at pixel (1, 2), dispersed with DM 4 over 6 channels (140 .. 165 MHz,
    50 ms steps: up to 5 steps of delay), is recovered in full at its arrival step at DM 4 and
    nowhere else; at the other trial DMs it is smeared."""
    C, T, N = 6, 40, 4
    freq = 140e6 + 5e6 * np.arange(C)
    dms = [0.0, 2.0, 4.0, 6.0]
    d = O.dispersion_delays(freq, 0.05, dms)
    assert len({tuple(r) for r in d}) == 4 and d[2].max() >= 3
    t0 = 3
    imgs = np.zeros((T, C, N, N), dtype=np.float32)
    for c in range(C):
        imgs[t0 + d[2, c], c, 1, 2] = 3.0
    t_out = T - int(d.max())
    out = O.dedisperse(imgs, d, t_out)
    assert out[2, t0, 1, 2] == 3.0
    assert np.count_nonzero(out[2]) == 1
    for k in (0, 1, 3):
        assert out[k].max() < 3.0


EXTRA_PINS = [pin_direct_dft, pin_image_average, pin_es_kernel_values, pin_es_transform, pin_conv_width1_is_nearest_cell,
              pin_conv_hermitian, pin_conv_matches_direct_transform, pin_conv_batch_consistency,
              pin_corrections_identity, pin_corrections_undo_gains, pin_corrections_phase_centre,
              pin_correlate_matrix_product, pin_correlate_quarter_turns, pin_correlate_averaging_groups,
              pin_dispersion_delays_worked, pin_dedisperse_dm0_is_channel_mean, pin_dedisperse_recovers_pulse]


PINS = [pin_cell_worked, pin_tiny_grid, pin_ifft1d_bruteforce, pin_ifft2d_bruteforce,
        pin_ifft2d_library, pin_closed_forms, pin_parseval_and_sum, pin_snapped_dft,
        pin_ungridded_bound, pin_point_source_centre, pin_shift_theorem, pin_realness,
        pin_invariants, pin_degenerate, pin_pols_share_flags]
