"""Seeded synthetic MWA-shaped inputs for batched dirty imaging.

This module only *generates* inputs: tile layouts, baseline coordinates, channel
frequencies, flags and point-source visibilities. It contains none of the
imaging arithmetic (no cell indices, no weighting, no transforms), so both the
CPU oracle and the HIP path can be fed from it without sharing any of the
method's code.

The visibility model is the forward relation of Section 4, Eq. 4, with the
primary beam set to one and the 1/sqrt(1-l^2-m^2) factor dropped (apparent flux):

    V_c(b) = sum_k S_k exp(-2 pi i (u_b l_k + v_b m_k) f_c / c)

plus complex Gaussian noise drawn independently for every
(time, channel, polarisation, baseline).

Array layouts (all C-contiguous):
    uvw_m   float64    [T][B][3]   metres, zenith phase centre (u = dE, v = dN, w = 0)
    freq_hz float64    [C]
    flags   uint8      [T][C][B]   1 = flagged, shared by all polarisations
    vis     complex64  [T][C][P][B]

Baseline b of the cross pair (i, j), i > j, has index b = i(i-1)/2 + j and
uvw = pos_i - pos_j (Section 6.2.2: lower-triangular visibility matrices;
autocorrelations are not imaged).

Random numbers come from NumPy PCG64 seeded by
SeedSequence(entropy=250515204, spawn_key=(config, stream)), streams:
0 tiles, 1 sky, 2 noise, 3 flags, 4 per-image parameters.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

C_LIGHT = 299792458.0
ARCMIN = math.pi / 10800.0
ENTROPY = 250515204

STREAM_TILES, STREAM_SKY, STREAM_NOISE, STREAM_FLAGS, STREAM_IMAGES = 0, 1, 2, 3, 4


def rng(config: int, stream: int) -> np.random.Generator:
    return np.random.Generator(
        np.random.PCG64(np.random.SeedSequence(entropy=ENTROPY, spawn_key=(config, stream))))


@dataclasses.dataclass
class Spec:
    """One synthetic workload (time steps x channels x polarisations, one grid size)."""
    name: str
    config: int            # seed namespace
    n_tiles: int
    T: int
    P: int
    freq_hz: np.ndarray    # [C]
    grid_n: int
    pixel_scale: float     # direction-cosine units per pixel
    n_src: int
    flag_frac: float
    weighting: int = 0     # 0 natural, 1 uniform
    noise_sigma: float = 0.1
    lm_max: float = 0.1

    @property
    def C(self) -> int:
        return int(self.freq_hz.shape[0])

    @property
    def B(self) -> int:
        return self.n_tiles * (self.n_tiles - 1) // 2

    @property
    def n_images(self) -> int:
        return self.T * self.C * self.P


def vcs_channels(n: int = 768, start_hz: float = 139.0e6, width_hz: float = 40.0e3) -> np.ndarray:
    """Fine-channel centres of a 30.72 MHz MWA band: start + width*(c + 1/2)."""
    return start_hz + width_hz * (np.arange(n, dtype=np.float64) + 0.5)


def spec_tiny() -> Spec:
    """Plain method, tiny: 128 tiles, 1 pol, 1 time step, 1 channel at 150 MHz, 256^2, 1 arcmin."""
    return Spec("tiny-256", 1, 128, 1, 1, np.array([150.0e6]), 256, ARCMIN, 5, 0.0)


def spec_vcs(T: int = 100, C: int = 768, P: int = 2) -> Spec:
    """MWA VCS scale: 128 tiles, 2 pols, 768 x 40 kHz channels from 139 MHz, 100 x 1 ms, 1024^2."""
    freqs = vcs_channels()[:C]
    return Spec("vcs-1024", 2, 128, T, P, freqs, 1024, ARCMIN, 50, 0.10)


def spec_phase2(T: int = 20, C: int = 3072, P: int = 2) -> Spec:
    """Phase II scale: 144 tiles, 3072 x 10 kHz channels from 185 MHz, 2048^2 at 0.75 arcmin, uniform."""
    freqs = (185.0e6 + 10.0e3 * (np.arange(3072, dtype=np.float64) + 0.5))[:C]
    return Spec("phase2-2048", 3, 144, T, P, freqs, 2048, 0.75 * ARCMIN, 50, 0.10, weighting=1)


def spec_precision(T: int = 10, C: int = 256) -> Spec:
    """Precision form: config-2 channels c = 3j (j < 256), single pol, 4096^2 at 1 arcmin."""
    freqs = vcs_channels()[0:768:3][:C]
    return Spec("precision-4096", 4, 128, T, 1, freqs, 4096, ARCMIN, 50, 0.10)


def tile_positions(n_tiles: int, g: np.random.Generator, core_frac: float = 0.4,
                   core_radius: float = 50.0, array_radius: float = 1500.0) -> np.ndarray:
    """Tile (east, north) positions in metres: a dense core plus a uniform disc (r = R sqrt(U))."""
    n_core = int(round(core_frac * n_tiles))
    radius = np.concatenate([np.full(n_core, core_radius), np.full(n_tiles - n_core, array_radius)])
    r = radius * np.sqrt(g.random(n_tiles))
    phi = 2.0 * np.pi * g.random(n_tiles)
    return np.stack([r * np.cos(phi), r * np.sin(phi)], axis=1)


def baseline_uvw(pos: np.ndarray) -> np.ndarray:
    """Cross baselines i > j in lower-triangular order; uvw = pos_i - pos_j, w = 0. Shape [B][3]."""
    n = pos.shape[0]
    ii, jj = [], []
    for i in range(1, n):
        ii.extend([i] * i)
        jj.extend(range(i))
    ii = np.asarray(ii)
    jj = np.asarray(jj)
    uvw = np.zeros((ii.size, 3), dtype=np.float64)
    uvw[:, 0] = pos[ii, 0] - pos[jj, 0]
    uvw[:, 1] = pos[ii, 1] - pos[jj, 1]
    return uvw


def sky_model(n_src: int, g: np.random.Generator, lm_max: float = 0.1):
    """Point sources: flux U[1,10] Jy, (l, m) U[-lm_max, lm_max]^2. Returns (S, l, m)."""
    s = g.uniform(1.0, 10.0, n_src)
    l = g.uniform(-lm_max, lm_max, n_src)
    m = g.uniform(-lm_max, lm_max, n_src)
    return s, l, m


def model_visibilities(uvw_m: np.ndarray, freq_hz: np.ndarray, sky) -> np.ndarray:
    """Noise-free V[c][b] = sum_k S_k exp(-2 pi i (u l_k + v m_k) f_c / c), complex128 (Eq. 4, A = 1)."""
    s, l, m = sky
    ul = uvw_m[:, 0:1] * l[None, :] + uvw_m[:, 1:2] * m[None, :]          # [B][K] metres
    out = np.empty((freq_hz.size, uvw_m.shape[0]), dtype=np.complex128)
    for c, f in enumerate(freq_hz):
        out[c] = np.exp(-2j * np.pi * ul * (f / C_LIGHT)) @ s
    return out


@dataclasses.dataclass
class Problem:
    spec: Spec
    uvw_m: np.ndarray      # [T][B][3] float64
    freq_hz: np.ndarray    # [C] float64
    flags: np.ndarray      # [T][C][B] uint8
    vis: np.ndarray        # [T][C][P][B] complex64


def make_problem(spec: Spec, per_time_uvw_jitter: float = 0.0) -> Problem:
    """Generate every array of a workload on the host (use for sizes that fit comfortably in RAM)."""
    pos = tile_positions(spec.n_tiles, rng(spec.config, STREAM_TILES))
    uvw1 = baseline_uvw(pos)
    uvw = np.repeat(uvw1[None], spec.T, axis=0).copy()
    if per_time_uvw_jitter:
        jg = rng(spec.config, STREAM_IMAGES)
        uvw[:, :, :2] += jg.normal(0.0, per_time_uvw_jitter, size=uvw[:, :, :2].shape)
    sky = sky_model(spec.n_src, rng(spec.config, STREAM_SKY), spec.lm_max)
    model = model_visibilities(uvw1, spec.freq_hz, sky)                     # [C][B]
    ng = rng(spec.config, STREAM_NOISE)
    shape = (spec.T, spec.C, spec.P, spec.B)
    noise = ng.normal(0.0, spec.noise_sigma, size=shape + (2,))
    vis = np.empty(shape, dtype=np.complex64)
    vis.real = model.real[None, :, None, :] + noise[..., 0]
    vis.imag = model.imag[None, :, None, :] + noise[..., 1]
    if per_time_uvw_jitter:
        for t in range(spec.T):
            mt = model_visibilities(uvw[t], spec.freq_hz, sky)
            vis[t].real = mt.real[:, None, :] + noise[t, ..., 0]
            vis[t].imag = mt.imag[:, None, :] + noise[t, ..., 1]
    fg = rng(spec.config, STREAM_FLAGS)
    flags = (fg.random((spec.T, spec.C, spec.B)) < spec.flag_frac).astype(np.uint8)
    return Problem(spec, np.ascontiguousarray(uvw), spec.freq_hz.copy(), flags, vis)


def make_problem_device(spec: Spec, device, seed: Optional[int] = None):
    """Generate a workload directly in device memory (for sizes too large to build on the host).

    Tiles, baselines and the sky come from the same NumPy streams as make_problem, so
    the noise-free model is identical; the noise and flags are drawn with a seeded torch
    generator on the device instead of PCG64. Returns a dict of torch tensors
    (uvw_m, freq_hz, flags, vis) with the layouts above.
    """
    import torch

    pos = tile_positions(spec.n_tiles, rng(spec.config, STREAM_TILES))
    uvw1 = baseline_uvw(pos)
    sky = sky_model(spec.n_src, rng(spec.config, STREAM_SKY), spec.lm_max)
    gen = torch.Generator(device=device)
    gen.manual_seed(ENTROPY * 16 + spec.config if seed is None else seed)
    uvw_d = torch.from_numpy(np.repeat(uvw1[None], spec.T, axis=0).copy()).to(device)
    freq_d = torch.from_numpy(spec.freq_hz.copy()).to(device)
    s = torch.from_numpy(sky[0]).to(device)
    l = torch.from_numpy(sky[1]).to(device)
    m = torch.from_numpy(sky[2]).to(device)
    u = torch.from_numpy(uvw1[:, 0].copy()).to(device)
    v = torch.from_numpy(uvw1[:, 1].copy()).to(device)
    ul = u[:, None] * l[None, :] + v[:, None] * m[None, :]                   # [B][K]
    model = torch.empty((spec.C, spec.B), dtype=torch.complex64, device=device)
    cstep = 64
    for c0 in range(0, spec.C, cstep):
        f = freq_d[c0:c0 + cstep] / C_LIGHT
        ph = (-2.0 * math.pi) * f[:, None, None] * ul[None]                 # [c][B][K]
        re = torch.cos(ph) @ s
        im = torch.sin(ph) @ s
        model[c0:c0 + cstep] = torch.complex(re, im).to(torch.complex64)
    vis = torch.empty((spec.T, spec.C, spec.P, spec.B), dtype=torch.complex64, device=device)
    flags = torch.empty((spec.T, spec.C, spec.B), dtype=torch.uint8, device=device)
    vr = torch.view_as_real(vis)
    for t in range(spec.T):
        noise = torch.randn((spec.C, spec.P, spec.B, 2), generator=gen, device=device,
                            dtype=torch.float32) * spec.noise_sigma
        vr[t] = noise + torch.view_as_real(model)[:, None, :, :]
        flags[t] = (torch.rand((spec.C, spec.B), generator=gen, device=device)
                    < spec.flag_frac).to(torch.uint8)
    return {"uvw_m": uvw_d, "freq_hz": freq_d, "flags": flags, "vis": vis}


# ---------------------------------------------------------------------------- uneven batches
def uneven_layout(n_img: int = 4096, config: int = 5, n_tiles: int = 128, f_lo: float = 70.0e6,
                  f_hi: float = 300.0e6, sizes=(512, 1024, 2048), thresholds=(120.0e6, 200.0e6),
                  unflagged=(0.7, 1.0), n_src: int = 50, margin: float = 1.05):
    """Layout of a batch of images with channel-dependent grid sizes and visibility counts.

    Image i observes f_i = f_lo + (f_hi - f_lo)(i + 1/2)/n_img; its grid is sizes[0] below
    thresholds[0], sizes[1] below thresholds[1], else sizes[2]; its pixel scale is
    dl_i = 1 / (2 margin u_max f_i / c) so that every baseline falls on the grid; it keeps a
    fraction U[unflagged] of the baselines: a cyclic window of a seeded permutation of the array's
    baselines, stored once twice over so every window is contiguous. Returns a dict with the
    per-image fields of the descriptors (vis, uvw and image offsets, B_i, N_i, f_i, dl_i), the
    doubled baseline table uvw_ext [2B][3] and the sky.
    """
    g = rng(config, STREAM_IMAGES)
    pos = tile_positions(n_tiles, rng(config, STREAM_TILES))
    uvw = baseline_uvw(pos)
    B = uvw.shape[0]
    perm = g.permutation(B)
    uvw_ext = np.concatenate([uvw[perm], uvw[perm]], axis=0)
    u_max = float(np.abs(uvw[:, :2]).max())
    freq = f_lo + (f_hi - f_lo) * (np.arange(n_img) + 0.5) / n_img
    grid_n = np.where(freq < thresholds[0], sizes[0], np.where(freq < thresholds[1], sizes[1], sizes[2]))
    dl = 1.0 / (2.0 * margin * u_max * freq / C_LIGHT)
    frac = g.uniform(unflagged[0], unflagged[1], n_img)
    nb = np.maximum(1, np.round(frac * B)).astype(np.int64)
    start = g.integers(0, B, n_img)
    vis_off = np.concatenate([[0], np.cumsum(nb)[:-1]])
    img_off = np.concatenate([[0], np.cumsum(grid_n.astype(np.int64) ** 2)[:-1]])
    sky = sky_model(n_src, rng(config, STREAM_SKY))
    return {"n_img": n_img, "B": B, "uvw_ext": uvw_ext, "freq_hz": freq, "grid_n": grid_n.astype(np.int64),
            "pixel_scale": dl, "n_baselines": nb, "uvw_offset": start, "vis_offset": vis_off,
            "image_offset": img_off, "vis_len": int(nb.sum()),
            "images_len": int((grid_n.astype(np.int64) ** 2).sum()), "max_b": int(nb.max()),
            "max_n": int(grid_n.max()), "sky": sky, "config": config}


def uneven_descriptors(lay, dtype):
    """The layout's descriptors as a structured array of `dtype` (the library's blink_image_desc)."""
    d = np.zeros(lay["n_img"], dtype=dtype)
    d["vis_offset"] = lay["vis_offset"]
    d["uvw_offset"] = lay["uvw_offset"]
    d["flag_offset"] = 0
    d["image_offset"] = lay["image_offset"]
    d["freq_hz"] = lay["freq_hz"]
    d["pixel_scale"] = lay["pixel_scale"]
    d["n_baselines"] = lay["n_baselines"]
    d["grid_n"] = lay["grid_n"]
    return d


def uneven_image_inputs(lay, i, noise_sigma: float = 0.1):
    """Visibilities (complex64 [B_i]) and uvw ([B_i][3]) of image i on the host."""
    o, n = int(lay["uvw_offset"][i]), int(lay["n_baselines"][i])
    uvw = lay["uvw_ext"][o:o + n]
    model = model_visibilities(uvw, np.array([lay["freq_hz"][i]]), lay["sky"])[0]
    ng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        entropy=ENTROPY, spawn_key=(lay["config"], STREAM_NOISE, i))))
    noise = ng.normal(0.0, noise_sigma, size=(n, 2))
    vis = np.empty(n, np.complex64)
    vis.real = model.real + noise[:, 0]
    vis.imag = model.imag + noise[:, 1]
    return vis, uvw


def uneven_vis_host(lay, noise_sigma: float = 0.1):
    """All packed visibilities on the host (complex64 [sum B_i]); for small batches."""
    out = np.empty(lay["vis_len"], np.complex64)
    for i in range(lay["n_img"]):
        v, _ = uneven_image_inputs(lay, i, noise_sigma)
        o = int(lay["vis_offset"][i])
        out[o:o + v.size] = v
    return out


def uneven_vis_device(lay, device, noise_sigma: float = 0.1, seed: Optional[int] = None):
    """All packed visibilities generated on the device (same model; noise from a torch generator)."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(ENTROPY * 16 + lay["config"] if seed is None else seed)
    s, l, m = (torch.from_numpy(x).to(device) for x in lay["sky"])
    ext = torch.from_numpy(lay["uvw_ext"]).to(device)
    out = torch.empty(lay["vis_len"], dtype=torch.complex64, device=device)
    ov = torch.view_as_real(out)
    for i in range(lay["n_img"]):
        o, n, vo = int(lay["uvw_offset"][i]), int(lay["n_baselines"][i]), int(lay["vis_offset"][i])
        uvw = ext[o:o + n]
        ph = (-2.0 * math.pi * lay["freq_hz"][i] / C_LIGHT) * (uvw[:, 0:1] * l[None] + uvw[:, 1:2] * m[None])
        re = torch.cos(ph) @ s
        im = torch.sin(ph) @ s
        noise = torch.randn((n, 2), generator=gen, device=device, dtype=torch.float32) * noise_sigma
        ov[vo:vo + n, 0] = re.to(torch.float32) + noise[:, 0]
        ov[vo:vo + n, 1] = im.to(torch.float32) + noise[:, 1]
    return out
