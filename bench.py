#!/usr/bin/env python3
"""Benchmark: batched dirty imaging of the MWA VCS-scale workload on one MI355X.

Workload (synthetic, MWA-shaped): 128 tiles -> 8128 cross baselines, 2 polarisations,
768 fine channels of 40 kHz from 139 MHz, 100 time steps of 1 ms, 1024 x 1024 FP32 images,
natural weighting, 50 point sources plus noise, 10% random flags. All inputs are generated on
the GPU and stay resident in HBM; a step images one time step (768 x 2 = 1536 images) into an
HBM ring buffer; the default run times all 100 steps (153,600 images).

Prints one JSON line with images/s (FP32 form), the roofline position of the dominant kernel
(bytes from the algorithmic byte model / its hipEvent-measured launch time), per-kernel figures,
the FP64 CPU oracle timed on a bounded sample of the same workload on the host cores, and the
other forms measured beside it on the same GPU: the split-precision matrix-core FFT forms on
this workload and on the 4096^2 precision workload (images/s ratio to FP32), convolutional
gridding (W = 8) on this workload, the Stokes I + band average of one time step's images, and
the uneven batch (4096 images of 512^2 .. 2048^2 in one blink_image_batch_desc call, in the form
and plan the descriptor autotuner picks, eager and as a hipGraph).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "dirty images/sec (1024² grid, 8128 baselines) and % HBM roofline; MFMA vs FP32"
HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0     # dense int8 matrix-core peak of the MI355X


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# device sources of the batched FP32 imaging kernels (the host code in api.hip, the correlator, the
# uneven-batch kernel and the split forms' instantiation unit do not change their code; the launch
# configuration is checked separately through the plan)
IMAGING_KERNEL_SOURCES = ("conv_device.hpp", "fft_device.hpp", "imaging_device.hpp", "kernels.hip", "kernels.hpp",
                          "launch.hpp", "split_fft.hpp")


def kernel_source_hash():
    """SHA-256 prefix of the imaging kernels' sources; byte counters are reported only for the
    sources they came from."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_2505_15204_amd", "csrc")
    h = hashlib.sha256()
    for f in IMAGING_KERNEL_SOURCES:
        h.update(f.encode())
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def counter_traffic(tag, kernel, plan):
    """Scaled FETCH_SIZE + WRITE_SIZE bytes per launch of `kernel` from profiles/<tag>_hbm_counters.md,
    or None when absent or taken from different kernel sources or a different execution plan."""
    path = os.path.join(ROOT, "profiles", f"{tag}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    for ln in open(path):
        if ln.startswith("traffic-json:"):
            rec = json.loads(ln.split(":", 1)[1])
            if rec.get("source_hash") != kernel_source_hash() or rec.get("plan") != plan:
                return None
            return rec.get("bytes_per_launch", {}).get(kernel)
    return None


SPEED_OF_LIGHT = 299792458.0


def column_extent(torch, d, spec, steps):
    """Mean number of half-spectrum columns that carry data over the images of `steps` steps (step i
    images time step i mod T, every channel): 1 + the largest |ku| = |rint(u k)| over the kept
    visibilities of each (t, c) pair (not flagged, inside the grid), 0 when none is kept. Columns
    beyond it are zero in the grid and therefore in the half spectrum."""
    N = spec.grid_n
    k = d["freq_hz"] * (N * spec.pixel_scale / SPEED_OF_LIGHT)              # cells per metre, [C]
    per_t = {}
    for i in range(steps):
        t = i % spec.T
        if t not in per_t:
            iu = torch.round(d["uvw_m"][t, :, 0][None, :] * k[:, None])      # [C][B], ties to even
            iv = torch.round(d["uvw_m"][t, :, 1][None, :] * k[:, None])
            kept = (iu.abs() < N / 2) & (iv.abs() < N / 2) & (d["flags"][t] == 0)
            ext = torch.where(kept, iu.abs() + 1, torch.zeros_like(iu)).amax(dim=1)
            per_t[t] = float(ext.mean())
    return sum(per_t[i % spec.T] for i in range(steps)) / steps


def kernel_unit_bytes(spec, ext=None):
    """Algorithmic HBM bytes per unit of work of each kernel (unit, bytes).

    `ext` is the mean number of half-spectrum columns that carry data per image (column_extent);
    None means all N/2 (paths that transform every column).
    grid_colfft: per image, write the nonzero columns of the half-spectrum intermediate (N rows x
                 ext columns of complex64, 8 N ext B; 4 N^2 B with every column) and read each
                 visibility once (8 B) plus its placement record (8 B).
    row_fft:     per image, read those columns (8 N ext B) and write the FP32 image (4 N^2 B).
    bin:         per (t,c) pair, read the flag (1 B) of each baseline and write at most one
                 placement record (8 B) per baseline (one per kept visibility in the half plane,
                 two for the few on the u = 0 column); u, v (16 B per baseline) are shared by the
                 C channels of a time step, so each pair is charged 16 B / C of them.
    """
    N, B, C = spec.grid_n, spec.B, spec.C
    h = 8 * N * (N / 2 if ext is None else ext)
    return {
        "grid_colfft": ("image", round(h + 16 * B)),
        "row_fft": ("image", round(h + 4 * N * N)),
        "bin": ("pair", 9 * B + (16 * B) // C),
    }


def path_bytes_per_image(spec, ext=None):
    """The whole path per image: write and read the nonzero half-spectrum columns, write the image,
    read the visibilities and placements and the per-pair binning bytes shared by the pols."""
    N, B, P = spec.grid_n, spec.B, spec.P
    return round(16 * N * (N / 2 if ext is None else ext) + 4 * N * N + 8 * B + B // P)


def conv_unit_bytes(torch, d, spec, width, steps, strip=16, band=16):
    """Algorithmic bytes of the convolutional path (kernel support `width` cells), per unit.

    Counted from the workload's geometry over the (t, c) pairs of `steps` steps, with the keep
    rule and tap rule of the binning: a kept visibility's two placements reach the columns
    ceil(+-x - W/2) .. + n_u - 1 and the rows likewise (n = min(W, ceil(W/2 - d0)) taps).
    bin:         per pair, the flags (1 B per baseline), the shared u, v (16 B per baseline over C
                 pairs), one 16-byte record per (placement, column strip of `strip` columns, row
                 band of `band` rows) it reaches, and the (strips x bands + 1) 4-byte offsets;
    grid_colfft: per image, write the half-spectrum columns up to the last tap column (8 N ext B)
                 and read one record (16 B) and one visibility (8 B) per record;
    row_fft:     per image, read those columns and write the image (8 N ext + 4 N^2 B).
    Also returns the mean column extent."""
    N, B, C, W = spec.grid_n, spec.B, spec.C, width
    h = W / 2.0
    half = N // 2
    nstrips, nbands = half // strip, N // band
    recs, exts = [], []
    for i in range(steps):
        t = i % spec.T
        k = d["freq_hz"] * (N * spec.pixel_scale / SPEED_OF_LIGHT)                 # [C]
        x = d["uvw_m"][t, :, 0][None, :] * k[:, None]                               # [C][B] FP64
        y = d["uvw_m"][t, :, 1][None, :] * k[:, None]
        kept = (torch.round(x).abs() < half) & (torch.round(y).abs() < half) & (d["flags"][t] == 0)
        n_rec = torch.zeros(C, dtype=torch.float64, device=x.device)
        last = torch.zeros(C, dtype=torch.float64, device=x.device)
        for sgn in (1.0, -1.0):
            xs, ys = sgn * x, sgn * y
            ju0 = torch.ceil(xs - h)
            ju0 = torch.where(ju0 - xs > -h, ju0, ju0 + 1)
            jv0 = torch.ceil(ys - h)
            jv0 = torch.where(jv0 - ys > -h, jv0, jv0 + 1)
            nu = torch.clamp(torch.ceil(h - (ju0 - xs)), max=W)
            nv = torch.clamp(torch.ceil(h - (jv0 - ys)), max=W)
            ju0, jv0, nu, nv = ju0.long(), jv0.long(), nu.long(), nv.long()
            strips = torch.zeros_like(ju0)
            prev = torch.full_like(ju0, -2)
            for j in range(W):
                col = (ju0 + j) % N
                s_j = torch.where(col < half, col // strip, torch.where(col == half, torch.zeros_like(col), -1))
                s_j = torch.where(j < nu, s_j, torch.full_like(s_j, -1))
                strips += ((s_j >= 0) & (s_j != prev)).long()
                prev = s_j
                in_half = (j < nu) & (col < half)        # the Nyquist column is packed into column 0
                last = torch.maximum(last, torch.where(kept & in_half, col + 1, torch.zeros_like(col)).amax(dim=1).double())
            b0 = (jv0 % N) // band
            b1 = ((jv0 + nv - 1) % N) // band
            bands = torch.where(nv > 0, 1 + (b1 != b0).long(), torch.zeros_like(nv))
            n_rec += torch.where(kept, strips * bands, torch.zeros_like(strips)).sum(dim=1).double()
        recs.append(n_rec.mean().item())
        exts.append(last.mean().item())
    R, ext = sum(recs) / len(recs), sum(exts) / len(exts)
    hb = 8 * N * ext
    return {
        "grid_colfft": ("image", round(hb + 24 * R)),        # each image reads all of its pair's records
        "row_fft": ("image", round(hb + 4 * N * N)),
        "bin": ("pair", round(B + (16 * B) // C + 16 * R + 4 * (nstrips * nbands + 1))),
    }, ext


# The last-level cache (AMD Infinity Cache, "MALL") of the MI355X: 256 MB in front of HBM.
MALL_BYTES = 256 * 10**6


def cpu_baseline(d, spec, budget_s):
    """Time the FP64 oracle (as it stands) on channels 0..k-1 of time step 0, both pols."""
    import oracle

    oracle.build(force=False)
    threads = oracle.max_threads()
    vis = d["vis"][0:1].cpu().numpy()
    flags = d["flags"][0:1].cpu().numpy()
    uvw = d["uvw_m"][0:1].cpu().numpy()
    freq = d["freq_hz"].cpu().numpy()

    def run(k):
        t0 = time.perf_counter()
        oracle.image_batch(vis[:, :k], flags[:, :k], uvw, freq[:k], spec.grid_n, spec.pixel_scale, 0,
                           n_threads=threads)
        return time.perf_counter() - t0

    per_pair = run(threads)/threads          # one pair per thread for calibration
    k = max(threads, min(spec.C, int(budget_s / max(per_pair, 1e-6))))
    k = (k // threads) * threads or threads
    dt = run(k)
    n_img = k * spec.P
    return {"value": round(n_img / dt, 3), "unit": "images/s", "cores": threads, "kind": "oracle",
            "sample": f"time step 0, channels 0..{k - 1}, {spec.P} pols: {n_img} images of "
                      f"{spec.grid_n}^2 in {dt:.1f} s (FP64 C oracle, OpenMP over (t,c))"}


FORMS = (("fp32", 0), ("split_f16", 1), ("split_bf16", 2))


def timed(torch, fn, steps, warmup):
    """GPU milliseconds of `steps` calls of fn(i) after `warmup` untimed ones (events on the current stream)."""
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        fn(i)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def kernel_table(prof, units, ub):
    """Per-kernel launches, average duration and (with a byte model) achieved GB/s."""
    kernels = {}
    for name, (ms, launches) in prof.items():
        if launches == 0:
            continue
        avg_s = ms / launches / 1e3
        entry = {"launches": launches, "avg_ms": round(ms / launches, 5), "total_ms": round(ms, 3)}
        if name in ub:
            unit, per_unit = ub[name]
            per_launch = per_unit * units[unit] / launches
            gbs = per_launch / avg_s / 1e9
            entry.update({"unit": unit, "bytes_per_unit": per_unit, "bytes_per_launch": round(per_launch),
                          "achieved_GB_s": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)})
        kernels[name] = entry
    return kernels


def profiled(ctx, torch, fn, steps):
    """The same calls again with hipEvents around every library launch; returns (per-kernel, ms)."""
    ctx.profile_enable(True)
    ms = timed(torch, fn, steps, 0)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    return prof, ms


def bench_correlator(ctx, torch, steps, warmup):
    """The correlator on the high-time-resolution shape: 128 tiles x 2 pols, 3072 fine channels of
    10 kHz averaged by 4 into 768 output channels of 40 kHz, 100 us samples integrated over 20 ms
    (n_int = 200); a step correlates 10 intervals (0.2 s of data, 3.1 GB of int8 voltages)."""
    A, F, n_int, n_favg, T = 128, 3072, 200, 4, 10
    S = n_int * T
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(30)
    volt = torch.randint(-128, 128, (S, F, A, 2, 2), generator=gen, device="cuda:0", dtype=torch.int8)
    C, B, K = F // n_favg, A * (A - 1) // 2, n_int * n_favg
    out = {"workload": "correlator: 128 tiles x 2 pols, 3072 x 10 kHz fine channels -> 768 x 40 kHz, 100 us samples, "
                       "20 ms integrations; a step is 10 integrations (0.2 s of data)",
           "input_bytes_per_step": S * F * A * 4}
    for mode in (4, 2):
        vis = torch.empty((T, C, mode, B), dtype=torch.complex64, device="cuda:0")
        ms = timed(torch, lambda i: ctx.blink_correlate(volt, n_int, n_favg, mode, out=vis), steps, warmup) / steps
        # algorithmic work: every needed product of every pair over K terms, 8 integer ops per
        # complex multiply-accumulate; bytes: read the voltages once, write the visibilities
        ops = T * C * (B * mode) * K * 8
        nbytes = S * F * A * 4 + T * C * mode * B * 8
        out[f"pol_mode_{mode}"] = {
            "ms_per_step": round(ms, 4),
            "data_seconds_per_second": round(0.2 / (ms / 1e3), 2),
            "achieved_TOP_s": round(ops / (ms / 1e3) / 1e12, 1),
            "frac_int8_mfma": round(ops / (ms / 1e3) / 1e12 / INT8_PEAK_TOPS, 4),
            "achieved_GB_s": round(nbytes / (ms / 1e3) / 1e9, 1),
            "frac_hbm": round(nbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"correlator pol_mode {mode}: {ms:.3f} ms per 0.2 s of data, "
            f"{ops / (ms / 1e3) / 1e12:.0f} TOP/s, {nbytes / (ms / 1e3) / 1e9:.0f} GB/s")
        del vis
    del volt
    return out


def bench_dedispersion(ctx, torch, blink, steps, warmup):
    """Incoherent de-dispersion of a Stokes I cube shaped like the paper's FRB case (Table 1: 512^2
    images, 768 x 40 kHz channels): 40 steps of 50 ms, 16 trial DMs 0 .. 10 pc cm^-3."""
    import numpy as np
    T, C, N, dt = 40, 768, 512, 0.05
    freq = 139.0e6 + 40.0e3 * (np.arange(C) + 0.5)
    dms = np.linspace(0.0, 10.0, 16)
    delays = blink.dispersion_delays(freq, dt, dms)
    t_out = T - int(delays.max())
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(40)
    cube = torch.randn((T, C, N, N), generator=gen, device="cuda:0", dtype=torch.float32)
    out = torch.empty((len(dms), t_out, N, N), dtype=torch.float32, device="cuda:0")
    ws = torch.empty(blink.dedisperse_workspace_size(C, len(dms)), dtype=torch.uint8, device="cuda:0")
    ms = timed(torch, lambda i: ctx.blink_dedisperse(cube, delays, t_out, out=out, workspace=ws), steps, warmup) / steps
    # bytes of the direct method: every output image reads its C delayed channel images once
    nbytes = len(dms) * t_out * (C + 1) * N * N * 4
    res = {"workload": f"de-dispersion: {T} x 50 ms steps, {C} x 40 kHz channels from 139 MHz, {N}^2 Stokes I "
                       f"images, {len(dms)} trial DMs 0 .. 10 pc cm^-3 (max delay {int(delays.max())} steps)",
           "ms": round(ms, 3), "dedispersed_images_per_s": round(len(dms) * t_out / (ms / 1e3), 1),
           "bytes_direct_method": nbytes, "achieved_GB_s": round(nbytes / (ms / 1e3) / 1e9, 1),
           "frac_hbm": round(nbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"de-dispersion: {ms:.2f} ms for {len(dms)} x {t_out} images, {nbytes / (ms / 1e3) / 1e9:.0f} GB/s")
    del cube, out, ws
    torch.cuda.empty_cache()
    return res


def bench_precision_workload(ctx, torch, blink, synth, steps, warmup):
    """The 4096^2 precision workload (10 time steps x 256 channels x 1 pol) in every FFT form;
    a step images one time step (256 images) into a one-step ring buffer."""
    spec = synth.spec_precision()
    T, C, P, B, N = spec.T, spec.C, spec.P, spec.B, spec.grid_n
    log(f"precision workload {spec.name}: T={T} C={C} P={P} N={N}")
    d = synth.make_problem_device(spec, "cuda:0")
    images = torch.empty((1, C, P, N, N), dtype=torch.float32, device="cuda:0")
    ws = torch.empty(max(blink.image_batch_workspace_size(1, C, P, B, N, 0, p) for _, p in FORMS),
                     dtype=torch.uint8, device="cuda:0")
    out = {"workload": "precision-4096: 8128 baselines, 256 channels (every third VCS channel), 1 pol, "
                       "10 time steps, 4096^2 grid, 1 arcmin, natural weighting", "images_per_step": C * P}
    # images kept for the error check against the FP64 oracle (made in the CPU-baseline leg)
    samples = {"t": (steps - 1) % T, "channels": PRECISION_SAMPLE_CHANNELS, "images": {}}
    for name, prec in FORMS:
        def step(i, prec=prec):
            t = i % T
            ctx.blink_image_batch(d["vis"][t:t + 1], d["flags"][t:t + 1], d["uvw_m"][t:t + 1], d["freq_hz"], N,
                                  spec.pixel_scale, 0, precision=prec, out=images, workspace=ws)
        ms = timed(torch, step, steps, warmup)
        out[name] = {"images_per_s": round(steps * C * P / (ms / 1e3), 1), "ms_per_step": round(ms / steps, 3)}
        samples["images"][name] = images[0, list(samples["channels"]), 0].cpu().numpy()
    for name, _ in FORMS[1:]:
        out[name]["vs_fp32"] = round(out[name]["images_per_s"] / out["fp32"]["images_per_s"], 4)
    t = samples["t"]
    samples["inputs"] = {"vis": d["vis"][t:t + 1].cpu().numpy(), "flags": d["flags"][t:t + 1].cpu().numpy(),
                         "uvw_m": d["uvw_m"][t:t + 1].cpu().numpy(), "freq_hz": d["freq_hz"].cpu().numpy(),
                         "grid_n": N, "pixel_scale": spec.pixel_scale}
    del d, images, ws
    torch.cuda.empty_cache()
    return out, samples


# channels of the 4096^2 precision workload whose images are compared with the FP64 oracle
PRECISION_SAMPLE_CHANNELS = (0, 127, 255)


def precision_errors(samples):
    """Per-image error of every FFT form against the FP64 oracle on the sampled 4096^2 images:
    relative L2, peak-pixel relative error and the 6-sigma detections missing / spurious. Runs in
    the CPU-baseline leg (it times the oracle on these images as well)."""
    import numpy as np

    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from image_checks import local_maxima, peak_error, recovery, rel_l2, robust_sigma

    inp = samples["inputs"]
    ch = list(samples["channels"])
    t0 = time.perf_counter()
    ref = oracle.image_batch(inp["vis"][:, ch], inp["flags"][:, ch], inp["uvw_m"], inp["freq_hz"][ch],
                             inp["grid_n"], inp["pixel_scale"], 0, n_threads=oracle.max_threads())["images"]
    dt = time.perf_counter() - t0
    out = {"time_step": samples["t"], "channels": ch, "oracle_seconds": round(dt, 2),
           "oracle_threads": oracle.max_threads()}
    for name, imgs in samples["images"].items():
        per = []
        for j in range(len(ch)):
            r = ref[0, j, 0]
            missing, spurious = recovery(imgs[j], r)
            per.append({"rel_l2": float(f"{rel_l2(imgs[j], r):.3e}"), "peak_err": float(f"{peak_error(imgs[j], r):.3e}"),
                        "oracle_6sigma_maxima": len(local_maxima(r, 6.0 * robust_sigma(r))),
                        "missing_6sigma": len(missing), "spurious_6sigma": len(spurious)})
        out[name] = per
        log(f"precision-4096 {name}: rel_l2 " + ", ".join(f"{p['rel_l2']:.2e}" for p in per) +
            "; peak " + ", ".join(f"{p['peak_err']:.2e}" for p in per) +
            f"; 6-sigma missing/spurious {sum(p['missing_6sigma'] for p in per)}/"
            f"{sum(p['spurious_6sigma'] for p in per)}")
    return out


def bench_phase2(ctx, torch, blink, synth, steps, warmup):
    """The Phase II shape: 144 tiles (10296 baselines), 2 pols, 3072 x 10 kHz channels from 185 MHz,
    20 time steps of 1 ms, 2048^2 at 0.75 arcmin, uniform weighting. A step images one time step
    (6144 images) in four calls of 768 channels into a ring of 1536 images."""
    spec = synth.spec_phase2()
    T, C, P, B, N = spec.T, spec.C, spec.P, spec.B, spec.grid_n
    log(f"Phase II workload {spec.name}: T={T} C={C} P={P} B={B} N={N}, uniform")
    d = synth.make_problem_device(spec, "cuda:0")
    CH = 768
    images = torch.empty((1, CH, P, N, N), dtype=torch.float32, device="cuda:0")
    wsum = torch.empty((1, CH, P), dtype=torch.float64, device="cuda:0")
    nout = torch.empty((1, CH), dtype=torch.int32, device="cuda:0")
    ws = torch.empty(blink.image_batch_workspace_size(1, CH, P, B, N, 1), dtype=torch.uint8, device="cuda:0")

    def step(i):
        t = i % T
        for c0 in range(0, C, CH):
            ctx.blink_image_batch(d["vis"][t:t + 1, c0:c0 + CH], d["flags"][t:t + 1, c0:c0 + CH], d["uvw_m"][t:t + 1],
                                  d["freq_hz"][c0:c0 + CH], N, spec.pixel_scale, 1, out=images, weight_sum=wsum,
                                  n_out=nout, workspace=ws)
    ms = timed(torch, step, steps, warmup)
    n_img = steps * C * P
    value = n_img / (ms / 1e3)
    prof, _ = profiled(ctx, torch, step, 1)
    kernels = kernel_table(prof, {"image": C * P, "pair": C}, kernel_unit_bytes(spec, column_extent(torch, d, spec, 1)))
    ext = column_extent(torch, d, spec, steps)
    per_image = path_bytes_per_image(spec, ext)
    out = {"workload": "phase2-2048: 144 tiles (10296 cross baselines), 2 pols, 3072 x 10 kHz channels from 185 MHz, "
                       "20 x 1 ms time steps, 2048^2 FP32 grid, 0.75 arcmin pixels, uniform weighting, 10% flags; "
                       "one step = one time step = 6144 images in 4 calls of 768 channels",
           "images_per_step": C * P, "steps": steps, "images_per_s": round(value, 1),
           "ms_per_step": round(ms / steps, 3), "plan": ctx.get_plan(N, 1),
           "path_roofline": {"bytes_per_image_model": per_image,
                             "column_extent": {"mean_columns": round(ext, 1), "of": N // 2},
                             "achieved_GB_s": round(value * per_image / 1e9, 1),
                             "frac_hbm": round(value * per_image / 1e9 / HBM_PEAK_GBS, 4)},
           "kernels": kernels}
    log(f"Phase II: {value:.0f} images/s ({ms / steps:.2f} ms per time step), "
        f"{value * per_image / 1e9:.0f} GB/s on the path model (mean column extent {ext:.0f} of {N // 2})")
    del d, images, ws, wsum, nout
    torch.cuda.empty_cache()
    return out


def bench_uneven(ctx, torch, blink, synth, reps, desc_form="auto"):
    """One blink_image_batch_desc call over 4096 images of 512^2, 1024^2 and 2048^2 (70-300 MHz,
    70-100% of 8128 baselines each), FP32 and split forms, eager and replayed from a hipGraph; the
    descriptor autotuner picks the form (staged or persistent) and its plan for each."""
    import numpy as np

    lay = synth.uneven_layout()
    dev = "cuda:0"
    log(f"uneven batch: {lay['n_img']} images, {lay['images_len'] * 4 / 1e9:.1f} GB of images")
    desc = torch.from_numpy(synth.uneven_descriptors(lay, blink.DESC_DTYPE).view(np.uint8).copy()).to(dev)
    vis = synth.uneven_vis_device(lay, dev)
    uvw = torch.from_numpy(lay["uvw_ext"]).to(dev)
    images = torch.empty(lay["images_len"], dtype=torch.float32, device=dev)
    n_img = lay["n_img"]
    ws = torch.empty(blink.desc_workspace_size(n_img, lay["max_b"], lay["max_n"], 1024), dtype=torch.uint8,
                     device=dev)
    # per image: the nonzero half-spectrum columns written and read back (16 N E), the image
    # (4 N^2) and 9 B per baseline; E = 1 + the largest |ku| over the image's baselines (none is
    # flagged in this batch)
    ext = []
    for i in range(n_img):
        n, o, nb = int(lay["grid_n"][i]), int(lay["uvw_offset"][i]), int(lay["n_baselines"][i])
        k = lay["freq_hz"][i] / SPEED_OF_LIGHT * n * lay["pixel_scale"][i]
        u = np.rint(lay["uvw_ext"][o:o + nb, :2] * k)
        keep = (np.abs(u) < n / 2).all(axis=1)
        ext.append(int(np.abs(u[keep, 0]).max()) + 1 if keep.any() else 0)
    model = int(sum(16 * int(n) * e + 4 * int(n) ** 2 + 9 * int(b)
                    for n, e, b in zip(lay["grid_n"], ext, lay["n_baselines"])))
    sizes = {int(n): int((lay["grid_n"] == n).sum()) for n in sorted(set(lay["grid_n"].tolist()))}
    out = {"workload": "uneven: 4096 images, f = 70-300 MHz, N = 512 / 1024 / 2048 below 120 / 200 MHz / above, "
                       "pixel scale per channel so every baseline fits, 70-100% of 8128 baselines per image",
           "images": n_img, "images_per_size": sizes, "bytes_model_total": model,
           "column_extent_mean_fraction": round(float(np.mean([e / (n / 2) for e, n in zip(ext, lay["grid_n"])])), 3)}
    for name, prec in FORMS:
        if desc_form == "auto":
            # the descriptor autotuner picks the form (staged or persistent) and the persistent form's block
            # and workgroups
            plan, tune_ms = ctx.autotune_desc(desc, vis, uvw, None, images, lay["max_b"], lay["max_n"],
                                              precision=prec, workspace=ws)
            log(f"uneven {name}: autotuned plan {plan} ({tune_ms:.2f} ms)")
        else:
            ctx.set_desc_plan(1024 if desc_form == "persistent" and prec == 0 else 512, 0,
                              form=blink.DESC_STAGED if desc_form == "staged" else blink.DESC_PERSISTENT)
            plan = ctx.get_desc_plan()

        def run(i, prec=prec):
            ctx.blink_image_batch_desc(desc, vis, uvw, None, images, lay["max_b"], lay["max_n"], precision=prec,
                                       workspace=ws)
        ms = timed(torch, run, reps, 1) / reps
        g = ctx.graph_desc(desc, vis, uvw, None, images, lay["max_b"], lay["max_n"], precision=prec, workspace=ws)
        try:
            gms = timed(torch, lambda i: g.launch(), reps, 1) / reps
        finally:
            g.close()
        gbs = model / (ms / 1e3) / 1e9
        out[name] = {"desc_plan": plan, "images_per_s": round(n_img / (ms / 1e3), 1), "ms_per_batch": round(ms, 3),
                     "graph_images_per_s": round(n_img / (gms / 1e3), 1), "graph_ms_per_batch": round(gms, 3),
                     "model_GB_s": round(gbs, 1), "frac_hbm_model": round(gbs / HBM_PEAK_GBS, 4)}
    for name, _ in FORMS[1:]:
        out[name]["vs_fp32"] = round(out[name]["images_per_s"] / out["fp32"]["images_per_s"], 4)
    del desc, vis, uvw, images, ws
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="time steps to image (1536 images each)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the execution plan on time step 0 instead of loading the committed plan file")
    ap.add_argument("--save-plans", default="", help="write the context's plans (JSON) to this path")
    ap.add_argument("--plan", default="", help="force a plan col_strip,row_block,group[,col_loop]")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the split-precision and uneven-batch measurements beside the headline")
    ap.add_argument("--form-steps", type=int, default=20, help="steps per split-precision form measurement")
    ap.add_argument("--desc-form", choices=("auto", "staged", "persistent"), default="auto",
                    help="form of the uneven batch: auto runs the descriptor autotuner per precision (default); "
                         "staged or persistent fix the form with its default plan (for profiles)")
    ap.add_argument("--no-cache-probe", action="store_true",
                    help="skip the pass with image groups whose half spectra exceed the last-level cache (profiles "
                         "of the headline kernels use it so that every traced launch has the headline plan)")
    ap.add_argument("--forms", default="all",
                    help="comma-separated subset of the forms measured beside the headline: split, conv, "
                         "corrected, average, correlator, dedispersion, precision, uneven, phase2 (default all)")
    ap.add_argument("--only-correlator", action="store_true",
                    help="only measure the correlator form (for profiling it alone); prints its JSON")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy (read + write of this many MiB) --steps times; used "
                         "to scale the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU: every image is independent, so a multi-GPU run is this "
              f"single-GPU path on each GPU's share of time steps; --gpus {args.gpus} is not supported.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2505_15204_amd as blink
    from paper_2505_15204_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            torch.mul(src, 1.0, out=dst)       # elementwise: reads n*4 bytes, writes n*4 bytes
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                          "launches": args.steps}), flush=True)
        return
    if args.only_correlator:
        ctx = blink.Context(0)
        print(json.dumps({"form": "correlator", **bench_correlator(ctx, torch, args.steps, args.warmup)}), flush=True)
        ctx.close()
        return
    spec = synth.spec_vcs()
    T, C, P, B, N = spec.T, spec.C, spec.P, spec.B, spec.grid_n
    log(f"generating workload {spec.name}: T={T} C={C} P={P} B={B} N={N} on cuda:0")
    d = synth.make_problem_device(spec, "cuda:0")
    torch.cuda.synchronize()
    ctx = blink.Context(0)
    images = torch.empty((1, C, P, N, N), dtype=torch.float32, device="cuda:0")   # ring: one time step
    wsum = torch.empty((1, C, P), dtype=torch.float64, device="cuda:0")
    nout = torch.empty((1, C), dtype=torch.int32, device="cuda:0")
    ws = torch.empty(blink.image_batch_workspace_size(1, C, P, B, N), dtype=torch.uint8, device="cuda:0")

    def step(i):
        t = i % T
        ctx.blink_image_batch(d["vis"][t:t + 1], d["flags"][t:t + 1], d["uvw_m"][t:t + 1], d["freq_hz"], N,
                              spec.pixel_scale, 0, out=images, weight_sum=wsum, n_out=nout, workspace=ws)

    tune = None
    if args.plan:
        c, r, g, *lp = (int(x) for x in args.plan.split(","))
        ctx.set_plan(N, 0, c, r, g, col_loop=lp[0] if lp else 1)
    elif not args.autotune and os.path.exists(blink.PLANS_PATH):
        ctx.load_plans(blink.PLANS_PATH)
        tune = {"source": os.path.relpath(blink.PLANS_PATH, ROOT)}
    else:
        log("autotuning the execution plan on time step 0")
        t0 = time.perf_counter()
        plan, best_ms = ctx.autotune_image_batch(d["vis"][0:1], d["flags"][0:1], d["uvw_m"][0:1], d["freq_hz"], N,
                                                 spec.pixel_scale, 0, out=images, workspace=ws)
        tune = {"source": "autotuned", "best_step_ms": round(best_ms, 4),
                "seconds": round(time.perf_counter() - t0, 2)}
        log(f"plan {plan}: {best_ms:.3f} ms per step")
    if args.save_plans:
        ctx.save_plans(args.save_plans)
    plan = ctx.get_plan(N, 0)
    log(f"warmup {args.warmup} steps, timing {args.steps} steps")
    w0 = time.perf_counter()
    gpu_ms = timed(torch, step, args.steps, args.warmup)
    wall = time.perf_counter() - w0
    n_images = args.steps * C * P
    value = n_images / (gpu_ms / 1e3)
    log(f"{n_images} images in {gpu_ms:.1f} ms (wall {wall * 1e3:.1f} ms): {value:.0f} images/s")

    # Per-kernel durations: the same steps again with hipEvents around every launch (the events
    # cost a little time per launch, so they are kept out of the headline pass).
    log(f"kernel timing pass: {args.steps} steps with per-launch events")
    prof, prof_ms = profiled(ctx, torch, step, args.steps)
    units = {"image": n_images, "pair": args.steps * C}
    ext = column_extent(torch, d, spec, args.steps)
    ub = kernel_unit_bytes(spec, ext)
    kernels = kernel_table(prof, units, ub)
    dom = max((k for k in kernels if k in ub), key=lambda k: kernels[k]["total_ms"])
    roof = {"kernel": dom, "bound": "hbm", "achieved": kernels[dom]["achieved_GB_s"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": kernels[dom]["frac_hbm"],
            "traffic": counter_traffic("vcs1024_fp32", dom, plan)}
    # The half spectra of one image group (group x 4 N^2 bytes) are written by the column launch and
    # read by the row launch; when they fit the 256 MB last-level cache they are served from it, and
    # the byte counters (which sit above that cache) count those hits as HBM traffic. The same steps
    # with a group whose half spectra exceed the cache give the kernels' rates from DRAM.
    h_image = 8 * N * ext           # the half-spectrum columns one image writes and reads back (mean)
    h_group = plan["group"] * h_image
    big = 0 if args.no_cache_probe else max(plan["group"], 1)
    while big and big * h_image <= 1.5 * MALL_BYTES:
        big += max(plan["group"], 1)
    if big:
        ctx.set_plan(N, 0, plan["col_strip"], plan["row_block"], big, col_loop=plan["col_loop"])
        bprof, bms = profiled(ctx, torch, step, min(args.steps, 10))
        ctx.set_plan(N, 0, plan["col_strip"], plan["row_block"], plan["group"], col_loop=plan["col_loop"])
        bk = kernel_table(bprof, {"image": min(args.steps, 10) * C * P, "pair": min(args.steps, 10) * C},
                          kernel_unit_bytes(spec, column_extent(torch, d, spec, min(args.steps, 10))))
    else:
        bk, bms = {}, float("nan")
    roof["last_level_cache"] = {
        "note": f"a group's half spectra ({plan['group']} images x {h_image / 2**20:.2f} MiB of nonzero columns = "
                f"{h_group / 2**20:.0f} MiB) fit the {MALL_BYTES // 10**6} MB Infinity Cache between the column and "
                f"the row launch; the byte counters count its hits, so this fraction includes reads served from "
                f"that cache",
        "group_beyond_cache": big,
        "half_spectra_MiB": round(big * h_image / 2**20),
        "frac_hbm": {k: bk[k]["frac_hbm"] for k in ("grid_colfft", "row_fft") if k in bk},
        "images_per_s": round(min(args.steps, 10) * C * P / (bms / 1e3), 1) if big else None}
    log(f"groups of {big} (half spectra beyond the cache): row kernel at "
        f"{bk.get('row_fft', {}).get('frac_hbm', 0):.3f} of HBM, column kernel at "
        f"{bk.get('grid_colfft', {}).get('frac_hbm', 0):.3f}")
    per_image = path_bytes_per_image(spec, ext)
    path = {"bytes_per_image_model": per_image,
            "column_extent": {"mean_columns": round(ext, 1), "of": N // 2},
            "achieved_GB_s": round(value * per_image / 1e9, 1),
            "frac_hbm": round(value * per_image / 1e9 / HBM_PEAK_GBS, 4),
            "kernel_timing_pass_ms": round(prof_ms, 3)}

    forms = None
    precision_samples = None
    known = ("split", "conv", "corrected", "average", "correlator", "dedispersion", "precision", "uneven", "phase2")
    want = set(known) if args.forms == "all" else {f.strip() for f in args.forms.split(",") if f.strip()}
    if want - set(known):
        print(f"unknown forms {sorted(want - set(known))}; known: {', '.join(known)}", file=sys.stderr)
        sys.exit(2)
    if not args.no_forms:
        forms = {"vcs-1024": {"fp32": {"images_per_s": round(value, 1)}}}
        fs = min(args.form_steps, T)
        if "split" in want:
            # The split-precision matrix-core forms on the same workload and buffers (MFMA vs FP32).
            for name, prec in FORMS[1:]:
                def fstep(i, prec=prec):
                    t = i % T
                    ctx.blink_image_batch(d["vis"][t:t + 1], d["flags"][t:t + 1], d["uvw_m"][t:t + 1], d["freq_hz"], N,
                                          spec.pixel_scale, 0, precision=prec, out=images, weight_sum=wsum, n_out=nout,
                                          workspace=ws)
                ms = timed(torch, fstep, fs, 2)
                fprof, _ = profiled(ctx, torch, fstep, fs)
                fk = kernel_table(fprof, {"image": fs * C * P, "pair": fs * C},
                                  kernel_unit_bytes(spec, column_extent(torch, d, spec, fs)))
                v = fs * C * P / (ms / 1e3)
                forms["vcs-1024"][name] = {"images_per_s": round(v, 1), "vs_fp32": round(v / value, 4),
                                           "plan": ctx.get_plan(N, 0, prec),
                                           "kernels": {k: fk[k] for k in ("grid_colfft", "row_fft") if k in fk}}
                log(f"{name}: {v:.0f} images/s ({v / value:.3f} x FP32)")
        if "conv" in want:
            # Convolutional gridding (W = 8, beta = 18.4) on the same workload, FP32.
            cws = torch.empty(blink.image_batch_conv_workspace_size(1, C, P, B, N, 8), dtype=torch.uint8, device="cuda:0")

            def cstep(i):
                t = i % T
                ctx.blink_image_batch_conv(d["vis"][t:t + 1], d["flags"][t:t + 1], d["uvw_m"][t:t + 1], d["freq_hz"], N,
                                           spec.pixel_scale, 8, 18.4, out=images, weight_sum=wsum, n_out=nout,
                                           workspace=cws)
            ms = timed(torch, cstep, fs, 2)
            cprof, _ = profiled(ctx, torch, cstep, fs)
            # byte model from the workload's records and its column extent (the last tap column)
            cbytes, cext = conv_unit_bytes(torch, d, spec, 8, fs)
            ck = kernel_table(cprof, {"image": fs * C * P, "pair": fs * C}, cbytes)
            v = fs * C * P / (ms / 1e3)
            forms["vcs-1024"]["conv_w8_fp32"] = {"images_per_s": round(v, 1), "vs_fp32": round(v / value, 4),
                                                 "kernel": "exponential of semicircle, W = 8, beta = 18.4",
                                                 "column_extent": {"mean_columns": round(cext, 1), "of": N // 2},
                                                 "kernels": {k: ck[k] for k in ("bin", "grid_colfft", "row_fft") if k in ck}}
            log(f"conv W=8: {v:.0f} images/s ({v / value:.3f} x nearest-cell FP32)")
            del cws
        if "corrected" in want:
            # Pre-gridding corrections (per-antenna solutions + phase-centre rotation) on the same workload.
            gen = torch.Generator(device="cuda:0")
            gen.manual_seed(20)
            amp = 0.5 + torch.rand((C, P, spec.n_tiles), generator=gen, device="cuda:0", dtype=torch.float64)
            pha = 2 * torch.pi * torch.rand((C, P, spec.n_tiles), generator=gen, device="cuda:0", dtype=torch.float64)
            gains = torch.polar(amp, pha).to(torch.complex64)
            xws = torch.empty(blink.image_batch_corrected_workspace_size(1, C, P, B, N), dtype=torch.uint8,
                              device="cuda:0")

            def xstep(i):
                t = i % T
                ctx.blink_image_batch_corrected(d["vis"][t:t + 1], d["flags"][t:t + 1], d["uvw_m"][t:t + 1],
                                                d["freq_hz"], N, spec.pixel_scale, 0, gains=gains, l0=0.02, m0=-0.015,
                                                out=images, weight_sum=wsum, n_out=nout, workspace=xws)
            ms = timed(torch, xstep, fs, 2)
            xprof, _ = profiled(ctx, torch, xstep, fs)
            xub = dict(kernel_unit_bytes(spec, column_extent(torch, d, spec, fs)),
                       correct=("pair", P * B * 16 + 24 * B // C + P * spec.n_tiles * 8))
            xk = kernel_table(xprof, {"image": fs * C * P, "pair": fs * C}, xub)
            v = fs * C * P / (ms / 1e3)
            forms["vcs-1024"]["corrected_fp32"] = {
                "images_per_s": round(v, 1), "vs_fp32": round(v / value, 4),
                "corrections": "per-antenna complex solutions [C][P][128] and phase-centre rotation (l0, m0) = "
                               "(0.02, -0.015) with the w term",
                "kernels": {k: xk[k] for k in ("correct", "grid_colfft", "row_fft") if k in xk}}
            log(f"corrected: {v:.0f} images/s ({v / value:.3f} x FP32)")
            del xws, gains
        if "average" in want:
            # Stokes I + band average of one time step's images (1536 images -> 1), HBM-bound.
            avg_out = torch.empty((1, 1, 1, N, N), dtype=torch.float32, device="cuda:0")
            ms = timed(torch, lambda i: ctx.blink_image_average(images, blink.AVG_CHANNEL | blink.AVG_POL, out=avg_out),
                       10, 2) / 10
            moved = (C * P + 1) * 4 * N * N
            forms["vcs-1024"]["stokes_i_band_average"] = {
                "images_in": C * P, "ms": round(ms, 4), "bytes": moved,
                "achieved_GB_s": round(moved / (ms / 1e3) / 1e9, 1),
                "frac_hbm": round(moved / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
            log(f"Stokes I + band average of {C * P} images: {ms:.3f} ms "
                f"({moved / (ms / 1e3) / 1e9:.0f} GB/s)")
        if "correlator" in want:
            forms["correlator"] = bench_correlator(ctx, torch, 5, 2)
        if "dedispersion" in want:
            forms["dedispersion"] = bench_dedispersion(ctx, torch, blink, 3, 1)
        if "precision" in want:
            forms["precision-4096"], precision_samples = bench_precision_workload(ctx, torch, blink, synth, 3, 1)
        if "uneven" in want:
            forms["uneven"] = bench_uneven(ctx, torch, blink, synth, 3, args.desc_form)
        if "phase2" in want:
            forms["phase2-2048"] = bench_phase2(ctx, torch, blink, synth, 2, 1)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        cpu = cpu_baseline(d, spec, args.cpu_seconds)
        log(f"CPU oracle: {cpu['value']} images/s on {cpu['cores']} threads")
        if precision_samples is not None:
            # the oracle on the sampled 4096^2 images: per-image errors of every FFT form
            log("FP64 oracle on the sampled 4096^2 precision images")
            forms["precision-4096"]["errors_vs_fp64_oracle"] = precision_errors(precision_samples)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(gpu_ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": "vcs-1024: 128 tiles (8128 cross baselines), 2 pols, 768 x 40 kHz channels from "
                        "139 MHz, 100 x 1 ms time steps, 1024^2 FP32 grid, 1 arcmin pixels, natural weighting, "
                        "50 point sources + noise, 10% flags; one step = one time step = 1536 images",
            "images_per_step": C * P,
            "grid_n": N,
            "baselines": B,
            "path": "fp32: bin -> fused grid+column FFT -> weights -> row FFT (C2R)",
            "plan": plan,
            "autotune": tune,
        },
        "roofline": roof,
        "path_roofline": path,
        "kernels": kernels,
        "wall_s": round(wall, 4),
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
