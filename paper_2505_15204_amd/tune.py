"""Autotune the execution plans of blink_image_batch on this GPU and write them to a plan file.

For every grid size, weighting and precision form asked for, one time step of a synthetic
MWA-shaped workload of that size is imaged with every compiled (strip width, row block) pair and
image-group size (blink_autotune_image_batch); the fastest plan is kept. The result is a JSON file
that Context.load_plans reads (by default the package's plans_gfx950.json, which bench.py loads).

    python -m paper_2505_15204_amd.tune [--sizes 256,512,1024,2048,4096] [--precisions 0,1,2]
                                        [--weightings 0,1] [--out FILE]
"""
from __future__ import annotations

import argparse
import sys


def workload(synth, N: int):
    """One time step of a synthetic workload of grid size N (inputs generated on the GPU)."""
    if N == 1024:
        return synth.spec_vcs(T=1)
    if N == 2048:
        return synth.spec_phase2(T=1, C=256)
    if N == 4096:
        return synth.spec_precision(T=1)
    # other sizes: the VCS channels with the pixel scaled so the field of view matches 1024 x 1 arcmin
    return synth.Spec(f"tune-{N}", 2, 128, 1, 2, synth.vcs_channels()[:768], N, synth.ARCMIN * 1024 / N, 50, 0.10)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--sizes", default="256,512,1024,2048,4096")
    ap.add_argument("--precisions", default="0,1,2")
    ap.add_argument("--weightings", default="0,1")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)

    import torch

    import paper_2505_15204_amd as blink
    from paper_2505_15204_amd import synth

    if not torch.cuda.is_available():
        print("tune needs a GPU", file=sys.stderr)
        return 1
    out = args.out or blink.PLANS_PATH
    ctx = blink.Context(0)
    try:
        ctx.load_plans(out)
    except FileNotFoundError:
        pass
    for N in (int(x) for x in args.sizes.split(",")):
        spec = workload(synth, N)
        d = synth.make_problem_device(spec, "cuda:0")
        for w in (int(x) for x in args.weightings.split(",")):
            for p in (int(x) for x in args.precisions.split(",")):
                plan, ms = ctx.autotune_image_batch(d["vis"], d["flags"], d["uvw_m"], d["freq_hz"], N,
                                                    spec.pixel_scale, w, precision=p)
                print(f"[tune] N={N} weighting={w} precision={p}: {plan} {ms:.3f} ms for {spec.n_images} images",
                      flush=True)
        del d
        torch.cuda.empty_cache()
    ctx.save_plans(out)
    print(f"[tune] wrote {out}", flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
