"""Benchmark: wavelength-summed FFT-ASM PSF at a 65536^2 padded grid.

One step = the whole PSF of the large workload (32768^2 DOE, 31 wavelengths,
padded to 65536^2): per wavelength the five HIP passes (phase + FFT digit
passes, transfer-function pass, inverse passes + |U|^2 accumulation).
Inputs are synthetic and resident in HBM before timing starts.

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FFT-ASM PSF Mpix*lambda/s at 65536^2 (padded pixels x wavelengths per second)"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pass_bytes(n, m, k_first, amp=False):
    """Algorithmic HBM bytes of each pass for one wavelength (crop output).

    A : read h (and amp) N^2, write N rows of the M x M c64 field
    B : read N rows, write M rows
    C : read + write M rows
    B': read M rows, write N rows
    A': read N rows, read-modify-write the N^2 fp32 PSF (write only for k=0)
    """
    f = 8.0 * n * m  # N rows of c64
    full = 8.0 * m * m
    nn = float(n) * n
    return {
        "pass_a_fwd": nn * 4 * (2 if amp else 1) + f,
        "pass_b_fwd": f + full,
        "pass_c": 2 * full,
        "pass_b_inv": full + f,
        "pass_a_inv": f + nn * 4 * (1 if k_first else 2),
    }


def cpu_baseline(h, p):
    """The FP64 oracle on a bounded sample: the central 8192^2 window of the
    same height map (same pitch, distance and 550 nm-class wavelength),
    padded 2x to 16384^2, one wavelength."""
    import oracle
    from oracle import asm
    n_s = 8192
    m_s = 2 * n_s
    c = (h.shape[0] - n_s) // 2
    hs = np.array(h[c:c + n_s, c:c + n_s], dtype=np.float32)
    k = 15  # 550 nm
    t0 = time.perf_counter()
    oracle.psf(hs, p["dx"], p["z"], m_s, [p["lams"][k]], [p["n_index"][k]])
    dt = time.perf_counter() - t0
    return {
        "value": round(m_s * m_s * 1 / dt / 1e6, 3),
        "unit": "Mpix*lambda/s",
        "cores": int(asm.WORKERS),
        "kind": "oracle",
        "sample": (f"central {n_s}^2 window of the large workload's height map, padded to "
                   f"{m_s}^2, one wavelength ({p['lams'][k]:.2f} um), FP64 NumPy/SciPy oracle, "
                   f"{dt:.1f} s"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="large", choices=["large", "mid", "small"])
    ap.add_argument("--lambdas", type=int, default=0,
                    help="profiling runs only: keep the first K wavelengths")
    ap.add_argument("--calib-copy", action="store_true",
                    help="profiling runs only: first run a plain 4 GiB device copy, the "
                         "reference for HBM byte counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the path shards by wavelength across GPUs, but this "
              "build runs and reports a single MI355X only (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2505_22313_amd import api
    from paper_2505_22313_amd import workloads as wl

    p = wl.problem(args.workload)
    if args.lambdas:
        for key in ("lams", "n_index", "weights"):
            p[key] = p[key][:args.lambdas]
    n, m, k = p["n"], p["m"], len(p["lams"])
    log(f"workload {args.workload}: N={n} M={m} K={k}; generating heights on the host")
    t0 = time.time()
    h = wl.heights(args.workload)
    log(f"heights ready in {time.time() - t0:.1f} s")

    torch.cuda.set_device(0)
    if args.calib_copy:
        src = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 4 GiB read + 4 GiB written")
        del src, dst
    ctx = api.default_context(0)
    prob = api.Problem.from_dict(p)
    hd = torch.from_numpy(h).cuda()
    psf = torch.empty((n, n), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    log("inputs resident on the GPU; warming up")

    for i in range(args.warmup):
        api.psf(hd, prob, out=psf, ctx=ctx)
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")

    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        api.psf(hd, prob, out=psf, ctx=ctx)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    log(f"timed {args.steps} steps in {t1 - t0:.3f} s")

    dt = (t1 - t0) / args.steps
    value = k * float(m) * m / dt / 1e6

    # per-pass averages and the roofline of the dominant pass
    per_lambda = pass_bytes(n, m, k_first=False)
    first = pass_bytes(n, m, k_first=True)
    passes = {}
    for name, (cnt, tot) in prof.items():
        avg_ms = tot / max(cnt, 1)
        # average algorithmic bytes per launch (first wavelength writes the PSF once)
        b = (first[name] + (k - 1) * per_lambda[name]) / k
        passes[name] = {"launches": int(cnt), "avg_ms": round(avg_ms, 4),
                        "alg_bytes": b, "alg_gbs": round(b / (avg_ms * 1e-3) / 1e9, 1)}
    dom = max(passes, key=lambda x: passes[x]["avg_ms"])
    dp = passes[dom]
    achieved = dp["alg_gbs"]
    step_bytes = sum(first.values()) + (k - 1) * sum(per_lambda.values())
    torch.cuda.synchronize()
    sumv = float(psf.double().sum().item())

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mpix*lambda/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": {
                "large": "large-area DOE: 32768^2 heights (0.5 um pitch), 16-level Fresnel lens "
                         "f=50 mm + smooth noise, 31 wavelengths 400-700 nm, z=50 mm, padded "
                         "to 65536^2, wavelength-summed PSF on the 32768^2 window",
                "mid": "8192^2 lens + noise, 3 wavelengths, padded to 16384^2",
                "small": "512^2 uniform heights, 550 nm, padded to 1024^2",
            }[args.workload],
            "n": n, "m": m, "n_lambda": k, "dx_um": p["dx"], "z_um": p["z"],
        },
        "hbm_gbs_alg": round(step_bytes / dt / 1e9, 1),
        "alg_bytes_per_padded_pixel_lambda": round(step_bytes / (k * float(m) * m), 2),
        "passes": {kk: {"avg_ms": v["avg_ms"], "alg_gbs": v["alg_gbs"]} for kk, v in passes.items()},
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
        },
        "psf_sum": sumv,
    }
    if not args.no_cpu_baseline and args.workload == "large":
        log("timing the CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(h, p)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
