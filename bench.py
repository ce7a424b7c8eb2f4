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
    """Algorithmic HBM bytes of each pass for one wavelength (crop output);
    n and m are ints (square) or (rows, columns).

    A : read h (and amp) N^2, write N rows of the M x M c64 field
    B : read N rows, write M rows
    C : read + write M rows
    B': read M rows, write N rows
    A': read N rows, read-modify-write the N^2 fp32 PSF (write only for k=0)
    """
    ny, nx = (n, n) if np.ndim(n) == 0 else n
    my, mx = (m, m) if np.ndim(m) == 0 else m
    f = 8.0 * ny * mx  # Ny rows of c64
    full = 8.0 * my * mx
    nn = float(ny) * nx
    return {
        "pass_a_fwd": nn * 4 * (2 if amp else 1) + f,
        "pass_b_fwd": f + full,
        "pass_c": 2 * full,
        "pass_b_inv": full + f,
        "pass_a_inv": f + nn * 4 * (1 if k_first else 2),
    }


def step_pass_bytes(n, m, k, groups, amp=False):
    """Algorithmic bytes of each pass over one call of k wavelengths run in
    `groups` groups (dop_psf with a workspace of several fields): pass A
    reads h once per group and pass A' read-modify-writes the PSF once per
    group (the first group only writes it); B, C and B' move their bytes per
    wavelength.  groups = k is the one-wavelength-at-a-time call."""
    ny, nx = (n, n) if np.ndim(n) == 0 else n
    one = pass_bytes(n, m, k_first=False, amp=amp)
    f = 8.0 * ny * pass_cols(m)
    hb = 4.0 * ny * nx * (2 if amp else 1)
    psf = 4.0 * ny * nx
    tot = {name: k * one[name] for name in ("pass_b_fwd", "pass_c", "pass_b_inv")}
    tot["pass_a_fwd"] = k * f + groups * hb
    tot["pass_a_inv"] = k * f + psf + (groups - 1) * 2 * psf
    return tot


def pass_cols(m):
    return m if np.ndim(m) == 0 else m[1]


def pass_rates(prof, n, m, k):
    """Per-pass average launch time, algorithmic bytes per launch and GB/s
    from a profile of whole PSF calls ({name: (launches, total ms)}); the
    group count per call follows from the launch counts of passes A and C."""
    calls = prof["pass_c"][0] / k
    groups = max(1, round(prof["pass_a_fwd"][0] / calls))
    tot = step_pass_bytes(n, m, k, groups)
    res = {}
    for name, (cnt, ms) in prof.items():
        b = tot[name] * calls / max(cnt, 1)
        res[name] = {"launches": int(cnt), "avg_ms": round(ms / max(cnt, 1), 4), "alg_bytes": b,
                     "alg_gbs": round(tot[name] * calls / (ms * 1e-3) / 1e9, 1)}
    return res, groups, tot


def cpu_baseline(h, p):
    """The FP64 oracle on a bounded sample: the central 8192^2 window of the
    same height map (same pitch and distance), padded 2x to 16384^2, two of
    the workload's wavelengths (about 15 s on 16 cores)."""
    import oracle
    from oracle import asm
    n_s = 8192
    m_s = 2 * n_s
    c = (h.shape[0] - n_s) // 2
    hs = np.array(h[c:c + n_s, c:c + n_s], dtype=np.float32)
    ks = [10, 20]  # 500 and 600 nm
    t0 = time.perf_counter()
    oracle.psf(hs, p["dx"], p["z"], m_s, [p["lams"][k] for k in ks], [p["n_index"][k] for k in ks])
    dt = time.perf_counter() - t0
    lam_text = ", ".join("%.2f" % p["lams"][k] for k in ks)
    return {
        "value": round(m_s * m_s * len(ks) / dt / 1e6, 3),
        "unit": "Mpix*lambda/s",
        "cores": int(asm.WORKERS),
        "kind": "oracle",
        "sample": (f"central {n_s}^2 window of the large workload's height map, padded to "
                   f"{m_s}^2, {len(ks)} wavelengths ({lam_text} um), FP64 NumPy/SciPy oracle, "
                   f"{dt:.1f} s"),
    }


def measured_traffic(kernel, m):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated against a plain copy), or
    None if it was measured on another version of the kernels or grid."""
    from paper_2505_22313_amd import profiling
    path = os.path.join(ROOT, "profiles", "traffic_large_65536.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha") != profiling.kernel_source_hash() or rec.get("m") != m:
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else round(k["traffic_bytes"])


def _pct(v, q):
    v = sorted(v)
    pos = q * (len(v) - 1)
    i = int(pos)
    f = pos - i
    return v[i] * (1 - f) + v[min(i + 1, len(v) - 1)] * f


def serve_measure(api, wl, torch, count, rate_hz, pool, slots=4, seed=5,
                  policies=("chunked", "fifo")):
    """Replay a Poisson trace of PSF requests on the same GPU: one request at
    a time on one stream (the plain path, dop_psf with wavelength groups),
    then through the continuous-batching server under each policy (`slots`
    admitted requests, an arena of 2 * slots of the largest one-field
    workspaces).  Latency = completion - arrival.  The timing does not read
    the results (the serve tests check them), so outputs are reused round-robin
    once a size has more than kOutPerSize requests: a 2000-request trace would
    otherwise need about 700 GB of PSF buffers."""
    import threading
    kOutPerSize = 16
    trace = wl.serve_trace(count, rate_hz, seed=seed, sizes=tuple(sorted(pool)))
    reqs = []
    for r in trace:
        prob = api.Problem(r["n"], r["m"], r["dx"], r["z"], r["lams"], r["n_index"])
        reqs.append((r["t"], prob, pool[r["n"]][r["pool"]]))
    bufs, outs = {}, []
    for _, p, _ in reqs:
        ring = bufs.setdefault(p.n, [])
        if len(ring) < kOutPerSize:
            ring.append(torch.empty((p.n, p.n), dtype=torch.float32, device="cuda"))
            outs.append(ring[-1])
        else:
            outs.append(ring[len(outs) % kOutPerSize])
    work = sum(p.k * float(p.m) ** 2 for _, p, _ in reqs) / 1e6
    torch.cuda.synchronize()

    # one request at a time, in arrival order
    lat_seq = []
    t0 = time.perf_counter()
    for i, ((ta, prob, h), o) in enumerate(zip(reqs, outs)):
        now = time.perf_counter() - t0
        if now < ta:
            time.sleep(ta - now)
        api.psf(h, prob, out=o)
        torch.cuda.synchronize()
        lat_seq.append((time.perf_counter() - t0 - ta) * 1e3)
        if (i + 1) % 250 == 0:
            log(f"serving: one at a time, {i + 1} of {count} requests")
    span_seq = time.perf_counter() - t0
    api.default_context().release_workspaces()
    torch.cuda.empty_cache()

    # continuous batching, under each policy
    big = max(api.workspace_size(p) for _, p, _ in reqs)

    def served(spec):
        # "chunked" or "chunked:<age bound s>", "fifo", "size_aware"
        policy, _, arg = spec.partition(":")
        kw = {"age_bound_s": float(arg)} if arg else {}
        srv = api.Server(2 * slots * big, max_slots=slots, policy=policy, **kw)
        tickets = [None] * len(reqs)
        t0 = time.perf_counter()

        def submitter():
            for i, ((ta, prob, h), o) in enumerate(zip(reqs, outs)):
                now = time.perf_counter() - t0
                if now < ta:
                    time.sleep(ta - now)
                tickets[i] = srv.submit(prob, h, o)
                if (i + 1) % 250 == 0:
                    log(f"serving: {spec}, {i + 1} of {count} requests submitted")

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        for t in tickets:
            srv.wait(t, 600.0)
        span = time.perf_counter() - t0
        lat = [srv.latency_ms(t) for t in tickets]
        peak = srv.stats()["arena_peak"]
        srv.close()
        return {"p50_ms": round(_pct(lat, 0.5), 2), "p99_ms": round(_pct(lat, 0.99), 2),
                "throughput_req_s": round(count / span, 2),
                "mpix_lambda_s": round(work / span, 1), "arena_peak_gb": round(peak / 1e9, 2)}

    res = {pol: served(pol) for pol in policies}
    del outs, bufs
    torch.cuda.synchronize()
    return {
        "requests": count, "offered_rate_hz": round(rate_hz, 2), "slots": slots,
        "mpix_lambda": round(work, 1),
        "served": res[policies[0]],
        "policy": policies[0],
        **{f"served_{pol}": res[pol] for pol in policies[1:]},
        "sequential": {"p50_ms": round(_pct(lat_seq, 0.5), 2),
                       "p99_ms": round(_pct(lat_seq, 0.99), 2),
                       "throughput_req_s": round(count / span_seq, 2),
                       "mpix_lambda_s": round(work / span_seq, 1)},
    }


def design_measure(api, wl, torch, steps=200):
    """The design workload: 8192^2 heights, 3 wavelengths, padded to 16384^2,
    L2 loss to a Gaussian target, `steps` Adam steps with cosine decay."""
    from paper_2505_22313_amd.design import design_loop
    p = wl.problem("design")
    n = p["n"]
    h = torch.from_numpy(wl.heights("design")).cuda()
    t = torch.from_numpy(wl.gaussian_target(n, 3.0, total=3.0 * n * n)).cuda()
    prob = api.Problem.from_dict(p)
    design_loop(h, prob, t, steps=3)  # warm-up
    _, losses, dt = design_loop(h, prob, t, steps=steps)
    return {"workload": "8192^2 heights, 3 wavelengths, z=20 mm, padded to 16384^2, "
                        "Gaussian target sigma=3 px", "steps": steps,
            "ms_per_step": round(dt * 1e3, 2), "loss_first": losses[0], "loss_last": losses[-1]}


def paper_table2_measure(api, wl, torch):
    """Design iterations on two of the paper's own Table 2 problems, on one
    GPU: forward PSF, L2 loss, hand-written adjoint and an Adam step on a
    coarse 2 um design upsampled by nearest neighbour inside the first pass.
    The paper's wall-clock per iteration (its Table 2 time divided by its
    iteration count, on A100s with its own loss and, for imaging, a radially
    symmetric parameterisation) is quoted beside each for context."""
    from paper_2505_22313_amd.design import design_loop
    cases = [
        # 3.6 mm CHD DOE, 2 um features at 8x (0.25 um), 28800^2 grid, 520.6 nm, z = 1 cm
        dict(name="chd_conventional_8x_upsampling", nc=1800, s=8, dx=0.25, m=28800,
             lams=[0.5206], z=10000.0, steps=20,
             paper="14 min / 3000 iterations = 0.28 s per iteration on 1x A100 80 GB"),
        # 10 mm imaging DOE, 2 um features at 4x (0.5 um), 6 wavelengths, 40000^2 grid, f/8
        dict(name="imaging_conventional_4x_upsampling", nc=5000, s=4, dx=0.5, m=40000,
             lams=list(np.linspace(0.4, 0.7, 6)), z=80000.0, steps=6,
             paper="9 h / 20000 iterations = 1.62 s per iteration on 12x A100 80 GB (mesh [6, 2])"),
        # 32.16 x 21.44 mm large-area CHD, 2 um features at 4x (0.5 um), 128640 x 85760 grid,
        # z = 6 cm (the paper's hologram wavelength is not stated for it; 520.6 nm here)
        dict(name="large_area_chd_conventional_4x_upsampling", nc=(16080, 10720), s=4, dx=0.5,
             m=(128640, 85760), lams=[0.5206], z=60000.0, steps=3,
             paper="13 h / 3000 iterations = 15.6 s per iteration on 16x A100 80 GB (mesh [1, 16])"),
    ]
    res = {}
    for c in cases:
        ncy, ncx = (c["nc"], c["nc"]) if np.ndim(c["nc"]) == 0 else c["nc"]
        my, mx = (c["m"], c["m"]) if np.ndim(c["m"]) == 0 else c["m"]
        ny, nx = ncy * c["s"], ncx * c["s"]
        lams = np.asarray(c["lams"])
        log(f"paper design {c['name']}")
        prob = api.Problem((ny, nx), (my, mx), c["dx"], c["z"], lams, wl.cauchy_index(lams),
                           upsample=c["s"])
        h0 = torch.from_numpy(wl.uniform_heights((ncy, ncx), seed=ncy)).cuda()
        target = torch.from_numpy(wl.gaussian_target((ny, nx), 50.0,
                                                     total=len(lams) * float(ny) * nx)).cuda()
        design_loop(h0, prob, target, steps=2)  # warm-up
        _, losses, dt = design_loop(h0, prob, target, steps=c["steps"])
        res[c["name"]] = {"design": f"{ncy}x{ncx} at 2 um, nearest x{c['s']} -> {ny}x{nx}, "
                                    f"grid {my}x{mx}, {len(lams)} wavelength(s)",
                          "s_per_iteration": round(dt, 4), "steps": c["steps"],
                          "loss_first": losses[0], "loss_last": losses[-1],
                          "paper": c["paper"]}
        del h0, target
        api.default_context(0).release_workspaces()
        torch.cuda.empty_cache()
    return res


def _event_ms(torch, fn, reps):
    """Average ms of fn() over reps runs, timed with HIP events on the current stream."""
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def copy_ceiling_gbs(torch, nbytes=1 << 32):
    """Device-to-device copy rate (read + write bytes per second), the
    practical ceiling of a read+write pass on this GPU."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    ms = _event_ms(torch, lambda: dst.copy_(src), 5)
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def ceilings_measure(api, torch, ws, m, stream_bytes=16 << 30):
    """Measured HBM ceilings (dop_probe_bandwidth) on the workspace memory
    itself: 16-byte non-temporal stream kernels over 16 GiB (read, write,
    copy, in-place read+write) and pass C's access pattern without its
    arithmetic on the m x m field.  GB/s of bytes moved, HIP-event timed."""
    out = {}
    for kind in ("read", "write", "copy", "inplace"):
        moved = api.probe_bandwidth(kind, ws, stream_bytes)
        ms = _event_ms(torch, lambda: api.probe_bandwidth(kind, ws, stream_bytes), 5)
        out[kind] = round(moved / (ms * 1e-3) / 1e9, 1)
    if m >= 16384 and m & (m - 1) == 0:
        moved = api.probe_bandwidth("passc", ws, m=m)
        ms = _event_ms(torch, lambda: api.probe_bandwidth("passc", ws, m=m), 5)
        out["passc_pattern"] = round(moved / (ms * 1e-3) / 1e9, 1)
        out["passc_pattern_ms"] = round(ms, 3)
    return out


def other_workloads_measure(api, wl, torch, ctx):
    """The small (512^2 -> 1024^2, 1 wavelength, launch-bound) and mid
    (8192^2 -> 16384^2, 3 wavelengths) workloads: time per PSF call."""
    res = {}
    for name, reps in (("small", 200), ("mid", 5)):
        q = wl.problem(name)
        prob = api.Problem.from_dict(q)
        h = torch.from_numpy(wl.heights(name)).cuda()
        out = torch.empty((q["n"], q["n"]), dtype=torch.float32, device="cuda")
        ms = _event_ms(torch, lambda: api.psf(h, prob, out=out, ctx=ctx), reps)
        k = len(q["lams"])
        step = sum(step_pass_bytes(q["n"], q["m"], k, -(-k // min(4, k))).values())
        res[name] = {"n": q["n"], "m": q["m"], "n_lambda": k, "us_per_call": round(ms * 1e3, 1),
                     "value": round(k * float(q["m"]) ** 2 / (ms * 1e-3) / 1e6, 1),
                     "alg_gbs": round(step / (ms * 1e-3) / 1e9, 1)}
        if name == "small":
            # the same call captured once into a HIP graph and replayed
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                api.psf(h, prob, out=out, ctx=ctx)
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                api.psf(h, prob, out=out, ctx=ctx)
            gms = _event_ms(torch, graph.replay, reps)
            res[name]["us_per_graph_replay"] = round(gms * 1e3, 1)
            del graph
        del h, out
        ctx.release_workspaces()
        torch.cuda.empty_cache()
    return res


def variants_measure(api, wl, torch, p, hd, ctx, base_ms):
    """The NEXT-row options on the same workload: nearest 8x upsampling fused
    into pass A (a 4096^2 design on the 32768^2 grid), band-limited ASM, and
    the standalone Lanczos-3 upsampling kernel and its adjoint."""
    n, k = p["n"], len(p["lams"])
    s = 8
    hc = hd[::s, ::s].contiguous()
    out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    res = {}
    pu = api.Problem(n, p["m"], p["dx"], p["z"], p["lams"], p["n_index"], p.get("weights"),
                     upsample=s)
    ctx.profile_enable(True)
    ms = _event_ms(torch, lambda: api.psf(hc, pu, out=out, ctx=ctx), 1)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    res["upsample_nearest_fused"] = {
        "factor": s, "design": f"{n // s}^2 -> {n}^2", "ms_per_step": round(ms, 2),
        "vs_plain_step": round(ms / base_ms, 4),
        "pass_a_fwd_avg_ms": round(prof["pass_a_fwd"][1] / max(prof["pass_a_fwd"][0], 1), 4)}
    pb = api.Problem(n, p["m"], p["dx"], p["z"], p["lams"], p["n_index"], p.get("weights"),
                     bandlimit=True)
    ctx.profile_enable(True)
    ms = _event_ms(torch, lambda: api.psf(hd, pb, out=out, ctx=ctx), 1)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    res["bandlimit"] = {"ms_per_step": round(ms, 2), "vs_plain_step": round(ms / base_ms, 4),
                        "pass_c_avg_ms": round(prof["pass_c"][1] / max(prof["pass_c"][0], 1), 4)}
    del out
    fine = torch.empty((n, n), dtype=torch.float32, device="cuda")
    ms_up = _event_ms(torch, lambda: api.upsample(hc, s, "lanczos3", ctx=ctx, out=fine), 3)
    gc = torch.empty_like(hc)
    ms_adj = _event_ms(torch, lambda: api.upsample_adjoint(fine, s, "lanczos3", ctx=ctx, out=gc), 3)
    nbytes = 4.0 * (n * n + (n // s) ** 2)
    res["lanczos3_kernels"] = {
        "factor": s, "design": f"{n // s}^2 -> {n}^2",
        "upsample_ms": round(ms_up, 3), "upsample_alg_gbs": round(nbytes / (ms_up * 1e-3) / 1e9, 1),
        "adjoint_ms": round(ms_adj, 3), "adjoint_alg_gbs": round(nbytes / (ms_adj * 1e-3) / 1e9, 1),
        "share_of_step": round((ms_up + ms_adj) / base_ms, 5), "n_lambda": k}
    del fine, gc, hc
    torch.cuda.empty_cache()
    # the paper's own grids that are not powers of two (Table 2), 6 wavelengths
    lams6 = np.linspace(0.4, 0.7, 6)
    grids = {}
    for m_, dx_ in ((28800, 0.25), (40000, 0.25)):
        n_ = m_ // 2
        hg = torch.rand((n_, n_), generator=torch.Generator(device="cuda").manual_seed(m_),
                        device="cuda") * 1.2
        pg = api.Problem(n_, m_, dx_, p["z"], lams6, wl.cauchy_index(lams6))
        og = torch.empty((n_, n_), dtype=torch.float32, device="cuda")
        ctx.profile_enable(True)
        ms = _event_ms(torch, lambda: api.psf(hg, pg, out=og, ctx=ctx), 2)
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        rates, _, _ = pass_rates(prof, n_, m_, 6)
        grids[str(m_)] = {
            "n": n_, "n_lambda": 6, "ms_per_step": round(ms, 2),
            "value": round(6 * float(m_) * m_ / (ms * 1e-3) / 1e6, 1),
            "passes_alg_gbs": {k: v["alg_gbs"] for k, v in rates.items()}}
        del hg, og
        ctx.release_workspaces()
        torch.cuda.empty_cache()
    res["np2_grids"] = grids
    # the largest grid one GPU holds: 65536^2 DOE padded to 131072^2 (137 GB workspace)
    ctx.release_workspaces()
    torch.cuda.empty_cache()
    n_h, m_h = 65536, 131072
    lams3 = np.array([0.45, 0.55, 0.65])
    hh = torch.rand((n_h, n_h), generator=torch.Generator(device="cuda").manual_seed(17),
                    device="cuda") * 1.2
    ph = api.Problem(n_h, m_h, p["dx"], p["z"], lams3, wl.cauchy_index(lams3))
    oh = torch.empty((n_h, n_h), dtype=torch.float32, device="cuda")
    ctx.profile_enable(True)
    ms = _event_ms(torch, lambda: api.psf(hh, ph, out=oh, ctx=ctx), 1)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    rates, _, _ = pass_rates(prof, n_h, m_h, 3)
    res["largest_grid"] = {
        "n": n_h, "m": m_h, "n_lambda": 3, "workspace_gb": round(api.workspace_size(ph) / 1e9, 1),
        "ms_per_step": round(ms, 1), "value": round(3 * float(m_h) ** 2 / (ms * 1e-3) / 1e6, 1),
        "passes_alg_gbs": {k: v["alg_gbs"] for k, v in rates.items()}}
    del hh, oh
    ctx.release_workspaces()
    torch.cuda.empty_cache()
    # the paper's largest grid (Table 2): a 32.16 x 21.44 mm DOE at 0.5 um, 64320 x 42880,
    # padded to 128640 x 85760 (radix-67 stages on both axes, an 88 GB workspace)
    ny, nx, my, mx = 64320, 42880, 128640, 85760
    hp = torch.rand((ny, nx), generator=torch.Generator(device="cuda").manual_seed(18),
                    device="cuda") * 1.2
    pp = api.Problem((ny, nx), (my, mx), 0.5, 60000.0, lams3, wl.cauchy_index(lams3))
    op = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    ctx.profile_enable(True)
    ms = _event_ms(torch, lambda: api.psf(hp, pp, out=op, ctx=ctx), 1)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    rates, _, _ = pass_rates(prof, (ny, nx), (my, mx), 3)
    res["paper_grid"] = {
        "doe": f"{ny}x{nx}", "grid": f"{my}x{mx}", "n_lambda": 3,
        "workspace_gb": round(api.workspace_size(pp) / 1e9, 1), "ms_per_step": round(ms, 1),
        "value": round(3 * float(my) * mx / (ms * 1e-3) / 1e6, 1),
        "passes_avg_ms": {k: round(v[1] / v[0], 3) for k, v in prof.items()},
        "passes_alg_gbs": {k: v["alg_gbs"] for k, v in rates.items()}}
    del hp, op
    ctx.release_workspaces()
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="large", choices=["large", "mid", "small", "paper"])
    ap.add_argument("--lambdas", type=int, default=0,
                    help="profiling runs only: keep the first K wavelengths")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--group", type=int, default=4,
                    help="wavelengths per group in the timed PSF calls (1 = one at a time)")
    ap.add_argument("--no-design", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=400,
                    help="requests in the trace at 0.7 x capacity (the 200 req/s trace, "
                         "about 11 x overload, uses a quarter of them)")
    ap.add_argument("--serve-policies", default="chunked,chunked:0.5,fifo",
                    help="server policies to replay (chunked[:age bound s], fifo, size_aware), "
                         "the first reported as 'served'")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the upsampling / band-limit measurements")
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
    (ny, nx), (my, mx) = wl.shape2(n), wl.shape2(m)
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
    psf = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    log("inputs resident on the GPU; warming up")

    for i in range(args.warmup):
        api.psf(hd, prob, out=psf, ctx=ctx, group=args.group)
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")

    ctx.profile_enable(True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record()
    for i in range(args.steps):
        api.psf(hd, prob, out=psf, ctx=ctx, group=args.group)
        marks[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = sorted(marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps))
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    log(f"timed {args.steps} steps in {t1 - t0:.3f} s")

    dt = (t1 - t0) / args.steps
    value = k * float(my) * mx / dt / 1e6

    # per-pass averages and the roofline of the dominant pass (algorithmic
    # bytes per launch; passes A and A' run once per wavelength group)
    passes, groups, totals = pass_rates(prof, n, m, k)
    # the dominant kernel is the one that takes most of the step
    dom = max(passes, key=lambda x: passes[x]["avg_ms"] * passes[x]["launches"])
    dp = passes[dom]
    achieved = dp["alg_gbs"]
    traffic = measured_traffic(dom, m)
    step_bytes = sum(totals.values())
    torch.cuda.synchronize()
    sumv = float(psf.double().sum().item())
    copy_gbs = copy_ceiling_gbs(torch)
    log(f"device copy ceiling {copy_gbs:.0f} GB/s")
    ceil = ceilings_measure(api, torch, ctx.workspace(0, torch.cuda.current_stream().cuda_stream),
                            m if mx == my else 0)
    log(f"probe ceilings (GB/s): {ceil}")
    ceiling = ceil["inplace"]
    pattern = ceil.get("passc_pattern") if dom == "pass_c" else None

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mpix*lambda/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "ms_per_step_median": round(step_ms[len(step_ms) // 2], 3),
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
                "paper": "the paper's largest grid (Table 2 large-area hologram): a 16080x10720 "
                         "design at 2 um upsampled 4x to 64320x42880 heights at 0.5 um "
                         "(32.16 x 21.44 mm), padded to 128640x85760, 520.6 nm, z=60 mm",
            }[args.workload],
            "n": n, "m": m, "n_lambda": k, "dx_um": p["dx"], "z_um": p["z"],
        },
        "value_unpadded": round(k * float(ny) * nx / dt / 1e6, 1),
        "hbm_gbs_alg": round(step_bytes / dt / 1e9, 1),
        "alg_bytes_per_padded_pixel_lambda": round(step_bytes / (k * float(my) * mx), 2),
        "passes": {kk: {"avg_ms": v["avg_ms"], "alg_gbs": v["alg_gbs"]} for kk, v in passes.items()},
        "wavelength_groups": groups,
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_gbs": None if traffic is None else round(traffic / (dp["avg_ms"] * 1e-3) / 1e9, 1),
            "copy_ceiling_gbs": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4),
            "ceiling_gbs": ceiling,
            "frac_of_ceiling": round(achieved / ceiling, 4),
            "pattern_ceiling_gbs": pattern,
            "frac_of_pattern": None if pattern is None else round(achieved / pattern, 4),
            "ceilings": ceil,
        },
        "psf_sum": sumv,
    }
    if not args.no_variants and args.workload == "large" and not args.lambdas:
        log("variants: fused 8x nearest upsampling, band limit, Lanczos-3 kernels, paper grids")
        line["variants"] = variants_measure(api, wl, torch, p, hd, ctx, dt * 1e3)
        log("small and mid workloads")
        line["other_workloads"] = other_workloads_measure(api, wl, torch, ctx)
    if not args.no_cpu_baseline and args.workload == "large":
        log("timing the CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(h, p)
    del hd, psf
    ctx.release_workspaces()
    torch.cuda.empty_cache()
    if not args.no_design:
        log("design workload: 200 Adam steps")
        line["design"] = design_measure(api, wl, torch)
        ctx.release_workspaces()
        torch.cuda.empty_cache()
        log("design iterations on the paper's Table 2 grids")
        line["paper_table2_design"] = paper_table2_measure(api, wl, torch)
    if not args.no_serve:
        log("serving: generating the height pool")
        pool = {n_: [torch.from_numpy(x).cuda() for x in wl.serve_height_pool(n_)]
                for n_ in (2048, 4096, 8192, 16384)}
        pols = tuple(args.serve_policies.split(","))
        log("serving: trace at 200 req/s")
        hot = serve_measure(api, wl, torch, max(8, args.serve_requests // 4), 200.0, pool,
                            policies=pols)
        cap = hot["sequential"]["throughput_req_s"]
        log(f"serving: trace at 0.7 x capacity ({0.7 * cap:.1f} req/s)")
        cool = serve_measure(api, wl, torch, args.serve_requests, 0.7 * cap, pool, seed=6,
                             policies=pols)
        line["serve"] = {"trace": "Poisson arrivals, N in {2048,4096,8192,16384}, M=2N, "
                                  "1-31 wavelengths over 400-700 nm, z in [5,50] mm",
                         "at_200_req_s": hot, "at_0.7x_capacity": cool}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
