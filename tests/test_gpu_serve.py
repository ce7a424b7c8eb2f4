"""Continuous-batching server on the GPU, through the C ABI.

Each request's PSF must be bitwise identical whether it runs alone (dop_psf
on one stream) or admitted into the server's mix, where its passes overlap
with other requests on other streams; a sample is also checked against the
FP64 oracle.
"""

import os

import numpy as np
import pytest

import oracle
from oracle import asm
from paper_2505_22313_amd import workloads as wl
from _close import assert_close, INTENSITY_ELEM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

asm.WORKERS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_22313_amd import api as _api
    return _api


def make_requests(api, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        n = int(rng.choice([256, 384, 512, 1024]))
        m = 2 * n if n != 384 else 1024
        k = int(rng.integers(1, 6))
        lams = np.linspace(0.4, 0.7, k) if k > 1 else np.array([0.55])
        mode = "full" if rng.random() < 0.25 else "crop"
        prob = api.Problem(n, m, 1.0, float(rng.uniform(500.0, 5000.0)), lams,
                           wl.cauchy_index(lams), out_mode=mode)
        h = torch.from_numpy(wl.uniform_heights(n, seed=1000 * seed + i)).cuda()
        amp = None
        if rng.random() < 0.3:
            amp = torch.from_numpy(wl.circular_aperture(n, 1.0, 0.4 * n)).cuda()
        reqs.append((prob, h, amp))
    return reqs


@pytest.mark.parametrize("policy", ["chunked", "fifo"])
def test_serve_bitwise_alone_vs_mix(api, policy):
    """Under the chunked policy a request runs in wavelength-group chunks
    interleaved with other requests' chunks on one stream; under FIFO whole
    requests run side by side on several streams.  Either way each PSF is
    bitwise the one dop_psf computes for the request alone."""
    reqs = make_requests(api, 24, seed=7)
    alone = [api.psf(h, prob, amp=amp).clone() for prob, h, amp in reqs]
    torch.cuda.synchronize()
    # arena for about three of the largest workspaces: admission is memory-bound
    big = max(api.workspace_size(p) for p, _, _ in reqs)
    srv = api.Server(3 * big, max_slots=4, policy=policy)
    try:
        outs = [torch.full(p.out_shape, float("nan"), device="cuda") for p, _, _ in reqs]
        torch.cuda.synchronize()
        tickets = [srv.submit(p, h, o, amp=a) for (p, h, a), o in zip(reqs, outs)]
        for t in tickets:
            srv.wait(t, 60.0)
        stats = srv.stats()
        assert stats["completed"] == len(reqs) and stats["failed"] == 0
        assert stats["arena_peak"] <= 3 * big
        for i, (a, b) in enumerate(zip(alone, outs)):
            assert torch.equal(a, b), f"request {i} differs between alone and mix"
    finally:
        srv.close()
    # a sample against the oracle
    for i in (0, 5, 11):
        prob, h, amp = reqs[i]
        want = oracle.psf(h.cpu().numpy(), prob.dx, prob.z, prob.m, prob.lambdas, prob.n_index,
                          amp=None if amp is None else amp.cpu().numpy(), out_mode=prob.out_mode)
        got = alone[i].cpu().numpy()
        assert_close(got, want, 2e-5, INTENSITY_ELEM, f"request {i}")


def test_serve_many_small_requests_overlap(api):
    """Many requests with a roomy arena: all complete, several run at once."""
    reqs = make_requests(api, 40, seed=11)
    arena = 8 * max(api.workspace_size(p) for p, _, _ in reqs)
    srv = api.Server(arena, max_slots=8)
    try:
        outs = [torch.empty(p.out_shape, device="cuda") for p, _, _ in reqs]
        torch.cuda.synchronize()
        tickets = [srv.submit(p, h, o, amp=a) for (p, h, a), o in zip(reqs, outs)]
        peak = 0
        while srv.stats()["completed"] < len(reqs):
            peak = max(peak, srv.stats()["running"])
        for t in tickets:
            srv.wait(t, 60.0)
        s = srv.stats()
        assert s["failed"] == 0 and s["completed"] == len(reqs)
        assert peak >= 2
        assert s["p50_ms"] <= s["p99_ms"]
        ref = api.psf(reqs[3][1], reqs[3][0], amp=reqs[3][2])
        assert torch.equal(ref, outs[3])
    finally:
        srv.close()


def test_serve_mixed_problem_kinds(api):
    """Requests that use the band limit, the fused 8x nearest upsampling,
    grids that are not powers of two and rectangular grids (one with the
    radix-67 stage), mixed with plain ones: each result is bitwise the same
    as the request run alone, and a sample matches the oracle."""
    from oracle import upsample as ups
    rng = np.random.default_rng(13)
    reqs = []
    for i in range(18):
        kind = i % 6
        lams = np.linspace(0.45, 0.65, 1 + i % 3)
        z = float(rng.uniform(500.0, 4000.0))
        if kind == 0:
            prob = api.Problem(512, 1024, 1.0, z, lams, wl.cauchy_index(lams), bandlimit=True)
            h = wl.uniform_heights(512, seed=300 + i)
        elif kind == 1:
            prob = api.Problem(512, 1024, 0.5, z, lams, wl.cauchy_index(lams), upsample=8)
            h = wl.uniform_heights(64, seed=300 + i)
        elif kind == 2:
            prob = api.Problem(360, 720, 1.0, z, lams, wl.cauchy_index(lams))
            h = wl.uniform_heights(360, seed=300 + i)
        elif kind == 3:
            prob = api.Problem(1500, 3600, 0.5, z, lams, wl.cauchy_index(lams), out_mode="full")
            h = wl.uniform_heights(1500, seed=300 + i)
        elif kind == 4:
            prob = api.Problem((200, 1500), (240, 2144), 1.0, z, lams, wl.cauchy_index(lams))
            h = wl.uniform_heights((200, 1500), seed=300 + i)
        else:
            prob = api.Problem((500, 150), (720, 240), 0.5, z, lams, wl.cauchy_index(lams),
                               out_mode="full")
            h = wl.uniform_heights((500, 150), seed=300 + i)
        reqs.append((prob, torch.from_numpy(h).cuda(), h))
    alone = [api.psf(hd, prob).clone() for prob, hd, _ in reqs]
    torch.cuda.synchronize()
    big = max(api.workspace_size(p) for p, _, _ in reqs)
    srv = api.Server(3 * big, max_slots=4)
    try:
        outs = [torch.full(p.out_shape, float("nan"), device="cuda") for p, _, _ in reqs]
        torch.cuda.synchronize()
        tickets = [srv.submit(p, hd, o) for (p, hd, _), o in zip(reqs, outs)]
        for t in tickets:
            srv.wait(t, 60.0)
        assert srv.stats()["failed"] == 0
        for i, (a, b) in enumerate(zip(alone, outs)):
            assert torch.equal(a, b), f"request {i} differs between alone and mix"
    finally:
        srv.close()
    for i in range(6):
        prob, _, h = reqs[i]
        hf = ups.upsample(h, 8, "nearest") if prob.upsample > 1 else h
        want = oracle.psf(hf, prob.dx, prob.z, prob.grid_shape, prob.lambdas, prob.n_index,
                          out_mode=prob.out_mode, bandlimit=prob.bandlimit)
        assert_close(alone[i].cpu().numpy(), want, 2e-5, INTENSITY_ELEM, f"request {i}")


@pytest.mark.timeout(900)
def test_serve_serving_workload_sizes(api):
    """Requests at the serving workload's sizes: N in {2048, 4096, 8192,
    16384} on 2x-padded grids, 1..31 wavelengths over 400..700 nm, z in
    [5, 50] mm, smooth random heights, through a 4-slot server whose arena
    (about 26 GB) holds three of the largest workspaces, so admission waits
    for memory as well as slots.  Every result is bitwise the same alone and
    in the mix; the N = 2048 requests (one with all 31 wavelengths) are also
    checked against the FP64 oracle."""
    rng = np.random.default_rng(55)
    sizes = [2048, 16384, 4096, 8192, 2048, 16384, 8192, 4096]
    ks = [31, 31, 17, 24, 3, 9, 1, 12]
    pools = {n: torch.from_numpy(wl.serve_height_pool(n, count=1, seed=55)[0]).cuda()
             for n in set(sizes)}
    reqs = []
    for i, (n, k) in enumerate(zip(sizes, ks)):
        lams = np.array([0.55]) if k == 1 else np.linspace(0.40, 0.70, k)
        mode = "full" if i == 7 else "crop"
        prob = api.Problem(n, 2 * n, 1.0, float(rng.uniform(5000.0, 50000.0)), lams,
                           wl.cauchy_index(lams), out_mode=mode)
        reqs.append((prob, pools[n]))
    print("  alone", flush=True)
    alone = [api.psf(h, prob).clone() for prob, h in reqs]
    torch.cuda.synchronize()
    api.default_context(0).release_workspaces()
    torch.cuda.empty_cache()
    big = max(api.workspace_size(p) for p, _ in reqs)
    srv = api.Server(3 * big, max_slots=4)
    try:
        outs = [torch.full(p.out_shape, float("nan"), device="cuda") for p, _ in reqs]
        torch.cuda.synchronize()
        print("  mix", flush=True)
        tickets = [srv.submit(p, h, o) for (p, h), o in zip(reqs, outs)]
        peak = 0
        while srv.stats()["completed"] < len(reqs):
            peak = max(peak, srv.stats()["running"])
        for t in tickets:
            srv.wait(t, 120.0)
        stats = srv.stats()
        assert stats["completed"] == len(reqs) and stats["failed"] == 0
        assert stats["arena_peak"] <= 3 * big
        assert peak >= 2
        for i, (a, b) in enumerate(zip(alone, outs)):
            assert torch.equal(a, b), f"request {i} (N {sizes[i]}, k {ks[i]}) differs"
    finally:
        srv.close()
        del outs
        torch.cuda.empty_cache()
    for i, (prob, h) in enumerate(reqs):
        if prob.n != 2048:
            continue
        print(f"  oracle request {i}: k {prob.k}", flush=True)
        want = oracle.psf(h.cpu().numpy(), prob.dx, prob.z, prob.m, prob.lambdas, prob.n_index,
                          out_mode=prob.out_mode)
        assert_close(alone[i].cpu().numpy(), want, 2e-5, INTENSITY_ELEM, f"request {i}")
