"""HIP path vs the FP64 oracle, element by element (GPU only).

Every call goes through the C ABI (libdop.so) via the thin Python binding.
Tolerances: complex fields rel-L2 <= 1e-5 (FP32 butterflies, FP64-argument
phase and transfer function, stated for 4096^2 fields), intensities
rel-L2 <= 2e-5 at these sizes, gradients rel-L2 <= 1e-4.
"""

import os

import numpy as np
import pytest

import oracle
from oracle import asm
from paper_2505_22313_amd import workloads as wl
from _close import assert_close, FIELD_ELEM, GRAD_ELEM, INTENSITY_ELEM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

asm.WORKERS = min(16, os.cpu_count() or 1)

FIELD_TOL = 1e-5
INTENSITY_TOL = 2e-5
GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_22313_amd import api as _api
    return _api


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def rand_field(rng, n):
    return (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64)


# (m, n, dx, lam, z): sizes span one-tile grids to several tiles per pass and
# ragged N (not a multiple of any tile edge); some cases cut evanescent bins.
PROP_CASES = [
    (16, 8, 1.0, 0.55, 40.0),
    (16, 16, 0.3, 0.5, 9.0),       # no padding, evanescent bins
    (32, 17, 0.3, 0.5, 12.0),
    (64, 1, 1.0, 0.55, 100.0),      # single-pixel source
    (64, 63, 0.27, 0.5, 30.0),
    (128, 100, 1.0, 0.6, 700.0),
    (256, 128, 0.25, 0.5206, 80.0),
    (512, 301, 1.0, 0.55, 2000.0),
    (1024, 512, 1.0, 0.55, 5000.0),
    (2048, 1500, 0.5, 0.45, -3000.0),  # negative z
    (4096, 2048, 1.0, 0.55, 20000.0),
]


@pytest.mark.parametrize("m,n,dx,lam,z", PROP_CASES)
@pytest.mark.parametrize("out_mode", ["crop", "full"])
def test_propagate_matches_oracle(api, m, n, dx, lam, z, out_mode):
    rng = np.random.default_rng(m * 7 + n)
    u = rand_field(rng, n)
    prob = api.Problem(n, m, dx, z, [lam], [1.5], out_mode=out_mode)
    got = api.propagate(dev(u, torch.complex64), prob).cpu().numpy()
    want = oracle.propagate(u.astype(np.complex128), m, dx, lam, z, out_mode=out_mode)
    assert_close(got, want, FIELD_TOL, FIELD_ELEM)


def test_small_workload_psf(api):
    """512^2 uniform heights, 1 um pitch, 550 nm, z = 5 mm, padded to 1024^2."""
    p = wl.problem("small")
    h = wl.heights("small")
    prob = api.Problem.from_dict(p)
    got, saved = api.psf(dev(h, torch.float32), prob, save_fields=True)
    want, fields = oracle.psf(h, p["dx"], p["z"], p["m"], p["lams"], p["n_index"],
                              return_fields=True)
    assert_close(got.cpu().numpy(), want, INTENSITY_TOL, INTENSITY_ELEM)
    assert_close(saved[0].cpu().numpy(), fields[0], FIELD_TOL, FIELD_ELEM)


def test_field_4096(api):
    """Field parity at a 4096^2 padded grid (2048^2 DOE)."""
    n, m, dx, z = 2048, 4096, 1.0, 10000.0
    lams = [0.45, 0.65]
    nidx = wl.cauchy_index(lams)
    h = wl.uniform_heights(n, seed=41)
    prob = api.Problem(n, m, dx, z, lams, nidx)
    got, saved = api.psf(dev(h, torch.float32), prob, save_fields=True)
    want, fields = oracle.psf(h, dx, z, m, lams, nidx, return_fields=True)
    for k in range(2):
        assert_close(saved[k].cpu().numpy(), fields[k], FIELD_TOL, FIELD_ELEM)
    assert_close(got.cpu().numpy(), want, INTENSITY_TOL, INTENSITY_ELEM)


@pytest.mark.parametrize("out_mode", ["crop", "full"])
def test_psf_weights_amp_multi_lambda(api, out_mode):
    n, m, dx, z = 200, 512, 0.5, 1500.0
    lams = np.array([0.40, 0.47, 0.55, 0.62, 0.70])
    nidx = wl.cauchy_index(lams)
    w = np.array([0.3, 1.0, 2.0, 0.5, 1.5], dtype=np.float32)
    h = wl.uniform_heights(n, seed=42)
    amp = wl.circular_aperture(n, dx, 40.0) * np.float32(0.8)
    prob = api.Problem(n, m, dx, z, lams, nidx, weights=w, out_mode=out_mode)
    got = api.psf(dev(h, torch.float32), prob, amp=dev(amp, torch.float32)).cpu().numpy()
    want = oracle.psf(h, dx, z, m, lams, nidx, weights=w, amp=amp, out_mode=out_mode)
    assert_close(got, want, INTENSITY_TOL, INTENSITY_ELEM)


def test_evanescent_cut_energy(api):
    """Pitch 0.25 um at 520.6 nm: axis bins beyond 1/lambda are cut; the GPU
    output energy matches the oracle's."""
    n, m, dx, lam, z = 512, 1024, 0.25, 0.5206, 300.0
    h = wl.uniform_heights(n, seed=43)
    prob = api.Problem(n, m, dx, z, [lam], [1.46], out_mode="full")
    got = api.psf(dev(h, torch.float32), prob).cpu().numpy().astype(np.float64)
    want = oracle.psf(h, dx, z, m, [lam], [1.46], out_mode="full")
    assert_close(got, want, INTENSITY_TOL, INTENSITY_ELEM)
    assert abs(got.sum() / want.sum() - 1) < 1e-5
    assert want.sum() < n * n * 0.999


def test_backward_matches_oracle(api):
    n, m, dx, z = 256, 512, 1.0, 3000.0
    lams = np.array([0.45, 0.55, 0.65])
    nidx = wl.cauchy_index(lams)
    w = np.array([1.0, 0.5, 2.0], dtype=np.float32)
    rng = np.random.default_rng(44)
    h = wl.uniform_heights(n, seed=44)
    amp = rng.uniform(0.5, 1.0, (n, n)).astype(np.float32)
    g = rng.standard_normal((n, n)).astype(np.float32)
    prob = api.Problem(n, m, dx, z, lams, nidx, weights=w)
    hd, ad = dev(h, torch.float32), dev(amp, torch.float32)
    _, saved = api.psf(hd, prob, amp=ad, save_fields=True)
    got = api.psf_backward(hd, prob, saved, dev(g, torch.float32), amp=ad).cpu().numpy()
    want = oracle.psf_backward(h, dx, z, m, lams, nidx, g, weights=w, amp=amp)
    assert_close(got, want, GRAD_TOL, GRAD_ELEM)


def test_autograd_function(api):
    """DopPSF inside a torch loss: backward equals the oracle gradient of the
    same loss."""
    n, m, dx, z = 128, 256, 1.0, 2000.0
    lams = np.array([0.5, 0.6])
    nidx = wl.cauchy_index(lams)
    h = wl.uniform_heights(n, seed=45)
    target = wl.gaussian_target(n, 3.0, total=2 * n * n)
    prob = api.Problem(n, m, dx, z, lams, nidx)
    hd = dev(h, torch.float32).requires_grad_(True)
    td = dev(target, torch.float32)
    loss = torch.mean((api.DopPSF.apply(hd, prob) - td) ** 2)
    loss.backward()
    p = oracle.psf(h, dx, z, m, lams, nidx)
    g = 2.0 * (p - target) / (n * n)
    want = oracle.psf_backward(h, dx, z, m, lams, nidx, g)
    assert_close(hd.grad.cpu().numpy(), want, GRAD_TOL, GRAD_ELEM)
    assert abs(loss.item() / np.mean((p - target) ** 2) - 1) < 1e-5


def test_deterministic_bitwise(api):
    p = wl.problem("small")
    h = dev(wl.heights("small"), torch.float32)
    prob = api.Problem.from_dict(p)
    a = api.psf(h, prob).clone()
    b = api.psf(h, prob).clone()
    assert torch.equal(a, b)


@pytest.mark.timeout(500)
def test_mid_workload_psf(api):
    """8192^2 lens + noise, 3 wavelengths, padded to 16384^2: the whole PSF
    against the oracle."""
    p = wl.problem("mid")
    h = wl.heights("mid")
    prob = api.Problem.from_dict(p)
    got = api.psf(dev(h, torch.float32), prob).cpu().numpy()
    torch.cuda.synchronize()
    want = np.zeros_like(got, dtype=np.float64)
    for k in range(3):
        print(f"  oracle lambda {p['lams'][k]}", flush=True)
        want += oracle.psf(h, p["dx"], p["z"], p["m"], [p["lams"][k]], [p["n_index"][k]])
    assert_close(got, want, 1e-4, 1e-4)


# Band-limited ASM: z large against M dx so that f_lim falls well inside the
# Nyquist band and the cut removes many bins.
BL_CASES = [
    (16, 9, 1.0, 0.55, 60.0),
    (64, 40, 0.5, 0.5, 400.0),
    (256, 200, 1.0, 0.55, 2000.0),
    (1024, 700, 0.5, 0.45, -6000.0),
    (4096, 2048, 1.0, 0.65, 40000.0),
]


@pytest.mark.parametrize("m,n,dx,lam,z", BL_CASES)
@pytest.mark.parametrize("out_mode", ["crop", "full"])
def test_propagate_bandlimit_matches_oracle(api, m, n, dx, lam, z, out_mode):
    flim = asm.band_limit(m, dx, lam, z)
    assert flim < 0.5 / dx
    rng = np.random.default_rng(m * 11 + n)
    u = rand_field(rng, n)
    prob = api.Problem(n, m, dx, z, [lam], [1.5], out_mode=out_mode, bandlimit=True)
    got = api.propagate(dev(u, torch.complex64), prob).cpu().numpy()
    want = oracle.propagate(u.astype(np.complex128), m, dx, lam, z, out_mode=out_mode,
                            bandlimit=True)
    assert_close(got, want, FIELD_TOL, FIELD_ELEM)
    plain = oracle.propagate(u.astype(np.complex128), m, dx, lam, z, out_mode=out_mode)
    assert rel(plain, want) > 1e-3


def test_psf_and_backward_bandlimit(api):
    n, m, dx, z = 256, 512, 1.0, 8000.0
    lams = np.array([0.45, 0.6])
    nidx = wl.cauchy_index(lams)
    w = np.array([1.0, 0.7], dtype=np.float32)
    rng = np.random.default_rng(46)
    h = wl.uniform_heights(n, seed=46)
    g = rng.standard_normal((n, n)).astype(np.float32)
    prob = api.Problem(n, m, dx, z, lams, nidx, weights=w, bandlimit=True)
    hd = dev(h, torch.float32)
    got, saved = api.psf(hd, prob, save_fields=True)
    want = oracle.psf(h, dx, z, m, lams, nidx, weights=w, bandlimit=True)
    assert_close(got.cpu().numpy(), want, INTENSITY_TOL, INTENSITY_ELEM)
    gh = api.psf_backward(hd, prob, saved, dev(g, torch.float32)).cpu().numpy()
    want_g = oracle.psf_backward(h, dx, z, m, lams, nidx, g, weights=w, bandlimit=True)
    assert_close(gh, want_g, GRAD_TOL, GRAD_ELEM)


def test_hip_graph_capture_replays(api):
    """The launch-bound small workload captured into a HIP graph (through
    torch.cuda.CUDAGraph; the library launches on the capturing stream and
    records no memset): every replay, with eager work and synchronisation in
    between, equals the eager result bitwise, and a replay after new heights
    are copied into the captured input matches an eager call on them."""
    p = wl.problem("small")
    prob = api.Problem.from_dict(p)
    h = dev(wl.heights("small"), torch.float32)
    eager = api.psf(h, prob).clone()
    out = torch.empty_like(eager)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        api.psf(h, prob, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        api.psf(h, prob, out=out)
    for _ in range(3):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager)
    h2 = dev(wl.uniform_heights(p["n"], seed=99), torch.float32)
    h.copy_(h2)
    graph.replay()
    torch.cuda.synchronize()
    assert torch.equal(out, api.psf(h2, prob))
    del graph
