"""Grids that are not powers of two (M = 2^a 3^b 5^c) on the GPU, through the
C ABI, against the FP64 oracle: small grids element by element, and the
paper's own single-GPU grids (28,800^2 and 40,000^2, Table 2) on whole PSFs.
Tolerances as in the power-of-two parity tests.
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
    yield _api
    torch.cuda.empty_cache()


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


# (m, n, dx, lam, z): every supported small grid, ragged N, evanescent bins,
# negative z, no padding
NP2_CASES = [
    (240, 100, 0.5, 0.55, 60.0),
    (240, 240, 0.3, 0.5, 9.0),
    (720, 333, 1.0, 0.6, 2000.0),
    (1440, 700, 0.5, 0.45, -3000.0),
    (3072, 1536, 1.0, 0.55, 20000.0),
    (3600, 1801, 0.25, 0.5206, 300.0),
]


@pytest.mark.parametrize("m,n,dx,lam,z", NP2_CASES)
@pytest.mark.parametrize("out_mode", ["crop", "full"])
def test_np2_propagate_matches_oracle(api, m, n, dx, lam, z, out_mode):
    rng = np.random.default_rng(m + 3 * n)
    u = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64)
    prob = api.Problem(n, m, dx, z, [lam], [1.5], out_mode=out_mode)
    got = api.propagate(dev(u, torch.complex64), prob).cpu().numpy()
    want = oracle.propagate(u.astype(np.complex128), m, dx, lam, z, out_mode=out_mode)
    assert_close(got, want, FIELD_TOL, FIELD_ELEM)


@pytest.mark.parametrize("m,n", [(720, 360), (3600, 1500)])
def test_np2_psf_and_backward(api, m, n):
    dx, z = 0.5, 1500.0
    lams = np.array([0.45, 0.55, 0.65])
    nidx = wl.cauchy_index(lams)
    w = np.array([1.0, 0.5, 2.0], dtype=np.float32)
    rng = np.random.default_rng(m)
    h = wl.uniform_heights(n, seed=m)
    amp = rng.uniform(0.5, 1.0, (n, n)).astype(np.float32)
    g = rng.standard_normal((n, n)).astype(np.float32)
    prob = api.Problem(n, m, dx, z, lams, nidx, weights=w)
    hd, ad = dev(h, torch.float32), dev(amp, torch.float32)
    got, saved = api.psf(hd, prob, amp=ad, save_fields=True)
    want = oracle.psf(h, dx, z, m, lams, nidx, weights=w, amp=amp)
    assert_close(got.cpu().numpy(), want, INTENSITY_TOL, INTENSITY_ELEM)
    gh = api.psf_backward(hd, prob, saved, dev(g, torch.float32), amp=ad).cpu().numpy()
    want_g = oracle.psf_backward(h, dx, z, m, lams, nidx, g, weights=w, amp=amp)
    assert_close(gh, want_g, GRAD_TOL, GRAD_ELEM)


def test_np2_full_output_and_bandlimit(api):
    m, n, dx, lam, z = 1440, 600, 0.5, 0.5, 4000.0
    h = wl.uniform_heights(n, seed=77)
    prob = api.Problem(n, m, dx, z, [lam], [1.46], out_mode="full", bandlimit=True)
    got = api.psf(dev(h, torch.float32), prob).cpu().numpy()
    want = oracle.psf(h, dx, z, m, [lam], [1.46], out_mode="full", bandlimit=True)
    assert_close(got, want, INTENSITY_TOL, INTENSITY_ELEM)


@pytest.mark.timeout(500)
@pytest.mark.parametrize("m,dx,lam,z", [
    (28800, 0.25, 0.5206, 20000.0),   # CHD grid of Table 2 (3.6 mm at 250 nm, 2x padded)
    (40000, 0.25, 0.55, 50000.0),     # broadband imaging grid of Table 2
])
def test_np2_paper_grid_whole_psf(api, m, dx, lam, z):
    """The paper's own grids at full size: the whole N x N PSF of a random
    height map (N = M/2) against the FP64 oracle (rel-L2 <= 1e-4, as for the
    other full-size workloads), and its energy."""
    n = m // 2
    nidx = float(wl.cauchy_index(lam))
    h = wl.uniform_heights(n, seed=m // 100)
    prob = api.Problem(n, m, dx, z, [lam], [nidx])
    got = api.psf(dev(h, torch.float32), prob).double().cpu().numpy()
    torch.cuda.empty_cache()
    want = oracle.psf_lowmem(h, dx, z, m, lam, nidx,
                             log=lambda msg: print("  oracle:", msg, flush=True))
    assert_close(got, want, 1e-4, 1e-4)
    assert abs(got.sum() / want.sum() - 1) < 1e-5
