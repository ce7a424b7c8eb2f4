"""Super-resolved front end on the GPU, through the C ABI, against the FP64
oracle: dop_upsample / dop_upsample_adjoint (nearest and Lanczos-3), the
nearest upsampling fused into dop_psf / dop_psf_backward, and the Lanczos-3
chain through autograd.

Tolerances: nearest upsampling copies floats (bitwise); Lanczos-3 forms its
weights in FP64, rounds them to float32 and sums 36 products in float32, so
rel-L2 <= 1e-6 on the fine map; adjoints sum up to 7s terms per axis in
float32, rel-L2 <= 1e-5.  PSF and gradient tolerances as in the parity
tests.
"""

import os

import numpy as np
import pytest

import oracle
from oracle import asm
from oracle import upsample as ups
from paper_2505_22313_amd import workloads as wl
from _close import assert_close, GRAD_ELEM, INTENSITY_ELEM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

asm.WORKERS = min(16, os.cpu_count() or 1)

INTENSITY_TOL = 2e-5
GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_22313_amd import api as _api
    return _api


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


# (nc, s): one-pixel designs, odd factors, fine grids that are not a multiple
# of the 64-pixel tile, factor 1 and 16
SIZES = [(1, 1), (1, 16), (5, 3), (37, 8), (100, 2), (64, 16), (130, 1), (333, 5)]


@pytest.mark.parametrize("nc,s", SIZES)
@pytest.mark.parametrize("kind", ["nearest", "lanczos3"])
def test_upsample_matches_oracle(api, nc, s, kind):
    rng = np.random.default_rng(nc * 31 + s)
    hc = rng.uniform(0.0, 1.2, (nc, nc)).astype(np.float32)
    got = api.upsample(dev(hc), s, kind).cpu().numpy()
    want = ups.upsample(hc, s, kind)
    if kind == "nearest":
        assert np.array_equal(got, want.astype(np.float32))
    else:
        assert_close(got, want, 1e-6, 1e-6)


@pytest.mark.parametrize("nc,s", SIZES)
@pytest.mark.parametrize("kind", ["nearest", "lanczos3"])
def test_upsample_adjoint_matches_oracle(api, nc, s, kind):
    rng = np.random.default_rng(nc * 37 + s)
    g = rng.standard_normal((nc * s, nc * s)).astype(np.float32)
    got = api.upsample_adjoint(dev(g), s, kind).cpu().numpy()
    want = ups.upsample_adjoint(g, s, kind)
    assert_close(got, want, 1e-5, 1e-5)


def test_lanczos_large_sampled_rows(api):
    """A 4096^2 design at 8x (32768^2, the large workload's DOE grid):
    sampled fine rows against rows of the oracle's W hc W^T."""
    nc, s = 4096, 8
    hc = wl.uniform_heights(nc, seed=61)
    fine = api.upsample(dev(hc), s, "lanczos3")
    rows = [0, 1, 7, 12345, 16384, 32760, 32767]
    w = ups.axis_matrix(nc, s, "lanczos3")
    want = (w[rows] @ hc.astype(np.float64)) @ w.T
    got = fine[torch.tensor(rows, device="cuda")].cpu().numpy()
    assert_close(got, want, 1e-6, 1e-6)
    del fine
    torch.cuda.empty_cache()


def test_fused_nearest_psf_and_backward(api):
    """8x nearest upsampling inside pass A, with a fine-grid aperture: the
    PSF of a 64^2 design equals the oracle's PSF of its 512^2 upsampled map,
    and bitwise the library's own PSF of the separately upsampled map; the
    coarse gradient is the oracle gradient summed over 8 x 8 blocks."""
    nc, s, m, dx, z = 64, 8, 1024, 0.25, 400.0
    n = nc * s
    lams = np.array([0.45, 0.55, 0.65])
    nidx = wl.cauchy_index(lams)
    rng = np.random.default_rng(62)
    hc = rng.uniform(0.0, 1.2, (nc, nc)).astype(np.float32)
    g = rng.standard_normal((n, n)).astype(np.float32)
    amp = wl.circular_aperture(n, dx, 50.0)
    ad = dev(amp)
    hf = ups.upsample(hc, s, "nearest")
    pu = api.Problem(n, m, dx, z, lams, nidx, upsample=s)
    pf = api.Problem(n, m, dx, z, lams, nidx)
    got, saved = api.psf(dev(hc), pu, amp=ad, save_fields=True)
    want = oracle.psf(hf, dx, z, m, lams, nidx, amp=amp)
    assert_close(got.cpu().numpy(), want, INTENSITY_TOL, INTENSITY_ELEM)
    hf_dev = api.upsample(dev(hc), s, "nearest")
    ref, saved_ref = api.psf(hf_dev, pf, amp=ad, save_fields=True)
    assert torch.equal(got, ref) and torch.equal(saved, saved_ref)
    gc = api.psf_backward(dev(hc), pu, saved, dev(g), amp=ad)
    assert tuple(gc.shape) == (nc, nc)
    want_g = ups.upsample_adjoint(oracle.psf_backward(hf, dx, z, m, lams, nidx, g, amp=amp), s,
                                  "nearest")
    assert_close(gc.cpu().numpy(), want_g, GRAD_TOL, GRAD_ELEM)
    gf = api.psf_backward(hf_dev, pf, saved_ref, dev(g), amp=ad)
    assert torch.equal(gc, api.upsample_adjoint(gf, s, "nearest"))


def test_lanczos_design_gradient_through_autograd(api):
    """Lanczos-3 front end chained with the PSF in a torch loss: the gradient
    with respect to the coarse design equals the oracle chain
    U^T (dPSF/dh)^T dL/dPSF."""
    nc, s, m, dx, z = 48, 4, 512, 0.5, 600.0
    n = nc * s
    lams = np.array([0.5, 0.62])
    nidx = wl.cauchy_index(lams)
    rng = np.random.default_rng(63)
    hc = rng.uniform(0.0, 1.2, (nc, nc)).astype(np.float32)
    target = wl.gaussian_target(n, 3.0, total=2 * n * n)
    prob = api.Problem(n, m, dx, z, lams, nidx)
    hcd = dev(hc).requires_grad_(True)
    h = api.DopUpsample.apply(hcd, s, "lanczos3")
    loss = torch.mean((api.DopPSF.apply(h, prob) - dev(target)) ** 2)
    loss.backward()
    hf = ups.upsample(hc, s, "lanczos3")
    p = oracle.psf(hf, dx, z, m, lams, nidx)
    gpsf = 2.0 * (p - target) / (n * n)
    want = ups.upsample_adjoint(oracle.psf_backward(hf, dx, z, m, lams, nidx, gpsf), s, "lanczos3")
    assert_close(hcd.grad.cpu().numpy(), want, GRAD_TOL, GRAD_ELEM)


# (ncy, ncx, s): rectangular designs, one-sample axes, fine axes that are not
# a multiple of the 64-pixel tile
RECT_SIZES = [(1, 5, 16), (5, 37, 3), (37, 8, 8), (100, 70, 2), (64, 130, 5), (9, 200, 1)]


@pytest.mark.parametrize("ncy,ncx,s", RECT_SIZES)
@pytest.mark.parametrize("kind", ["nearest", "lanczos3"])
def test_rect_upsample_and_adjoint_match_oracle(api, ncy, ncx, s, kind):
    rng = np.random.default_rng(ncy * 131 + ncx * 7 + s)
    hc = rng.uniform(0.0, 1.2, (ncy, ncx)).astype(np.float32)
    got = api.upsample(dev(hc), s, kind).cpu().numpy()
    want = ups.upsample(hc, s, kind)
    assert got.shape == (ncy * s, ncx * s)
    if kind == "nearest":
        assert np.array_equal(got, want.astype(np.float32))
    else:
        assert_close(got, want, 1e-6, 1e-6)
    g = rng.standard_normal((ncy * s, ncx * s)).astype(np.float32)
    got_a = api.upsample_adjoint(dev(g), s, kind).cpu().numpy()
    assert got_a.shape == (ncy, ncx)
    assert_close(got_a, ups.upsample_adjoint(g, s, kind), 1e-5, 1e-5)


def test_rect_lanczos_design_gradient_through_autograd(api):
    """A 60 x 30 design, Lanczos-3 at 4x, on the 720 x 240 grid: the gradient
    of a PSF loss with respect to the coarse design equals the oracle chain."""
    ncy, ncx, s, my, mx, dx, z = 60, 30, 4, 720, 240, 0.5, 600.0
    ny, nx = ncy * s, ncx * s
    lams = np.array([0.5, 0.62])
    nidx = wl.cauchy_index(lams)
    rng = np.random.default_rng(64)
    hc = rng.uniform(0.0, 1.2, (ncy, ncx)).astype(np.float32)
    target = wl.gaussian_target((ny, nx), 3.0, total=2.0 * ny * nx)
    prob = api.Problem((ny, nx), (my, mx), dx, z, lams, nidx)
    hcd = dev(hc).requires_grad_(True)
    h = api.DopUpsample.apply(hcd, s, "lanczos3")
    loss = torch.mean((api.DopPSF.apply(h, prob) - dev(target)) ** 2)
    loss.backward()
    hf = ups.upsample(hc, s, "lanczos3")
    p = oracle.psf(hf, dx, z, (my, mx), lams, nidx)
    gpsf = 2.0 * (p - target) / (ny * nx)
    want = ups.upsample_adjoint(oracle.psf_backward(hf, dx, z, (my, mx), lams, nidx, gpsf), s,
                                "lanczos3")
    assert_close(hcd.grad.cpu().numpy(), want, GRAD_TOL, GRAD_ELEM)
