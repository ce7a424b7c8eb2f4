"""Rectangular grids and the radix-67 stage on the GPU, through the C ABI,
against the FP64 oracle, element by element: every rectangular grid of the
plan table and the square 2144 = 2^5 67 grid, ragged DOEs, no padding along
one axis, evanescent bins, negative z, CROP and FULL, weights and amplitude,
the band limit (its own f_lim per axis), the adjoint, the fused nearest
upsampling, and a 16080 x 10720 grid whose digit split (670 x 16 columns,
16 x 1005 rows: radix 2, 5, 67 and 15, 67 DFTs) is that of the paper's
128,640 x 85,760 grid at an eighth of its digits.  Tolerances as in the
square parity tests.
"""

import os

import numpy as np
import pytest

import oracle
from oracle import asm
from oracle import upsample as ups
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


def cfield(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


# (my, mx, ny, nx, dx, lam, z)
RECT_CASES = [
    (720, 240, 500, 117, 0.5, 0.55, 60.0),
    (512, 2048, 300, 1000, 0.3, 0.5, 9.0),         # evanescent corners
    (240, 2144, 240, 1072, 1.0, 0.6, 2000.0),      # no padding along y; radix 67 in x
    (5360, 240, 2681, 240, 0.5, 0.45, -3000.0),    # no padding along x; radix 67 in y
    (2144, 2144, 1072, 1001, 0.25, 0.5206, 300.0),  # square, radix 67 on both axes
]


@pytest.mark.parametrize("my,mx,ny,nx,dx,lam,z", RECT_CASES)
@pytest.mark.parametrize("out_mode", ["crop", "full"])
def test_rect_propagate_matches_oracle(api, my, mx, ny, nx, dx, lam, z, out_mode):
    print(f"rect propagate {my}x{mx} doe {ny}x{nx} {out_mode}", flush=True)
    rng = np.random.default_rng(my + 7 * mx + ny)
    u = cfield(rng, (ny, nx))
    prob = api.Problem((ny, nx), (my, mx), dx, z, [lam], [1.5], out_mode=out_mode)
    got = api.propagate(dev(u, torch.complex64), prob).cpu().numpy()
    want = oracle.propagate(u.astype(np.complex128), (my, mx), dx, lam, z, out_mode=out_mode)
    assert got.shape == want.shape
    assert_close(got, want, FIELD_TOL, FIELD_ELEM)


@pytest.mark.parametrize("my,mx,ny,nx", [(720, 240, 360, 120), (240, 2144, 200, 1500),
                                         (2144, 2144, 1000, 1072)])
def test_rect_psf_and_backward(api, my, mx, ny, nx):
    print(f"rect psf/backward {my}x{mx}", flush=True)
    dx, z = 0.5, 1500.0
    lams = np.array([0.45, 0.55, 0.65])
    nidx = wl.cauchy_index(lams)
    w = np.array([1.0, 0.5, 2.0], dtype=np.float32)
    rng = np.random.default_rng(my + mx)
    h = wl.uniform_heights((ny, nx), seed=my)
    amp = rng.uniform(0.5, 1.0, (ny, nx)).astype(np.float32)
    g = rng.standard_normal((ny, nx)).astype(np.float32)
    prob = api.Problem((ny, nx), (my, mx), dx, z, lams, nidx, weights=w)
    hd, ad = dev(h, torch.float32), dev(amp, torch.float32)
    got, saved = api.psf(hd, prob, amp=ad, save_fields=True)
    want = oracle.psf(h, dx, z, (my, mx), lams, nidx, weights=w, amp=amp)
    assert_close(got.cpu().numpy(), want, INTENSITY_TOL, INTENSITY_ELEM)
    gh = api.psf_backward(hd, prob, saved, dev(g, torch.float32), amp=ad).cpu().numpy()
    want_g = oracle.psf_backward(h, dx, z, (my, mx), lams, nidx, g, weights=w, amp=amp)
    assert_close(gh, want_g, GRAD_TOL, GRAD_ELEM)


@pytest.mark.parametrize("my,mx,ny,nx,z", [(5360, 240, 2000, 200, 4000.0),
                                           (512, 2048, 256, 1024, -2500.0)])
def test_rect_full_output_and_bandlimit(api, my, mx, ny, nx, z):
    """Band-limited ASM on a rectangular grid: each axis is cut at the limit
    of its own length (f_lim differs between the axes here)."""
    dx, lam = 0.5, 0.5
    h = wl.uniform_heights((ny, nx), seed=78)
    prob = api.Problem((ny, nx), (my, mx), dx, z, [lam], [1.46], out_mode="full", bandlimit=True)
    got = api.psf(dev(h, torch.float32), prob).cpu().numpy()
    want = oracle.psf(h, dx, z, (my, mx), [lam], [1.46], out_mode="full", bandlimit=True)
    assert got.shape == (my, mx)
    assert_close(got, want, INTENSITY_TOL, INTENSITY_ELEM)


def test_rect_fused_nearest_upsampling(api):
    """4x nearest upsampling of a 100 x 50 design inside the first pass on the
    720 x 240 grid: PSF and coarse gradient against the oracle chain."""
    s, my, mx, dx, z = 4, 720, 240, 0.5, 800.0
    hc = np.random.default_rng(79).uniform(0, 1.2, (100, 50)).astype(np.float32)
    hf = np.kron(hc, np.ones((s, s), dtype=np.float32))
    ny, nx = hf.shape
    lams = np.array([0.5, 0.6])
    nidx = wl.cauchy_index(lams)
    g = np.random.default_rng(80).standard_normal((ny, nx)).astype(np.float32)
    prob = api.Problem((ny, nx), (my, mx), dx, z, lams, nidx, upsample=s)
    assert prob.h_shape == (100, 50)
    hd = dev(hc, torch.float32)
    got, saved = api.psf(hd, prob, save_fields=True)
    assert_close(got.cpu().numpy(), oracle.psf(hf, dx, z, (my, mx), lams, nidx), INTENSITY_TOL, INTENSITY_ELEM)
    gc = api.psf_backward(hd, prob, saved, dev(g, torch.float32)).cpu().numpy()
    want = oracle.psf_backward(hf, dx, z, (my, mx), lams, nidx, g)
    want_c = want.reshape(100, s, 50, s).sum(axis=(1, 3))
    assert gc.shape == (100, 50)
    assert_close(gc, want_c, GRAD_TOL, GRAD_ELEM)


@pytest.mark.timeout(300)
def test_rect_paper_digit_split_whole_psf(api):
    """16080 x 10720: the paper's 128,640 x 85,760 digit structure (x: 670 x
    BX, y: AY x 1005) with BX = AY = 16.  Whole PSF of an 8040 x 5360 DOE, 2
    wavelengths, against the FP64 oracle."""
    my, mx, ny, nx, dx, z = 16080, 10720, 8040, 5360, 0.5, 20000.0
    lams = np.array([0.5206, 0.62])
    nidx = wl.cauchy_index(lams)
    h = wl.uniform_heights((ny, nx), seed=81)
    prob = api.Problem((ny, nx), (my, mx), dx, z, lams, nidx)
    got = api.psf(dev(h, torch.float32), prob).double().cpu().numpy()
    torch.cuda.empty_cache()
    want = oracle.psf(h, dx, z, (my, mx), lams, nidx)
    assert_close(got, want, 1e-4, 1e-4)
    assert abs(got.sum() / want.sum() - 1) < 1e-5
