"""Wavelength groups (dop_psf with a workspace of several fields): pass A
forms up to four fields from one read of the heights and pass A' adds their
intensities to the PSF in one read-modify-write.  The sums are the same, in
the same order, as one wavelength at a time, so the PSF must be bitwise
identical; checked over wavelength counts that leave partial groups, square,
non-power-of-two and rectangular grids, CROP and FULL, weights, amp, the band
limit and the fused upsampling, plus a grid whose pass A' ends in a radix-67
stage (no grouping there).  The launch counts show the grouping.  Square
power-of-two grids up to 2048 run the three-pass small-grid path, which does
not group wavelengths: there both calls run the same passes."""

import numpy as np
import pytest

from paper_2505_22313_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_22313_amd import api as _api
    yield _api
    _api.default_context(0).release_workspaces()
    torch.cuda.empty_cache()


CASES = [
    # (n, m, k, out_mode, bandlimit, upsample, amp)
    (512, 1024, 1, "crop", False, 1, False),
    (512, 1024, 2, "crop", False, 1, True),
    (500, 1024, 5, "full", False, 1, False),
    (512, 1024, 7, "crop", True, 4, False),
    (360, 720, 4, "crop", False, 1, True),
    ((300, 200), (720, 240), 6, "full", True, 1, False),
    ((200, 1000), (512, 2048), 9, "crop", False, 1, True),
    ((200, 1500), (240, 2144), 3, "crop", False, 1, False),   # radix 67 in x: no grouping
]


@pytest.mark.parametrize("n,m,k,mode,bl,up,amp", CASES)
def test_grouped_psf_is_bitwise_per_wavelength(api, n, m, k, mode, bl, up, amp):
    ny, nx = (n, n) if np.ndim(n) == 0 else n
    lams = np.linspace(0.42, 0.68, k)
    w = np.linspace(0.5, 1.5, k).astype(np.float32)
    prob = api.Problem(n, m, 0.5, 1200.0, lams, wl.cauchy_index(lams), weights=w, out_mode=mode,
                       bandlimit=bl, upsample=up)
    h = torch.from_numpy(wl.uniform_heights(prob.h_shape, seed=k)).cuda()
    a = None
    if amp:
        a = torch.from_numpy(np.random.default_rng(k).uniform(0.3, 1.0, (ny, nx))
                             .astype(np.float32)).cuda()
    ctx = api.default_context(0)
    ctx.release_workspaces()
    one = api.psf(h, prob, amp=a, group=1)
    ctx.profile_enable(True)
    grouped = api.psf(h, prob, amp=a, group=4)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    assert torch.equal(one, grouped)
    # square power-of-two grids up to 2048 take the three-pass small-grid
    # path, one wavelength at a time; the radix-67 grid is not grouped either
    small = np.ndim(m) == 0 and m <= 2048 and m & (m - 1) == 0
    groups = k if small or nx in (1500,) else -(-k // 4)
    assert prof["pass_a_fwd"][0] == groups and prof["pass_a_inv"][0] == groups
    assert prof["pass_c"][0] == k
