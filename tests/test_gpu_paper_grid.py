"""The paper's largest grid on one MI355X: a 32.16 mm x 21.44 mm DOE at
0.5 um (64,320 rows x 42,880 columns) padded to 128,640 x 85,760 (Table 2,
the large-area hologram designs the paper ran on 16 A100s; an 88 GB
workspace here).  Its axes carry the prime factor 67 (128,640 = 2^7 3 5 67,
85,760 = 2^8 5 67).  Checked: the paper's own upsampled design problem
against an FP64 oracle golden (12 whole PSF rows, total and peak; the
oracle needs about 200 GB of host memory, so the golden is written once by
tests/golden/make_paper_grid_golden.py), and properties that hold at any
size and pin every pass: z = 0 is the identity, Parseval on the full plane,
and the focus of an ideal lens against the exact on-axis Rayleigh-Sommerfeld
value and the sinc^2 profile of the rectangular pupil along both axes.
"""

import numpy as np
import pytest

from paper_2505_22313_amd import workloads as wl
from _close import errors, INTENSITY_ELEM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NY, NX, MY, MX, DX = 64320, 42880, 128640, 85760, 0.5


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_22313_amd import api as _api
    free(_api)
    yield _api
    free(_api)


def free(api):
    api.default_context(0).release_workspaces()
    torch.cuda.empty_cache()


def test_paper_grid_z0_identity(api):
    print("paper grid: z = 0", flush=True)
    gen = torch.Generator(device="cuda").manual_seed(50)
    u = torch.randn((NY, NX), generator=gen, device="cuda", dtype=torch.complex64)
    prob = api.Problem((NY, NX), (MY, MX), DX, 0.0, [0.5206], [1.5])
    out = api.propagate(u, prob)
    err = float(torch.linalg.vector_norm((out - u).flatten()).item()
                / torch.linalg.vector_norm(u.flatten()).item())
    assert err < 2e-6
    del u, out
    free(api)


def test_paper_grid_parseval_full_plane(api):
    """Every bin propagates at 520.6 nm with 0.5 um pitch (s_max = 0.54): the
    whole 128,640 x 85,760 PSF of a unit-modulus DOE sums to Ny Nx."""
    print("paper grid: Parseval", flush=True)
    gen = torch.Generator(device="cuda").manual_seed(51)
    h = torch.rand((NY, NX), generator=gen, device="cuda") * 1.2
    prob = api.Problem((NY, NX), (MY, MX), DX, 60000.0, [0.5206], wl.cauchy_index([0.5206]),
                       out_mode="full")
    full = api.psf(h, prob)
    assert tuple(full.shape) == (MY, MX)
    del h
    free(api)
    tot = sum(float(full[r0:r0 + 8192].sum(dtype=torch.float64).item()) for r0 in range(0, MY, 8192))
    assert abs(tot / (float(NY) * NX) - 1.0) < 1e-5
    del full
    free(api)


def test_paper_grid_lens_focus(api):
    """Ideal lens f = z = 100 mm wrapped at 550 nm over the whole 32.16 x
    21.44 mm aperture: the peak equals the exact scalar on-axis amplitude
    (f/lambda) sum dA/(rho^2 + f^2) (Goodman), and the focal spot is
    sinc^2(Lx x/(lambda f)) along x and sinc^2(Ly y/(lambda f)) along y, each
    with its own width."""
    print("paper grid: lens focus", flush=True)
    lam, f = 0.55, 100000.0
    h = torch.from_numpy(wl.fresnel_lens_heights((NY, NX), DX, f)).cuda()
    prob = api.Problem((NY, NX), (MY, MX), DX, f, [lam], wl.cauchy_index([lam]))
    p = api.psf(h, prob)
    cy, cx = NY // 2, NX // 2
    ycoord = (np.arange(NY) - cy) * DX
    xcoord = (np.arange(NX) - cx) * DX
    acc = 0.0
    for r0 in range(0, NY, 1024):
        y = ycoord[r0:r0 + 1024][:, None]
        acc += np.sum(1.0 / (y * y + xcoord[None, :] ** 2 + f * f))
    i_rs = (f / lam * acc * DX * DX) ** 2
    win = p[cy - 8:cy + 9, cx - 8:cx + 9].double().cpu().numpy()
    assert abs(win[8, 8] / i_rs - 1) < 1e-3
    assert np.unravel_index(np.argmax(win), win.shape) == (8, 8)
    t = np.arange(-8, 9) * DX
    assert np.max(np.abs(win[8, :] / win[8, 8] - np.sinc(NX * DX * t / (lam * f)) ** 2)) < 0.02
    assert np.max(np.abs(win[:, 8] / win[8, 8] - np.sinc(NY * DX * t / (lam * f)) ** 2)) < 0.02
    # the widths differ: the x profile is wider than the y profile
    assert win[8, 10] > win[10, 8]
    del h, p
    free(api)


def test_paper_grid_psf_rows_vs_oracle(api):
    """The paper's own large-area problem at full size against the FP64
    oracle: a seeded 16,080 x 10,720 design at 2 um, 4x nearest upsampling
    fused into the first pass, the 128,640 x 85,760 grid, 520.6 nm, z = 60 mm.
    12 whole PSF rows (rel-L2 <= 1e-4), the crop's total (1e-5) and peak
    (1e-4) against tests/golden/psf_paper_grid_rows.npz, which
    make_paper_grid_golden.py writes with the oracle alone."""
    import os
    print("paper grid: rows vs oracle golden", flush=True)
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "psf_paper_grid_rows.npz"))
    ncy, ncx, s = int(g["ncy"]), int(g["ncx"]), int(g["s"])
    assert (ncy * s, ncx * s, int(g["my"]), int(g["mx"])) == (NY, NX, MY, MX)
    hc = torch.from_numpy(wl.uniform_heights((ncy, ncx), seed=int(g["seed"]))).cuda()
    prob = api.Problem((NY, NX), (MY, MX), float(g["dx"]), float(g["z"]), [float(g["lam"])],
                       [float(g["n_index"])], upsample=s)
    p = api.psf(hc, prob)
    rows = torch.from_numpy(g["rows"]).cuda()
    got = p[rows].double().cpu().numpy()
    want = g["psf_rows"].astype(np.float64)
    err, el = errors(got, want)
    total = sum(float(p[r0:r0 + 8192].sum(dtype=torch.float64).item()) for r0 in range(0, NY, 8192))
    peak = float(p.max().item())
    print(f"  rows rel-L2 {err:.3e}, max|err|/max {el:.3e}, total {total / float(g['total']) - 1:.2e}, "
          f"peak {peak / float(g['peak']) - 1:.2e}", flush=True)
    assert err < 1e-4 and el < INTENSITY_ELEM
    assert abs(total / float(g["total"]) - 1) < 1e-5
    assert abs(peak / float(g["peak"]) - 1) < 1e-4
    del hc, p
    free(api)
