"""The five-pass plans between the oracle-checked sizes and the 65536^2
goldens: 8192^2, 16384^2 and 32768^2 grids (the serving workload's N = 4096,
8192 and 16384 requests).  Properties that hold at any size pin every pass:
z = 0 is the identity (forward and inverse transforms, the phase-free H = 1),
and with every bin propagating the full-plane PSF of a unit-modulus DOE sums
to N^2 (Parseval through the whole chain, any defect in a tile, a twiddle or
the transfer function's modulus shows)."""

import pytest

from paper_2505_22313_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GRIDS = [8192, 16384, 32768]


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_22313_amd import api as _api
    yield _api
    _api.default_context(0).release_workspaces()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("m", GRIDS)
def test_z0_identity(api, m):
    n = m // 2
    gen = torch.Generator(device="cuda").manual_seed(m)
    u = torch.randn((n, n), generator=gen, device="cuda", dtype=torch.complex64)
    prob = api.Problem(n, m, 0.5, 0.0, [0.55], [1.5])
    out = api.propagate(u, prob)
    err = float(torch.linalg.vector_norm((out - u).flatten()).item()
                / torch.linalg.vector_norm(u.flatten()).item())
    assert err < 2e-6


@pytest.mark.parametrize("m", GRIDS)
def test_parseval_full_plane(api, m):
    """700 nm at 0.5 um pitch: s_max = 2 (0.7 / 1.0)^2 = 0.98 < 1, so every
    bin propagates and |H| = 1; three wavelengths in one group."""
    n = m // 2
    gen = torch.Generator(device="cuda").manual_seed(m + 1)
    h = torch.rand((n, n), generator=gen, device="cuda") * 1.2
    lams = [0.60, 0.65, 0.70]
    w = [0.5, 1.0, 2.0]
    prob = api.Problem(n, m, 0.5, 20000.0, lams, wl.cauchy_index(lams), weights=w,
                       out_mode="full")
    full = api.psf(h, prob)
    tot = float(full.sum(dtype=torch.float64).item())
    assert abs(tot / (sum(w) * float(n) * n) - 1.0) < 1e-5
    # the PSF is non-negative and not concentrated in a few bins
    assert float(full.min().item()) >= 0.0
    assert float(full.max().item()) < 1e-3 * tot
