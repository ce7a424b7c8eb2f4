"""dop_psf_noalloc (the PSF entry point that allocates nothing: its workspace
is the library's static device scratch) against dop_psf, through the C ABI.

Two calls in a row, the second with a smaller problem (so it runs on what
the first left in the scratch): each result is bitwise dop_psf's on the
same inputs, and matches the FP64 oracle.  A grid whose workspace exceeds
the scratch is rejected before anything is enqueued, leaving the output
untouched.
"""

import ctypes
import os

import numpy as np
import pytest

import oracle
from oracle import asm
from paper_2505_22313_amd import workloads as wl
from _close import assert_close, FIELD_ELEM, INTENSITY_ELEM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

asm.WORKERS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_22313_amd import api as _api
    return _api


def _noalloc(api, prob, h, amp, out, saved):
    from paper_2505_22313_amd import _lib as L
    ctx = api.default_context(0)
    p = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())  # noqa: E731
    stream = ctypes.c_void_p(torch.cuda.current_stream(0).cuda_stream)
    return L.lib().dop_psf_noalloc(ctx.handle, prob.ptr(), p(h), p(amp), p(out), p(saved), stream)


def test_noalloc_matches_dop_psf_twice_then_smaller(api):
    from paper_2505_22313_amd import _lib as L
    # call 1: the largest grid the scratch holds (2048^2 DOE on 4096^2),
    # 3 wavelengths with weights and an aperture, fields saved
    n1, m1 = 2048, 4096
    lams1 = np.array([0.45, 0.55, 0.65])
    w1 = np.array([1.0, 0.5, 2.0], dtype=np.float32)
    prob1 = api.Problem(n1, m1, 1.0, 8000.0, lams1, wl.cauchy_index(lams1), weights=w1)
    h1 = wl.uniform_heights(n1, seed=71)
    amp1 = wl.circular_aperture(n1, 1.0, 900.0)
    # call 2: smaller, full plane, 5 wavelengths (a group of four, then one)
    n2, m2 = 300, 1024
    lams2 = np.linspace(0.40, 0.70, 5)
    prob2 = api.Problem(n2, m2, 0.5, 1500.0, lams2, wl.cauchy_index(lams2), out_mode="full")
    h2 = wl.uniform_heights(n2, seed=72)
    assert api.workspace_size(prob1) <= L.DOP_NOALLOC_MAX_BYTES

    hd1, ad1 = torch.from_numpy(h1).cuda(), torch.from_numpy(amp1).cuda()
    hd2 = torch.from_numpy(h2).cuda()
    out1 = torch.full(prob1.out_shape, float("nan"), device="cuda")
    saved1 = torch.empty((3, n1, n1), dtype=torch.complex64, device="cuda")
    out2 = torch.full(prob2.out_shape, float("nan"), device="cuda")
    torch.cuda.synchronize()
    assert _noalloc(api, prob1, hd1, ad1, out1, saved1) == L.DOP_OK
    assert _noalloc(api, prob2, hd2, None, out2, None) == L.DOP_OK
    torch.cuda.synchronize()

    ref1, rsaved1 = api.psf(hd1, prob1, amp=ad1, save_fields=True)
    ref2 = api.psf(hd2, prob2)
    torch.cuda.synchronize()
    assert torch.equal(out1, ref1) and torch.equal(saved1, rsaved1)
    assert torch.equal(out2, ref2)

    want1, fields1 = oracle.psf(h1, 1.0, 8000.0, m1, lams1, prob1.n_index, weights=w1, amp=amp1,
                                return_fields=True)
    assert_close(out1.cpu().numpy(), want1, 2e-5, INTENSITY_ELEM, "call 1 PSF")
    assert_close(saved1[1].cpu().numpy(), fields1[1], 1e-5, FIELD_ELEM, "call 1 field")
    want2 = oracle.psf(h2, 0.5, 1500.0, m2, lams2, prob2.n_index, out_mode="full")
    assert_close(out2.cpu().numpy(), want2, 2e-5, INTENSITY_ELEM, "call 2 PSF")


def test_noalloc_rejects_grids_beyond_the_scratch(api):
    from paper_2505_22313_amd import _lib as L
    prob = api.Problem(4096, 8192, 1.0, 8000.0, [0.55], [1.46])
    assert api.workspace_size(prob) > L.DOP_NOALLOC_MAX_BYTES
    h = torch.zeros((4096, 4096), device="cuda")
    out = torch.full((4096, 4096), 7.0, device="cuda")
    torch.cuda.synchronize()
    assert _noalloc(api, prob, h, None, out, None) == L.DOP_ERR_WORKSPACE
    assert "scratch" in L.last_error()
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))
