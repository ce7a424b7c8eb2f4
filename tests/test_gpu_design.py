"""Differentiable design at the design workload's size (8192^2 heights,
3 wavelengths, z = 20 mm, padded to 16384^2): the hand-written adjoint
against the FP64 oracle gradient, and a 200-step Adam run that lowers the
loss."""

import os

import numpy as np
import pytest

import oracle
from oracle import asm
from paper_2505_22313_amd import workloads as wl
from _close import errors, GRAD_ELEM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

asm.WORKERS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_22313_amd import api
    p = wl.problem("design")
    h = wl.heights("design")
    n = p["n"]
    target = wl.gaussian_target(n, 3.0, total=len(p["lams"]) * float(n) * n)
    return api, p, h, target


@pytest.mark.timeout(900)
def test_design_gradient_vs_oracle(setup):
    api, p, h, target = setup
    n = p["n"]
    prob = api.Problem.from_dict(p)
    hd = torch.from_numpy(h).cuda().requires_grad_(True)
    td = torch.from_numpy(target).cuda()
    loss = torch.mean((api.DopPSF.apply(hd, prob) - td) ** 2)
    loss.backward()
    got = hd.grad.cpu().numpy()
    torch.cuda.synchronize()
    print("  oracle forward", flush=True)
    ps = oracle.psf(h, p["dx"], p["z"], p["m"], p["lams"], p["n_index"])
    g = 2.0 * (ps - target) / (float(n) * n)
    print("  oracle gradient", flush=True)
    want = oracle.psf_backward(h, p["dx"], p["z"], p["m"], p["lams"], p["n_index"], g)
    err, el = errors(got, want)
    print(f"  gradient rel-L2 {err:.3e}, max|err|/max {el:.3e}", flush=True)
    assert err < 1e-4 and el < GRAD_ELEM
    assert abs(loss.item() / np.mean((ps - target) ** 2) - 1) < 1e-5


@pytest.mark.timeout(600)
def test_design_adam_200_steps(setup):
    api, p, h, target = setup
    from paper_2505_22313_amd.design import design_loop
    prob = api.Problem.from_dict(p)
    hd = torch.from_numpy(h).cuda()
    td = torch.from_numpy(target).cuda()
    _, losses, dt = design_loop(hd, prob, td, steps=200, lr=1e-2)
    print(f"  loss {losses[0]:.4g} -> {losses[-1]:.4g}, {dt * 1e3:.1f} ms/step", flush=True)
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0]


def test_design_on_coarse_upsampled_grid(setup):
    """Design on a coarse grid simulated 8x finer (the paper's conventional
    design with nearest upsampling): Adam on the 128^2 design lowers the
    loss, and the design keeps its coarse shape."""
    api = setup[0]
    from paper_2505_22313_amd.design import design_loop
    nc, s, m = 128, 8, 2048
    n = nc * s
    lams = np.array([0.5206])
    prob = api.Problem(n, m, 0.25, 2000.0, lams, wl.cauchy_index(lams), upsample=s)
    h0 = torch.from_numpy(wl.uniform_heights(nc, seed=5)).cuda()
    target = torch.from_numpy(wl.gaussian_target(n, 4.0, total=float(n) * n)).cuda()
    h, losses, _ = design_loop(h0, prob, target, steps=60, lr=2e-2)
    assert tuple(h.shape) == (nc, nc)
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.7 * losses[0]


def test_design_resume_is_bitwise(setup, tmp_path):
    """Checkpoint / resume on the library path: 3 steps, a checkpoint, a
    fresh loop resumed from it for 3 more, against 6 uninterrupted steps."""
    api = setup[0]
    from paper_2505_22313_amd.design import design_loop
    n, m = 256, 512
    lams = np.array([0.45, 0.55, 0.65])
    prob = api.Problem(n, m, 1.0, 20000.0, lams, wl.cauchy_index(lams))
    h0 = torch.from_numpy(wl.uniform_heights(n, seed=9)).cuda()
    target = torch.from_numpy(wl.gaussian_target(n, 3.0, total=3.0 * n * n)).cuda()
    h_ref, l_ref, _ = design_loop(h0, prob, target, steps=6, lr=1e-2)
    ck = str(tmp_path / "design.pt")

    calls = {"n": 0}

    def stop_after_3(h, p, a):
        if calls["n"] == 3:
            raise KeyboardInterrupt
        calls["n"] += 1
        return api.DopPSF.apply(h, p, a)

    with pytest.raises(KeyboardInterrupt):
        design_loop(h0, prob, target, steps=6, lr=1e-2, psf_fn=stop_after_3, checkpoint=ck,
                    checkpoint_every=1)
    h, losses, _ = design_loop(h0, prob, target, steps=6, lr=1e-2, checkpoint=ck,
                               checkpoint_every=1, resume=True)
    assert torch.equal(h, h_ref)
    assert losses == l_ref
