"""Checkpoint / resume of the design loop on the CPU: a run interrupted and
resumed from its checkpoint reproduces the uninterrupted run bit for bit
(height map and loss history), and the checkpoint loads with
weights_only=True.  The forward model here is a small differentiable torch
stand-in (|FFT of a phase screen|^2), passed through design_loop's psf_fn
hook, so no GPU is needed; the same loop on the library's DopPSF is checked
in test_gpu_design.py."""

import os

import pytest

torch = pytest.importorskip("torch")

from paper_2505_22313_amd.design import design_loop


def _toy_psf(h, prob, amp):
    m = prob
    u = torch.polar(torch.ones_like(h), 2 * torch.pi * h)
    spec = torch.fft.fft2(u, s=(m, m))
    return (spec.real ** 2 + spec.imag ** 2)[: h.shape[0], : h.shape[1]] / m ** 2


def _setup():
    g = torch.Generator().manual_seed(3)
    h0 = torch.rand((16, 16), generator=g, dtype=torch.float64)
    target = torch.rand((16, 16), generator=g, dtype=torch.float64)
    return h0, 32, target


def test_resume_reproduces_the_uninterrupted_run(tmp_path):
    h0, prob, target = _setup()
    h_ref, l_ref, _ = design_loop(h0, prob, target, steps=8, lr=5e-2, psf_fn=_toy_psf)
    ck = str(tmp_path / "design.pt")
    # first leg: the same schedule (steps=8), stopped after 5 steps by the
    # caller, checkpointing every step
    class Stop(Exception):
        pass

    calls = {"n": 0}

    def stopping_psf(h, p, a):
        if calls["n"] == 5:
            raise Stop()
        calls["n"] += 1
        return _toy_psf(h, p, a)

    with pytest.raises(Stop):
        design_loop(h0, prob, target, steps=8, lr=5e-2, psf_fn=stopping_psf, checkpoint=ck,
                    checkpoint_every=1)
    state = torch.load(ck, weights_only=True)
    assert state["step"] == 5 and len(state["losses"]) == 5
    assert not os.path.exists(ck + ".tmp")
    # second leg: resume from a different starting point (ignored)
    h, losses, _ = design_loop(torch.zeros_like(h0), prob, target, steps=8, lr=5e-2,
                               psf_fn=_toy_psf, checkpoint=ck, checkpoint_every=2, resume=True)
    assert torch.equal(h, h_ref)
    assert losses == l_ref
    assert torch.load(ck, weights_only=True)["step"] == 8


def test_resume_without_a_checkpoint_starts_fresh(tmp_path):
    h0, prob, target = _setup()
    h_ref, l_ref, _ = design_loop(h0, prob, target, steps=4, lr=5e-2, psf_fn=_toy_psf)
    h, losses, _ = design_loop(h0, prob, target, steps=4, lr=5e-2, psf_fn=_toy_psf,
                               checkpoint=str(tmp_path / "none.pt"), resume=True)
    assert torch.equal(h, h_ref) and losses == l_ref
