"""Gradient-based DOE design on the HIP path (the paper's Eq. 5 objective with
the fabrication model left out, i.e. the conventional-design objective of
Sec. 3.1 with an L2 PSF loss).

h* = argmin_h mean((sum_k |E_dest,k(h)|^2 - T)^2), solved with Adam and a
cosine learning-rate decay to zero (the schedule shape of Sec. 3.2's toy
example).  Forward and backward run in libdop (DopPSF); torch only holds the
parameter and optimiser state.

Checkpoint / resume: every `checkpoint_every` steps the loop writes the
height map, the Adam and schedule state, the step count and the loss history
to `checkpoint` (torch.save of tensors and plain containers, readable with
weights_only=True).  The kernels are deterministic (fixed wavelength order,
no floating-point atomics), so a run resumed from a checkpoint continues the
same trajectory bit for bit.
"""

import math
import os
import time

import torch

from . import api


def _sync(t):
    if t.is_cuda:
        torch.cuda.synchronize(t.device)


def _save(path, h, opt, sched, step, losses):
    state = {"h": h.detach().clone(), "opt": opt.state_dict(), "sched": sched.state_dict(),
             "step": step, "losses": torch.stack(losses).cpu() if losses else torch.zeros(0)}
    tmp = path + ".tmp"
    torch.save(state, tmp)
    os.replace(tmp, path)  # a crash mid-write leaves the previous checkpoint whole


def design_loop(h0, prob, target, steps=200, lr=1e-2, amp=None, log_every=0, log=print,
                checkpoint=None, checkpoint_every=0, resume=False, psf_fn=None):
    """Run Adam steps on the height map up to step `steps`.  Returns (h,
    losses, seconds per step run here).

    checkpoint / checkpoint_every: write the state every that many steps and
    after the last one.  resume: start from `checkpoint` if it exists (h0 then
    only gives the dtype and device).  psf_fn(h, prob, amp): the forward
    model, by default the library's DopPSF."""
    psf_fn = psf_fn or api.DopPSF.apply
    h = h0.detach().clone().requires_grad_(True)
    opt = torch.optim.Adam([h], lr=lr)
    sched = torch.optim.lr_scheduler.LambdaLR(
        opt, lambda s: 0.5 * (1.0 + math.cos(math.pi * min(s, steps) / steps)))
    start, losses = 0, []
    if resume and checkpoint and os.path.exists(checkpoint):
        state = torch.load(checkpoint, map_location=h0.device, weights_only=True)
        with torch.no_grad():
            h.copy_(state["h"])
        opt.load_state_dict(state["opt"])
        sched.load_state_dict(state["sched"])
        start = int(state["step"])
        losses = [x.to(h0.device) for x in state["losses"]]
    _sync(h)
    t0 = time.perf_counter()
    for step in range(start, steps):
        opt.zero_grad(set_to_none=True)
        psf = psf_fn(h, prob, amp)
        loss = torch.mean((psf - target) ** 2)
        loss.backward()
        opt.step()
        sched.step()
        losses.append(loss.detach())
        if log_every and (step % log_every == 0 or step == steps - 1):
            log(f"design step {step}: loss {loss.item():.6g}")
        if checkpoint and checkpoint_every and ((step + 1) % checkpoint_every == 0
                                                or step + 1 == steps):
            _save(checkpoint, h, opt, sched, step + 1, losses)
    _sync(h)
    dt = (time.perf_counter() - t0) / max(steps - start, 1)
    return h.detach(), [float(x) for x in torch.stack(losses).cpu()] if losses else [], dt
