"""Gradient-based DOE design on the HIP path (the paper's Eq. 5 objective with
the fabrication model left out, i.e. the conventional-design objective of
Sec. 3.1 with an L2 PSF loss).

h* = argmin_h mean((sum_k |E_dest,k(h)|^2 - T)^2), solved with Adam and a
cosine learning-rate decay to zero (the schedule shape of Sec. 3.2's toy
example).  Forward and backward run in libdop (DopPSF); torch only holds the
parameter and optimiser state.
"""

import math
import time

import torch

from . import api


def design_loop(h0, prob, target, steps=200, lr=1e-2, amp=None, log_every=0, log=print):
    """Run `steps` Adam steps on the height map.  Returns (h, losses,
    seconds per step)."""
    h = h0.detach().clone().requires_grad_(True)
    opt = torch.optim.Adam([h], lr=lr)
    sched = torch.optim.lr_scheduler.LambdaLR(
        opt, lambda s: 0.5 * (1.0 + math.cos(math.pi * min(s, steps) / steps)))
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(steps):
        opt.zero_grad(set_to_none=True)
        psf = api.DopPSF.apply(h, prob, amp)
        loss = torch.mean((psf - target) ** 2)
        loss.backward()
        opt.step()
        sched.step()
        losses.append(loss.detach())
        if log_every and (step % log_every == 0 or step == steps - 1):
            log(f"design step {step}: loss {loss.item():.6g}")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    return h.detach(), [float(x) for x in torch.stack(losses).cpu()], dt
