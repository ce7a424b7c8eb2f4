"""FP64 CPU oracle for FFT-based angular-spectrum (ASM) propagation of a DOE.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
definition that the HIP library is checked against.  Only the test suite, the
smoke check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may
import it.  The product package never imports it, and it imports nothing from
the product package: the two share no code.

Parity status per function (see the module docstrings for the passages):

* ``doe_field``, ``embed``, ``transfer_function``, ``propagate_padded``,
  ``propagate``, ``psf``, ``psf_backward``: pinned (brute-force DFT on tiny
  grids, Parseval, z = 0, +-z round trip, plane-wave eigenfunction,
  sinc^2 / Airy lens focus, finite differences, adjoint dot product).
* rectangular grids (``m`` = (My, Mx), DOE Ny x Nx) in all of the above:
  pinned (matrix DFT, per-bin brute-force sums, Parseval, z = 0, +-z round
  trip, the rectangular pupil's focal spot with its two widths, the per-axis
  band limit, the gradient against finite differences).
* ``psf_lowmem`` (one wavelength, blocked for memory): pinned to ``psf`` at
  small sizes (same values to rounding), and through it to the pins above.
* ``band_limit`` and the ``bandlimit`` option: pinned (reduces to plain ASM
  beyond Nyquist, per-bin mask, aliasing removed against a finer grid).
* ``upsample.upsample``, ``upsample.upsample_adjoint``: pinned (block
  repetition, closed-form kernel values, interpolation at odd factors,
  partition of unity, slow cosines, adjoint dot product).
"""

from .asm import (  # noqa: F401
    band_limit,
    brute_propagate,
    crop,
    direct_dft2,
    doe_field,
    embed,
    grid_shape,
    pad_offset,
    propagate,
    propagate_padded,
    psf,
    psf_backward,
    psf_lowmem,
    transfer_function,
    transfer_rows,
)
from . import upsample  # noqa: F401
