"""Comparison of a HIP result with the FP64 oracle's.

Two bounds, both required:
  - rel-L2 = ||got - want||_2 / ||want||_2 over the returned array (the
    error metric of the paper-reading list), and
  - a per-element bound, max |got - want| / max |want|, so that a defect
    confined to a few elements (one bad tile, the Nyquist row or column, the
    evanescent rim, one member of a wavelength group) cannot hide inside a
    small L2 error over millions of good ones.

Per-element bounds: complex fields 1e-5 and intensities 1e-4 (the stated
FP32-butterfly tolerances: field 1e-5 at 4096^2, intensity 1e-4 at 65536^2);
gradients 1e-4, as their rel-L2 bound.
"""

import numpy as np

FIELD_ELEM = 1e-5
INTENSITY_ELEM = 1e-4
GRAD_ELEM = 1e-4


def _as_np(x):
    if hasattr(x, "detach"):  # a torch tensor
        x = x.detach().cpu().numpy()
    x = np.asarray(x)
    return x.astype(np.complex128 if np.iscomplexobj(x) else np.float64)


def errors(got, want):
    """(rel-L2, max |got - want| / max |want|) of two arrays of one shape."""
    g, w = _as_np(got), _as_np(want)
    assert g.shape == w.shape, f"shape {g.shape} != {w.shape}"
    d = g - w
    l2 = float(np.linalg.norm(d.ravel()) / np.linalg.norm(w.ravel()))
    el = float(np.max(np.abs(d)) / np.max(np.abs(w)))
    return l2, el


def assert_close(got, want, l2_tol, elem_tol, what="result"):
    l2, el = errors(got, want)
    assert l2 <= l2_tol and el <= elem_tol, (
        f"{what}: rel-L2 {l2:.3e} (bound {l2_tol:g}), max|err|/max|ref| {el:.3e} "
        f"(bound {elem_tol:g})")
    return l2, el
