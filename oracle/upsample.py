"""FP64 oracle of the super-resolved DOE front end (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module; the product library never does.

The paper designs on a coarse feature grid and simulates the DOE on a grid s
times finer (Sec. 3.2 and its Table 2: 2 um features on a 250 nm grid, i.e.
8x, and on a 500 nm grid, 4x), filling the fine grid from the coarse design
by an interpolation kernel: nearest neighbour, which forces box-shaped
features, or a smooth Lanczos-3 kernel (Getreuer, "Linear Methods for Image
Interpolation", IPOL 2011).  Both are linear maps U from the coarse map
(ncy x ncx) to the fine one (ncy*s x ncx*s), separable over the two axes:
h_fine = Wy hc Wx^T with one-axis matrices W of shape (nc*s, nc), one per
axis length (Wy = Wx on a square design).

* Nearest: fine sample j takes coarse sample floor(j / s).
* Lanczos-3: fine sample j sits at coarse coordinate u_j = (j + 0.5)/s - 0.5
  (pixel centres aligned); its taps are the coarse samples i with
  |u_j - i| < 3, weighted by L(u_j - i), L(x) = sinc(x) sinc(x/3) (normalised
  sinc).  Taps outside [0, nc) are dropped and each row of W is divided by
  the sum of its remaining weights, so a constant map stays constant.

The design gradient needs the adjoint U^T: Wy^T g Wx (for nearest, the sum
of each s x s block).

Parity status: pinned (block repetition, interpolation of coarse samples at
odd s, partition of unity, reproduction of slowly varying cosines, mirror
symmetry, the kernel's closed-form values, adjoint dot-product identity).
"""

import numpy as np


def lanczos3(x):
    """L(x) = sinc(x) * sinc(x / 3) for |x| < 3, else 0 (normalised sinc)."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(np.abs(x) < 3.0, np.sinc(x) * np.sinc(x / 3.0), 0.0)


def axis_matrix(nc, s, kind):
    """One-axis interpolation matrix W, shape (nc*s, nc), float64."""
    nf = nc * s
    j = np.arange(nf)
    w = np.zeros((nf, nc))
    if kind == "nearest":
        w[j, j // s] = 1.0
        return w
    if kind != "lanczos3":
        raise ValueError(kind)
    u = (j + 0.5) / s - 0.5
    i = np.arange(nc)
    w = lanczos3(u[:, None] - i[None, :])
    return w / w.sum(axis=1, keepdims=True)


def upsample(hc, s, kind="nearest"):
    """h_fine = Wy hc Wx^T (float64, (ncy*s) x (ncx*s))."""
    hc = np.asarray(hc, dtype=np.float64)
    wy = axis_matrix(hc.shape[0], s, kind)
    wx = axis_matrix(hc.shape[1], s, kind)
    return wy @ hc @ wx.T


def upsample_adjoint(g, s, kind="nearest"):
    """U^T g = Wy^T g Wx (float64, ncy x ncx) for a fine-grid gradient g."""
    g = np.asarray(g, dtype=np.float64)
    wy = axis_matrix(g.shape[0] // s, s, kind)
    wx = axis_matrix(g.shape[1] // s, s, kind)
    return wy.T @ g @ wx
