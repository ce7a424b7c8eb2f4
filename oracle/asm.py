"""FP64 oracle of the DOE image-formation model (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module; the product library never does.

The model (paper Sec. 3.1, "Fabrication-aware Image Formation Model"):

* Eq. (1): the DOE phase at wavelength lambda is
  Phi = 2*pi/lambda * (n(lambda) - 1) * h.
* Eq. (2): the field leaving the DOE is the incident field times exp(i*Phi).
  Incident field here: a unit-amplitude normal plane wave, optionally
  multiplied by a real aperture amplitude ``amp``.
* Eq. (3): the field at distance z is F^-1{ F{E_doe} (.) H_lambda }.  The paper
  does not write H; this oracle takes the plain angular-spectrum transfer
  function of free space (Goodman) with the evanescent part cut off:
  H = exp(i*2*pi*z*sqrt(1/lambda^2 - fx^2 - fy^2)) where
  s = (lambda*fx)^2 + (lambda*fy)^2 < 1, and 0 elsewhere.
* Eq. (4): the intensity |E_dest|^2 is summed over wavelengths.
* The DOE (N x N samples) is zero-padded to an M x M grid, centred at offset
  p0 = (M - N) // 2 (the paper's grids are twice the DOE extent, Table 2).
  Grids may be rectangular (the paper's largest is 128,640 x 85,760): arrays
  are (rows, columns) = (y, x), ``m`` is an int or a (My, Mx) pair, and every
  axis is padded, transformed and sampled in frequency on its own.

Every array here is complex128 / float64.  ``scipy.fft`` is used as the FFT
primitive; ``direct_dft2`` and ``brute_propagate`` are the independent
definitions the FFT path is pinned against on tiny grids.

The adjoint (``psf_backward``) follows from the paper's remark in Sec. 4.1
that the DFT is a symmetric matrix, so the backward pass of a 2-D FFT is
another 2-D FFT: the adjoint of ifft2 o diag(H) o fft2 is
ifft2 o diag(conj H) o fft2.
"""

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.fft as sfft

# Threads handed to scipy.fft.  The CPU baseline reports this number.
WORKERS = os.cpu_count() or 1


def pad_offset(n, m):
    """Offset of the N x N DOE inside the M x M grid (centred placement)."""
    return (m - n) // 2


def grid_shape(m):
    """(My, Mx) of a padded grid given as an int (square) or a pair."""
    if np.ndim(m) == 0:
        return int(m), int(m)
    my, mx = m
    return int(my), int(mx)


def doe_field(h, lam, n_index, amp=None):
    """Eq. (1)-(2): E = amp * exp(i * 2*pi/lam * (n - 1) * h), complex128."""
    h = np.asarray(h, dtype=np.float64)
    phi = (2.0 * np.pi / lam) * (n_index - 1.0) * h
    e = np.exp(1j * phi)
    if amp is not None:
        e = e * np.asarray(amp, dtype=np.float64)
    return e


def embed(e, m):
    """Zero-pad an Ny x Nx field into an My x Mx grid at offset
    p0 = (M - N) // 2 on each axis."""
    ny, nx = e.shape
    my, mx = grid_shape(m)
    py, px = pad_offset(ny, my), pad_offset(nx, mx)
    ep = np.zeros((my, mx), dtype=np.complex128)
    ep[py:py + ny, px:px + nx] = e
    return ep


def crop(u, n):
    """The window of N samples at offset p0 on each axis of a padded grid;
    n is an int (square window) or an (Ny, Nx) pair."""
    ny, nx = grid_shape(n)
    py, px = pad_offset(ny, u.shape[0]), pad_offset(nx, u.shape[1])
    return u[py:py + ny, px:px + nx]


def band_limit(m, dx, lam, z):
    """Matsushima & Shimobaba (2009) band limit of the sampled transfer
    function: f_lim = 1 / (lam sqrt((2 z / (M dx))^2 + 1)).  Beyond it the
    phase of H changes by more than pi between neighbouring frequency samples
    of the M-point grid, so its samples alias."""
    t = 2.0 * abs(z) / (m * dx)
    return 1.0 / (lam * np.sqrt(t * t + 1.0))


def transfer_function(m, dx, lam, z, bandlimit=False):
    """Angular-spectrum transfer function on the FFT frequency grid (Eq. 3).

    Frequencies are numpy's fftfreq (k / (M dx), k signed), per axis.  Rows
    index fy, columns index fx.  A frequency propagates iff s < 1 with
    s = (lam*fx)^2 + (lam*fy)^2, each square and the sum rounded once in FP64.
    With ``bandlimit`` it must also satisfy |fx| < f_lim(Mx) and
    |fy| < f_lim(My) (band-limited ASM, one of the propagation variants the
    paper cites; the limit depends on the axis length).
    """
    return transfer_rows(m, dx, lam, z, 0, grid_shape(m)[0], bandlimit=bandlimit)


def transfer_rows(m, dx, lam, z, r0, r1, bandlimit=False):
    """Rows r0 .. r1-1 (fy bins) of ``transfer_function``."""
    my, mx = grid_shape(m)
    fy = np.fft.fftfreq(my, d=dx)
    fx = np.fft.fftfreq(mx, d=dx)
    ay, ax = lam * fy, lam * fx
    s = (ay * ay)[r0:r1, None] + (ax * ax)[None, :]
    prop = s < 1.0
    if bandlimit:
        in_y = np.abs(fy) < band_limit(my, dx, lam, z)
        in_x = np.abs(fx) < band_limit(mx, dx, lam, z)
        prop = prop & in_y[r0:r1, None] & in_x[None, :]
    root = np.sqrt(np.where(prop, 1.0 - s, 0.0))
    kz = 2.0 * np.pi * z / lam
    return np.where(prop, np.exp(1j * (kz * root)), 0.0 + 0.0j)


def propagate_padded(ep, dx, lam, z, adjoint=False, bandlimit=False):
    """Eq. (3) on an already padded M x M field: ifft2(fft2(ep) * H).

    ``adjoint=True`` applies the adjoint operator ifft2(fft2(ep) * conj(H)).
    """
    h = transfer_function(ep.shape, dx, lam, z, bandlimit=bandlimit)
    if adjoint:
        h = np.conj(h)
    a = sfft.fft2(ep, workers=WORKERS)
    return sfft.ifft2(a * h, workers=WORKERS)


def propagate(u_in, m, dx, lam, z, out_mode="crop", adjoint=False, bandlimit=False):
    """Propagate an N x N complex field (zero-padded to M x M) by z.

    Returns the N x N crop at [p0, p0+N)^2 (``out_mode="crop"``) or the whole
    M x M plane (``out_mode="full"``).
    """
    u_in = np.asarray(u_in, dtype=np.complex128)
    n = u_in.shape
    u = propagate_padded(embed(u_in, m), dx, lam, z, adjoint=adjoint, bandlimit=bandlimit)
    return crop(u, n) if out_mode == "crop" else u


def psf(h, dx, z, m, lams, n_index, weights=None, amp=None, out_mode="crop",
        return_fields=False, bandlimit=False):
    """Eq. (4): sum_k w_k |E_dest,k|^2 over the wavelengths, in k order.

    Returns the float64 PSF (N x N crop or M x M full).  With
    ``return_fields=True`` also returns the list of complex128 fields U_k
    (same region as the PSF).
    """
    h = np.asarray(h, dtype=np.float64)
    k_count = len(lams)
    if weights is None:
        weights = np.ones(k_count)
    shape = h.shape if out_mode == "crop" else grid_shape(m)
    acc = np.zeros(shape, dtype=np.float64)
    fields = []
    for k in range(k_count):
        e = doe_field(h, lams[k], n_index[k], amp)
        u = propagate(e, m, dx, lams[k], z, out_mode=out_mode, bandlimit=bandlimit)
        acc += float(weights[k]) * (u.real * u.real + u.imag * u.imag)
        if return_fields:
            fields.append(u)
    return (acc, fields) if return_fields else acc


def psf_lowmem(h, dx, z, m, lam, n_index, block=1024, log=None, rows=None):
    """``psf`` for one wavelength (CROP, no amplitude mask, weight 1) on grids
    whose full-plane temporaries do not fit in memory (square or
    rectangular).

    Same definition, same order of operations per element: the 2-D DFTs are
    taken as 1-D DFTs along rows and then along columns (the 2-D DFT is
    separable), each over blocks of rows or columns of one complex128 M x M
    array, and H is applied one block of rows at a time.  Rows of the padded
    field outside the DOE are zero, so their row DFTs are skipped; only the
    N crop rows of the inverse row DFT are taken.  Peak memory is about
    16 M^2 bytes plus a few blocks.  Returns the N x N float64 PSF; with
    ``rows`` (indices into the crop) returns (psf[rows], sum, max) instead,
    the sum and max taken over the whole crop without holding it.
    """
    keep = None if rows is None else np.asarray(rows, dtype=np.int64)
    h = np.asarray(h)
    ny, nx = h.shape
    my, mx = grid_shape(m)
    py, px = pad_offset(ny, my), pad_offset(nx, mx)
    say = log or (lambda msg: None)
    ep = np.zeros((my, mx), dtype=np.complex128)
    for r0 in range(0, ny, block):
        r1 = min(ny, r0 + block)
        rows = ep[py + r0:py + r1]
        rows[:, px:px + nx] = doe_field(h[r0:r1], lam, n_index)
        ep[py + r0:py + r1] = sfft.fft(rows, axis=1, workers=WORKERS)
    say("row DFTs done")
    for c0 in range(0, mx, block):
        c1 = min(mx, c0 + block)
        ep[:, c0:c1] = sfft.fft(ep[:, c0:c1], axis=0, workers=WORKERS)
    say("column DFTs done")
    def apply_h(r0):
        r1 = min(my, r0 + hblock)
        ep[r0:r1] *= transfer_rows((my, mx), dx, lam, z, r0, r1)

    hblock = max(1, min(block, (1 << 24) // mx))  # about 1 GB of temporaries per thread
    with ThreadPoolExecutor(WORKERS) as pool:
        list(pool.map(apply_h, range(0, my, hblock)))
    say("transfer function applied")
    for c0 in range(0, mx, block):
        c1 = min(mx, c0 + block)
        ep[:, c0:c1] = sfft.ifft(ep[:, c0:c1], axis=0, workers=WORKERS)
    say("inverse column DFTs done")
    out = np.empty((ny, nx) if keep is None else (len(keep), nx), dtype=np.float64)
    total, peak = 0.0, 0.0
    for r0 in range(0, ny, block):
        r1 = min(ny, r0 + block)
        u = sfft.ifft(ep[py + r0:py + r1], axis=1, workers=WORKERS)[:, px:px + nx]
        p = u.real * u.real + u.imag * u.imag
        if keep is None:
            out[r0:r1] = p
        else:
            sel = (keep >= r0) & (keep < r1)
            out[sel] = p[keep[sel] - r0]
            total += float(p.sum())
            peak = max(peak, float(p.max()))
    say("inverse row DFTs done")
    return out if keep is None else (out, total, peak)


def psf_backward(h, dx, z, m, lams, n_index, grad_psf, weights=None, amp=None,
                 out_mode="crop", bandlimit=False):
    """Gradient dL/dh of a real loss L given G = dL/dPSF (same region as the PSF).

    Convention: the gradient of L with respect to a complex field u is
    g = dL/dRe(u) + i dL/dIm(u).  Per wavelength k:
      g_U  = 2 w_k G * U_k
      g_Ep = ifft2(fft2(g_U embedded) * conj(H_k))       (adjoint of Eq. 3)
      dL/dh += c_k * Im(g_E * conj(E_k)),  c_k = 2*pi*(n_k - 1)/lam_k
    where g_E is g_Ep on the DOE window and E_k is Eq. (2).
    """
    h = np.asarray(h, dtype=np.float64)
    g = np.asarray(grad_psf, dtype=np.float64)
    n = h.shape
    k_count = len(lams)
    if weights is None:
        weights = np.ones(k_count)
    grad = np.zeros(n, dtype=np.float64)
    for k in range(k_count):
        e = doe_field(h, lams[k], n_index[k], amp)
        ep = embed(e, m)
        u = propagate_padded(ep, dx, lams[k], z, bandlimit=bandlimit)
        if out_mode == "crop":
            g_u = embed(2.0 * float(weights[k]) * g * crop(u, n), m)
        else:
            g_u = 2.0 * float(weights[k]) * g * u
        g_ep = propagate_padded(g_u, dx, lams[k], z, adjoint=True, bandlimit=bandlimit)
        g_e = crop(g_ep, n)
        c_k = 2.0 * np.pi * (n_index[k] - 1.0) / lams[k]
        grad += c_k * np.imag(g_e * np.conj(e))
    return grad


# ---------------------------------------------------------------------------
# Independent definitions used to pin the FFT path on tiny grids.
# ---------------------------------------------------------------------------

def direct_dft2(x, inverse=False):
    """2-D DFT written as the matrix product Wy x Wx^T (no FFT).

    Forward: X[u, v] = sum_{y, x} x[y, x] exp(-2 pi i (u y / My + v x / Mx)).
    Inverse: the conjugate kernels and a 1/(My Mx) factor.
    """
    x = np.asarray(x, dtype=np.complex128)
    my, mx = x.shape
    sign = 1.0 if inverse else -1.0

    def kernel(m):
        idx = np.arange(m)
        return np.exp(sign * 2j * np.pi * np.outer(idx, idx) / m)

    out = kernel(my) @ x @ kernel(mx).T
    return out / (my * mx) if inverse else out


def _signed_freq(k, m, dx):
    """Frequency of DFT bin k on an M-point grid of pitch dx: k/(M dx) for
    k < M/2, (k - M)/(M dx) otherwise."""
    ks = k if k < (m + 1) // 2 else k - m
    return ks / (m * dx)


def brute_propagate(u_in, m, dx, lam, z):
    """Eq. (3) by explicit sums over the M x M grid (tiny M only).

    Every bin's transfer value is evaluated on its own from the physical
    frequency, the spectrum and its inverse are plain double sums.  Returns the
    full My x Mx field for a centred Ny x Nx input (m an int or (My, Mx)).
    """
    my, mx = grid_shape(m)
    ep = embed(np.asarray(u_in, dtype=np.complex128), (my, mx))
    iy, ix = np.arange(my), np.arange(mx)
    u_out = np.zeros((my, mx), dtype=np.complex128)
    for fu in range(my):
        fy = _signed_freq(fu, my, dx)
        for fv in range(mx):
            fx = _signed_freq(fv, mx, dx)
            s = (lam * fx) * (lam * fx) + (lam * fy) * (lam * fy)
            if not s < 1.0:
                continue
            hval = np.exp(1j * 2.0 * np.pi * z * np.sqrt(1.0 / (lam * lam) - fx * fx - fy * fy))
            # forward DFT coefficient of bin (fu, fv)
            ky = np.exp(-2j * np.pi * fu * iy / my)
            kx = np.exp(-2j * np.pi * fv * ix / mx)
            coef = ky @ ep @ kx
            # add this bin's plane wave to the output
            u_out += (coef * hval / (my * mx)) * np.outer(np.conj(ky), np.conj(kx))
    return u_out


# ---------------------------------------------------------------------------
# Exact Eq. (3) outputs that can be evaluated one row at a time (for checks at
# grid sizes whose full M x M field does not fit the oracle's memory).
# ---------------------------------------------------------------------------

def transfer_value(ky, kx, m, dx, lam, z):
    """H at individual DFT bins (arrays of integer indices in [0, M)), with the
    same frequency grid and evanescent test as transfer_function."""
    f = np.fft.fftfreq(m, d=dx)
    ay = lam * f[np.asarray(ky)]
    ax = lam * f[np.asarray(kx)]
    s = ay * ay + ax * ax
    prop = s < 1.0
    root = np.sqrt(np.where(prop, 1.0 - s, 0.0))
    kz = 2.0 * np.pi * z / lam
    return np.where(prop, np.exp(1j * (kz * root)), 0.0 + 0.0j)


def plane_wave_rows(coeffs, bins, m, dx, lam, z, rows):
    """Eq. (3) for an unpadded (N = M) input that is a sum of DFT plane waves
    sum_i c_i exp(2 pi i (u_i y + v_i x) / M): each wave is an eigenfunction,
    so the output on the given rows is sum_i c_i H(u_i, v_i) (same wave)."""
    rows = np.asarray(rows)
    x = np.arange(m)
    out = np.zeros((len(rows), m), dtype=np.complex128)
    for c, (u, v) in zip(coeffs, bins):
        hval = transfer_value([u], [v], m, dx, lam, z)[0]
        ph = (np.outer((u * rows) % m, np.ones(m, dtype=np.int64)) + (v * x) % m) % m
        out += c * hval * np.exp(2j * np.pi * ph / m)
    return out


def point_source_rows(n, m, dx, lam, z, src, rows, row_block=256):
    """Eq. (3) for a unit point source at DOE pixel src = (sy, sx) (centred
    padding), on the given rows of the N x N output window.

    The padded input is a Kronecker delta, so its spectrum is
    exp(-2 pi i (u sy' + v sx') / M) with sy' = p0 + sy.  Row y' = p0 + y of
    the output is the inverse 2-D DFT restricted to that row: the sum over u
    of exp(2 pi i u y' / M) times the 1-D inverse DFT over v of row u of the
    filtered spectrum (row-column decomposition, Sec. 4.1), divided by M^2.
    Returns a complex128 array of shape (len(rows), N).
    """
    rows = np.asarray(rows)
    p0 = pad_offset(n, m)
    sy, sx = p0 + src[0], p0 + src[1]
    yo = p0 + rows
    f = np.fft.fftfreq(m, d=dx)
    a2 = (lam * f) ** 2
    kz = 2.0 * np.pi * z / lam
    v = np.arange(m)
    phase_x = np.exp(-2j * np.pi * ((v * sx) % m) / m)
    acc = np.zeros((len(rows), m), dtype=np.complex128)
    for u0 in range(0, m, row_block):
        u = np.arange(u0, min(m, u0 + row_block))
        s = a2[u][:, None] + a2[None, :]
        prop = s < 1.0
        hblk = np.where(prop, np.exp(1j * (kz * np.sqrt(np.where(prop, 1.0 - s, 0.0)))), 0.0)
        spec = hblk * np.exp(-2j * np.pi * ((u * sy) % m) / m)[:, None] * phase_x[None, :]
        g = sfft.ifft(spec, axis=1, workers=WORKERS) * m        # sum over v, no 1/M yet
        wy = np.exp(2j * np.pi * ((np.outer(yo, u)) % m) / m)  # (rows, block)
        acc += wy @ g
    acc /= float(m) * float(m)
    return acc[:, p0:p0 + n]
