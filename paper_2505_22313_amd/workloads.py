"""Seeded synthetic inputs for the DOE PSF workloads.

This module only draws and shapes input data (height maps, amplitude masks,
targets, request traces).  It holds none of the propagation arithmetic and is
shared by the tests, the benchmark and the smoke check; neither the HIP path
nor the CPU oracle imports it.

Lengths are in micrometres throughout.

Workloads (all synthetic; the paper's own targets and measured devices are not
used):

* ``small``:     512^2 i.i.d. uniform heights in [0, 1.2 um], dx = 1 um,
                 n = 1.46, lambda = 550 nm, z = 5 mm, padded to 1024^2.
* ``mid``:       8192^2 wrapped Fresnel lens (f = 20 mm, 2 pi at 550 nm) plus
                 smooth noise, dx = 1 um, lambda = 450/550/650 nm with the
                 Cauchy index, z = 20 mm, padded to 16384^2.
* ``large``:     32768^2 16-level Fresnel lens (f = 50 mm) plus smooth noise,
                 dx = 0.5 um, 31 wavelengths 400..700 nm, z = 50 mm, padded to
                 65536^2.
* ``design``:    8192^2 uniform init, 3 wavelengths, z = 20 mm, padded to
                 16384^2, Gaussian target (sigma = 3 px).
* ``serve``:     Poisson request trace, N in {2048, 4096, 8192, 16384}, 2x
                 padding, 1..31 wavelengths over 400..700 nm, z in [5, 50] mm.

The maximum height 1.2 um matches a 2 pi phase delay at 550 nm for the Cauchy
index (lambda0 / (n(lambda0) - 1) = 1.19 um), the depth the paper's
lithography is calibrated to (Sec. 3.2, contrast-curve footnote).
"""

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.fft as sfft


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def _parallel_rows(n, block, fn):
    """Run fn(r0, r1) over row blocks of [0, n) on a thread pool (NumPy
    releases the GIL inside its kernels)."""
    spans = [(r0, min(n, r0 + block)) for r0 in range(0, n, block)]
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(lambda s: fn(*s), spans))

LAMBDA0 = 0.55  # um, nominal design wavelength


def cauchy_index(lam_um):
    """Resin index used by the workloads: n = 1.45 + 3.6e-3 / lambda^2 (um)."""
    lam = np.asarray(lam_um, dtype=np.float64)
    return 1.45 + 3.6e-3 / (lam * lam)


def shape2(n):
    """(rows, columns) of a DOE given as an int (square) or a pair."""
    if np.ndim(n) == 0:
        return int(n), int(n)
    ny, nx = n
    return int(ny), int(nx)


def uniform_heights(n, seed, hmax=1.2):
    """i.i.d. uniform heights in [0, hmax] um, float32 (PCG64 stream `seed`);
    n is an int (square) or (rows, columns)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, hmax, size=shape2(n)).astype(np.float32)


def pixel_coords(n, dx):
    """Pixel j sits at (j - n/2) * dx, so the optical axis is on pixel n/2."""
    return (np.arange(n, dtype=np.float64) - n // 2) * dx


def fresnel_lens_heights(n, dx, f, lam0=LAMBDA0, levels=0, row_block=2048):
    """Hyperbolic focusing lens wrapped to 2 pi at lam0, as a height map.

    phi(r) = -(2 pi / lam0) (sqrt(r^2 + f^2) - f), wrapped into [0, 2 pi),
    h = phi_w * lam0 / (2 pi (n(lam0) - 1)).  With ``levels > 0`` the height
    is quantised to that many uniform levels (floor).  float32 result; n is
    an int (square) or (rows, columns).
    """
    n0 = float(cauchy_index(lam0))
    hmax = lam0 / (n0 - 1.0)
    ny, nx = shape2(n)
    out = np.empty((ny, nx), dtype=np.float32)
    y2 = pixel_coords(ny, dx) ** 2
    x2 = pixel_coords(nx, dx) ** 2

    def rows(r0, r1):
        r2 = y2[r0:r1, None] + x2[None, :]
        turns = -(np.sqrt(r2 + f * f) - f) / lam0
        frac = turns - np.floor(turns)  # wrapped phase / (2 pi), in [0, 1)
        h = frac * hmax
        if levels > 0:
            step = hmax / levels
            h = np.floor(h / step) * step
        out[r0:r1] = h.astype(np.float32)

    _parallel_rows(ny, min(row_block, 512), rows)
    return out


def smooth_noise(n, seed, sigma_px=8.0, std=0.02, truncate=4.0):
    """White N(0,1) noise blurred by a Gaussian (sigma in px, truncated at
    ``truncate`` sigma, circular boundary), rescaled to standard deviation
    ``std`` (um).  float32.

    The blur is the circular convolution with the separable truncated kernel,
    applied through its DFT along each axis.
    """
    # one PCG64 stream per block of rows, spawned from `seed`
    block = 1024
    nblk = (n + block - 1) // block
    seqs = np.random.SeedSequence(seed).spawn(nblk)
    noise = np.empty((n, n), dtype=np.float32)

    def rows(r0, r1):
        rng = np.random.default_rng(seqs[r0 // block])
        noise[r0:r1] = rng.standard_normal((r1 - r0, n), dtype=np.float32)

    _parallel_rows(n, block, rows)
    r = int(np.ceil(truncate * sigma_px))
    t = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-0.5 * (t / sigma_px) ** 2)
    g /= g.sum()
    kern = np.zeros(n, dtype=np.float64)
    kern[t.astype(np.int64) % n] += g
    # the kernel is real and even about 0, so its spectrum is real
    kspec = np.fft.rfft(kern).real
    kfull = np.fft.fft(kern).real
    spec = sfft.rfft2(noise, workers=_threads())
    del noise
    spec *= kspec[None, :].astype(np.float32)
    spec *= kfull[:, None].astype(np.float32)
    out = sfft.irfft2(spec, s=(n, n), workers=_threads()).astype(np.float32, copy=False)
    del spec
    out *= np.float32(std / float(out.std(dtype=np.float64)))
    return out


def gaussian_target(n, sigma_px, total):
    """Gaussian spot about pixel (ny/2, nx/2) scaled so that its sum is
    `total`; n is an int (square) or (rows, columns).  Formed as the product
    of its two axis profiles (float32), so large targets need no FP64 plane."""
    ny, nx = shape2(n)
    gy = np.exp(-((np.arange(ny, dtype=np.float64) - ny // 2) ** 2) / (2.0 * sigma_px ** 2))
    gx = np.exp(-((np.arange(nx, dtype=np.float64) - nx // 2) ** 2) / (2.0 * sigma_px ** 2))
    scale = total / (gy.sum() * gx.sum())
    return (gy * scale).astype(np.float32)[:, None] * gx.astype(np.float32)[None, :]


def square_lens_amp(n):
    """All-ones aperture."""
    return np.ones((n, n), dtype=np.float32)


def circular_aperture(n, dx, radius):
    """1 inside a disc of the given radius about the optical axis, else 0."""
    c = pixel_coords(n, dx)
    r2 = c[:, None] ** 2 + c[None, :] ** 2
    return (r2 <= radius * radius).astype(np.float32)


def ideal_lens_heights(n, dx, f, lam, n_index):
    """Unwrapped hyperbolic lens for wavelength lam, as heights modulo one
    wave (float32): phase -(2 pi/lam)(sqrt(r^2+f^2)-f) mod 2 pi; n is an int
    (square) or (rows, columns)."""
    ny, nx = shape2(n)
    r2 = pixel_coords(ny, dx)[:, None] ** 2 + pixel_coords(nx, dx)[None, :] ** 2
    turns = -(np.sqrt(r2 + f * f) - f) / lam
    frac = turns - np.floor(turns)
    return (frac * lam / (n_index - 1.0)).astype(np.float32)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def problem(name):
    """Scalar parameters of a named workload (dict)."""
    if name == "small":
        lams = np.array([0.55])
        return dict(n=512, m=1024, dx=1.0, z=5000.0, lams=lams,
                    n_index=np.array([1.46]), weights=np.ones(1))
    if name == "mid":
        lams = np.array([0.45, 0.55, 0.65])
        return dict(n=8192, m=16384, dx=1.0, z=20000.0, lams=lams,
                    n_index=cauchy_index(lams), weights=np.ones(3))
    if name == "large":
        lams = np.round(np.arange(31) * 0.01 + 0.40, 10)
        return dict(n=32768, m=65536, dx=0.5, z=50000.0, lams=lams,
                    n_index=cauchy_index(lams), weights=np.ones(31))
    if name == "design":
        lams = np.array([0.45, 0.55, 0.65])
        return dict(n=8192, m=16384, dx=1.0, z=20000.0, lams=lams,
                    n_index=cauchy_index(lams), weights=np.ones(3))
    if name == "paper":
        # Table 2's large-area hologram grid: a 32.16 x 21.44 mm DOE at 0.5 um
        # (rows x columns), padded to 128,640 x 85,760; z = 6 cm
        lams = np.array([0.5206])
        return dict(n=(64320, 42880), m=(128640, 85760), dx=0.5, z=60000.0, lams=lams,
                    n_index=cauchy_index(lams), weights=np.ones(1))
    raise KeyError(name)


def heights(name, n=None):
    """Height map (float32, um) of a named workload; `n` overrides the size."""
    p = problem(name)
    n = p["n"] if n is None else n
    if name == "small":
        return uniform_heights(n, seed=1)
    if name == "mid":
        h = fresnel_lens_heights(n, p["dx"], 20000.0)
        h += smooth_noise(n, seed=2)
        return h
    if name == "large":
        h = fresnel_lens_heights(n, p["dx"], 50000.0, levels=16)
        h += smooth_noise(n, seed=3)
        return h
    if name == "design":
        return uniform_heights(n, seed=4)
    if name == "paper":
        # a 2 um design (seeded uniform heights) upsampled 4x by nearest neighbour
        ny, nx = shape2(n)
        hc = uniform_heights((ny // 4, nx // 4), seed=16080)
        return np.repeat(np.repeat(hc, 4, axis=0), 4, axis=1)
    raise KeyError(name)


def serve_trace(count, rate_hz, seed=5, sizes=(2048, 4096, 8192, 16384),
                max_lambda=31):
    """Poisson request trace: list of dicts with arrival time (s), n, m, z and
    the wavelength set (k values evenly spaced over 400..700 nm; k = 1 is
    550 nm)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(count):
        n = int(rng.choice(sizes))
        k = int(rng.integers(1, max_lambda + 1))
        lams = np.array([0.55]) if k == 1 else np.linspace(0.40, 0.70, k)
        reqs.append(dict(t=float(t[i]), n=n, m=2 * n, dx=1.0,
                         z=float(rng.uniform(5000.0, 50000.0)), lams=lams,
                         n_index=cauchy_index(lams), pool=int(rng.integers(0, 4))))
    return reqs


def serve_height_pool(n, count=4, seed=5):
    """`count` smooth random height maps of size n (generation is not timed)."""
    out = []
    for i in range(count):
        sm = smooth_noise(n, seed=seed * 1000 + i, sigma_px=4.0, std=0.3)
        out.append(np.clip(0.6 + sm, 0.0, 1.2).astype(np.float32))
    return out
