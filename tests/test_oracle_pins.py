"""Pins of the FP64 oracle against facts fixed outside it (CPU only).

Each test checks the oracle against something it does not compute itself: a
direct DFT, an explicit per-bin sum, Parseval's theorem, the free-space
plane-wave eigenfunction, closed-form focal spots of an ideal lens (Goodman,
Introduction to Fourier Optics: sinc^2 for a square and Airy for a circular
pupil), invariances of Eq. (1)-(2), finite differences and the adjoint
identity.
"""

import numpy as np
import pytest
import scipy.special as sps

import oracle
from oracle import asm
from paper_2505_22313_amd import workloads as wl


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def rand_field(rng, n):
    return rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))


# ---------------------------------------------------------------------------
# FFT primitive and transfer function against direct sums
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m", [8, 16, 32, 64])
def test_fft_path_matches_direct_dft(m):
    """Eq. (3) through scipy.fft equals Eq. (3) through the matrix DFT."""
    rng = np.random.default_rng(m)
    ep = rand_field(rng, m)
    dx, lam, z = 0.3, 0.5, 7.0
    h = oracle.transfer_function(m, dx, lam, z)
    want = asm.direct_dft2(asm.direct_dft2(ep) * h, inverse=True)
    got = oracle.propagate_padded(ep, dx, lam, z)
    assert rel(got, want) < 1e-12


def _mask_margin(m, dx, lam):
    f = np.fft.fftfreq(m, d=dx)
    s = (lam * f)[:, None] ** 2 + (lam * f)[None, :] ** 2
    return float(np.min(np.abs(s - 1.0)))


@pytest.mark.parametrize("m,n,dx,lam,z", [
    (8, 5, 0.3, 0.5, 3.0),      # evanescent corners present
    (16, 8, 0.3, 0.5, 11.0),
    (16, 16, 1.0, 0.55, 40.0),  # all bins propagate, no padding
    (12, 7, 0.27, 0.5, 5.0),    # even, non power of two
])
def test_propagate_matches_brute_force(m, n, dx, lam, z):
    """Oracle propagate == per-bin explicit sum with an independently evaluated
    transfer value and evanescent test."""
    assert _mask_margin(m, dx, lam) > 1e-6  # no bin sits on the cutoff
    rng = np.random.default_rng(100 + m + n)
    u = rand_field(rng, n)
    got = oracle.propagate(u, m, dx, lam, z, out_mode="full")
    want = asm.brute_propagate(u, m, dx, lam, z)
    assert rel(got, want) < 1e-11


# ---------------------------------------------------------------------------
# Energy, identities, invariances
# ---------------------------------------------------------------------------

def test_parseval_all_bins_propagate():
    """Unit-modulus DOE, every bin propagating: sum |U|^2 over the full plane
    equals N^2 (the transfer function is unimodular)."""
    n, m, dx, lam, z = 96, 192, 1.0, 0.55, 5000.0
    h = wl.uniform_heights(n, seed=11)
    p = oracle.psf(h, dx, z, m, [lam], [1.46], out_mode="full")
    assert abs(p.sum() / n ** 2 - 1.0) < 1e-12


def test_evanescent_energy_loss():
    """With pitch 0.25 um at 520.6 nm (the paper's hologram wavelength) the
    axis bins beyond |f| = 1/lambda are cut: the output energy equals the
    spectral energy of the propagating bins (explicit per-bin test)."""
    n, m, dx, lam, z = 16, 32, 0.25, 0.5206, 30.0
    rng = np.random.default_rng(7)
    e = np.exp(1j * rng.uniform(0, 2 * np.pi, (n, n)))
    u = oracle.propagate(e, m, dx, lam, z, out_mode="full")
    spec = asm.direct_dft2(oracle.embed(e, m))
    keep = 0.0
    for fu in range(m):
        for fv in range(m):
            fy = asm._signed_freq(fu, m, dx)
            fx = asm._signed_freq(fv, m, dx)
            if (lam * fx) ** 2 + (lam * fy) ** 2 < 1.0:
                keep += abs(spec[fu, fv]) ** 2
    energy = float(np.sum(np.abs(u) ** 2))
    assert abs(energy - keep / m ** 2) / energy < 1e-12
    assert energy < n * n * (1 - 1e-3)


def test_z_zero_is_identity():
    n, m, dx, lam = 40, 64, 1.0, 0.55
    rng = np.random.default_rng(3)
    u = rand_field(rng, n)
    out = oracle.propagate(u, m, dx, lam, 0.0, out_mode="full")
    assert rel(out, oracle.embed(u, m)) < 1e-14


def test_plus_minus_z_round_trip():
    n, m, dx, lam, z = 40, 64, 1.0, 0.55, 3000.0
    rng = np.random.default_rng(4)
    u = rand_field(rng, n)
    fwd = oracle.propagate(u, m, dx, lam, z, out_mode="full")
    back = oracle.propagate_padded(fwd, dx, lam, -z)
    assert rel(back, oracle.embed(u, m)) < 1e-12


def test_constant_height_only_shifts_phase():
    n, m, dx, lam, nn, z = 48, 96, 1.0, 0.55, 1.46, 2000.0
    h = wl.uniform_heights(n, seed=5).astype(np.float64)
    a = oracle.psf(h, dx, z, m, [lam], [nn])
    b = oracle.psf(h + 0.37, dx, z, m, [lam], [nn])
    assert rel(b, a) < 1e-12


def test_one_wave_height_is_invisible():
    """Adding lambda/(n-1) to h adds exactly 2 pi to the phase of Eq. (1)."""
    n, m, dx, lam, nn, z = 48, 96, 1.0, 0.55, 1.46, 2000.0
    h = wl.uniform_heights(n, seed=6).astype(np.float64)
    e0 = oracle.doe_field(h, lam, nn)
    e1 = oracle.doe_field(h + lam / (nn - 1.0), lam, nn)
    assert rel(e1, e0) < 1e-13
    u0 = oracle.propagate(e0, m, dx, lam, z)
    u1 = oracle.propagate(e1, m, dx, lam, z)
    assert rel(u1, u0) < 1e-12


def test_wavelength_sum_is_linear():
    n, m, dx, z = 48, 96, 1.0, 2000.0
    lams = [0.45, 0.55, 0.65]
    nidx = wl.cauchy_index(lams)
    w = [0.5, 1.0, 2.0]
    h = wl.uniform_heights(n, seed=8)
    tot = oracle.psf(h, dx, z, m, lams, nidx, weights=w)
    parts = sum(w[k] * oracle.psf(h, dx, z, m, [lams[k]], [nidx[k]]) for k in range(3))
    assert rel(tot, parts) < 1e-13


@pytest.mark.parametrize("u0,v0", [(0, 3), (5, -7), (-20, 11), (31, 31)])
def test_plane_wave_eigenfunction(u0, v0):
    """A plane wave exp(2 pi i (fx x + fy y)) travels by exp(i 2 pi z cos(theta)
    / lambda) with cos(theta) = sqrt(1 - (lambda fx)^2 - (lambda fy)^2); an
    evanescent one is cut (Goodman, free-space transfer function)."""
    m, dx, lam, z = 64, 0.4, 0.6, 123.0
    yy, xx = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    wave = np.exp(2j * np.pi * (u0 * yy + v0 * xx) / m)
    out = oracle.propagate(wave, m, dx, lam, z, out_mode="full")
    fy, fx = u0 / (m * dx), v0 / (m * dx)
    cos2 = 1.0 - (lam * fx) ** 2 - (lam * fy) ** 2
    if cos2 > 0:
        want = np.exp(1j * 2 * np.pi * z * np.sqrt(cos2) / lam) * wave
        assert rel(out, want) < 1e-12
    else:
        assert np.max(np.abs(out)) < 1e-12


# ---------------------------------------------------------------------------
# Closed-form focal spots of an ideal lens
# ---------------------------------------------------------------------------

def _lens_psf(amp, n, m, dx, lam, f, nn=1.5):
    h = wl.ideal_lens_heights(n, dx, f, lam, nn).astype(np.float64)
    return oracle.psf(h, dx, f, m, [lam], [nn], amp=amp)


def test_square_lens_focus_sinc2():
    """Square pupil of side L focused at f: I(x, 0) = (L^2/(lam f))^2
    sinc^2(L x/(lam f)) (Fraunhofer pattern at the focal plane)."""
    n, m, dx, lam, f = 512, 1024, 1.0, 0.55, 5000.0
    p = _lens_psf(None, n, m, dx, lam, f)
    c = n // 2
    side = n * dx
    i0 = (side * side / (lam * f)) ** 2
    assert abs(p[c, c] / i0 - 1.0) < 0.02
    assert np.unravel_index(np.argmax(p), p.shape) == (c, c)
    x = np.arange(-12, 13) * dx
    want = i0 * np.sinc(side * x / (lam * f)) ** 2
    assert np.max(np.abs(p[c, c - 12:c + 13] - want)) / i0 < 0.02
    assert np.max(np.abs(p[c - 12:c + 13, c] - want)) / i0 < 0.02


def test_circular_lens_focus_airy():
    """Circular pupil radius R: Airy pattern I0 [2 J1(v)/v]^2,
    v = 2 pi R rho/(lam f), I0 = (pi R^2/(lam f))^2; 83.8 % of the power lies
    inside the first dark ring (rho = 0.61 lam f / R)."""
    n, m, dx, lam, f, rad = 512, 1024, 1.0, 0.55, 5000.0, 200.0
    amp = wl.circular_aperture(n, dx, rad)
    p = _lens_psf(amp, n, m, dx, lam, f)
    c = n // 2
    i0 = (np.pi * rad * rad / (lam * f)) ** 2
    assert abs(p[c, c] / i0 - 1.0) < 0.02
    x = np.arange(1, 20) * dx
    v = 2 * np.pi * rad * x / (lam * f)
    want = i0 * (2 * sps.j1(v) / v) ** 2
    assert np.max(np.abs(p[c, c + 1:c + 20] - want)) / i0 < 0.02
    yy, xx = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
    r_dark = 0.61 * lam * f / rad / dx
    inside = p[(yy ** 2 + xx ** 2) <= r_dark ** 2].sum()
    total = float(amp.astype(np.float64).sum())  # input power (Parseval)
    assert abs(inside / total - 0.838) < 0.02


# ---------------------------------------------------------------------------
# Gradient
# ---------------------------------------------------------------------------

def _loss_setup(out_mode):
    # the differentiable-design gradcheck instance: 64 x 64 heights on a
    # 128 x 128 grid, three wavelengths, FP64
    n, m, dx, z = 64, 128, 1.0, 1500.0
    lams = np.array([0.45, 0.55, 0.65])
    nidx = wl.cauchy_index(lams)
    w = np.array([1.0, 0.7, 1.3])
    rng = np.random.default_rng(21)
    h = rng.uniform(0, 1.2, (n, n))
    amp = rng.uniform(0.5, 1.0, (n, n))
    shape = (n, n) if out_mode == "crop" else (m, m)
    target = rng.uniform(0, 2.0, shape)

    def loss(hh):
        p = oracle.psf(hh, dx, z, m, lams, nidx, weights=w, amp=amp, out_mode=out_mode)
        return float(np.mean((p - target) ** 2))

    def grad(hh):
        p = oracle.psf(hh, dx, z, m, lams, nidx, weights=w, amp=amp, out_mode=out_mode)
        g = 2.0 * (p - target) / p.size
        return oracle.psf_backward(hh, dx, z, m, lams, nidx, g, weights=w, amp=amp,
                                   out_mode=out_mode)

    return h, loss, grad, rng


@pytest.mark.parametrize("out_mode", ["crop", "full"])
def test_gradient_finite_differences(out_mode):
    h, loss, grad, rng = _loss_setup(out_mode)
    g = grad(h)
    eps = 1e-5
    d = rng.standard_normal(h.shape)
    fd = (loss(h + eps * d) - loss(h - eps * d)) / (2 * eps)
    assert abs(fd - np.sum(g * d)) / abs(fd) < 1e-7
    for _ in range(4):
        i, j = rng.integers(0, h.shape[0], 2)
        e = np.zeros_like(h)
        e[i, j] = 1.0
        fd = (loss(h + eps * e) - loss(h - eps * e)) / (2 * eps)
        assert abs(fd - g[i, j]) <= 1e-6 * np.max(np.abs(g)) + 1e-8 * abs(fd)


@pytest.mark.slow
def test_gradient_full_gradcheck_64():
    """Central finite differences of the loss with respect to every one of
    the 64 x 64 heights (step 1e-5 in FP64) against the adjoint gradient,
    element by element."""
    h, loss, grad, _ = _loss_setup("crop")
    g = grad(h)
    eps = 1e-5
    fd = np.empty_like(h)
    for i in range(h.shape[0]):
        for j in range(h.shape[1]):
            hp = h.copy()
            hp[i, j] += eps
            lp = loss(hp)
            hp[i, j] -= 2 * eps
            fd[i, j] = (lp - loss(hp)) / (2 * eps)
    scale = np.max(np.abs(g))
    assert np.max(np.abs(fd - g)) <= 1e-8 * scale + 1e-12
    assert np.linalg.norm(fd - g) <= 1e-8 * np.linalg.norm(g)


def test_adjoint_dot_product():
    """<P x, y> == <x, P^H y> for the padded propagation operator."""
    m, dx, lam, z = 64, 0.3, 0.5, 50.0
    rng = np.random.default_rng(9)
    x, y = rand_field(rng, m), rand_field(rng, m)
    px = oracle.propagate_padded(x, dx, lam, z)
    phy = oracle.propagate_padded(y, dx, lam, z, adjoint=True)
    lhs = np.vdot(y, px)
    rhs = np.vdot(phy, x)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


# ---------------------------------------------------------------------------
# Row-wise exact outputs used at grid sizes the full oracle cannot hold
# ---------------------------------------------------------------------------

def test_plane_wave_rows_match_propagate():
    m, dx, lam, z = 64, 0.4, 0.9, 77.0
    bins = [(0, 3), (5, 60), (31, 31), (17, 2)]      # (31, 31) is evanescent here
    coeffs = [1.0, 0.5 - 0.2j, 2.0, -0.3j]
    yy, xx = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    field = sum(c * np.exp(2j * np.pi * (u * yy + v * xx) / m) for c, (u, v) in zip(coeffs, bins))
    full = oracle.propagate(field, m, dx, lam, z, out_mode="full")
    rows = [0, 7, 63]
    got = asm.plane_wave_rows(coeffs, bins, m, dx, lam, z, rows)
    assert rel(got, full[rows]) < 1e-12
    assert asm.transfer_value([31], [31], m, dx, lam, z)[0] == 0


@pytest.mark.parametrize("n,m,src", [(32, 64, (16, 16)), (20, 64, (3, 17)), (64, 64, (0, 63))])
def test_point_source_rows_match_propagate(n, m, src):
    dx, lam, z = 0.5, 0.55, 120.0
    u = np.zeros((n, n), dtype=np.complex128)
    u[src] = 1.0
    full = oracle.propagate(u, m, dx, lam, z)
    rows = [0, src[0], n - 1]
    got = asm.point_source_rows(n, m, dx, lam, z, src, rows, row_block=16)
    assert rel(got, full[rows]) < 1e-12


# ---------------------------------------------------------------------------
# Band-limited ASM (Matsushima & Shimobaba 2009)
# ---------------------------------------------------------------------------

def test_bandlimit_is_plain_asm_when_limit_is_beyond_nyquist():
    n, m, dx, lam, z = 48, 96, 1.0, 0.55, 20.0
    assert oracle.band_limit(m, dx, lam, z) > 1.0 / (2 * dx)
    rng = np.random.default_rng(12)
    u = rand_field(rng, n)
    a = oracle.propagate(u, m, dx, lam, z)
    b = oracle.propagate(u, m, dx, lam, z, bandlimit=True)
    assert np.array_equal(a, b)


def test_bandlimit_mask_per_bin():
    """Explicit per-bin test of the band-limited propagating set."""
    m, dx, lam, z = 32, 0.4, 0.6, 150.0
    flim = 1.0 / (lam * np.sqrt((2.0 * z / (m * dx)) ** 2 + 1.0))
    hb = oracle.transfer_function(m, dx, lam, z, bandlimit=True)
    for fu in range(m):
        for fv in range(m):
            fy, fx = asm._signed_freq(fu, m, dx), asm._signed_freq(fv, m, dx)
            keep = ((lam * fx) ** 2 + (lam * fy) ** 2 < 1.0 and abs(fx) < flim and abs(fy) < flim)
            assert (hb[fu, fv] != 0) == keep


@pytest.mark.parametrize("z", [1000.0, 2000.0])
def test_bandlimit_removes_transfer_function_aliasing(z):
    """At long distance the plain transfer function is undersampled on a 2x
    grid and its aliases wrap light back into the window; the band-limited
    result stays close to a 16x-padded reference (Matsushima & Shimobaba,
    Opt. Express 17, 19662, 2009)."""
    n, m, dx, lam = 64, 128, 1.0, 0.5
    rng = np.random.default_rng(3)
    u = np.exp(1j * rng.uniform(0, 2 * np.pi, (n, n)))
    ref = oracle.propagate(u, 16 * n, dx, lam, z)
    plain = oracle.propagate(u, m, dx, lam, z)
    bl = oracle.propagate(u, m, dx, lam, z, bandlimit=True)
    e_plain, e_bl = rel(plain, ref), rel(bl, ref)
    assert e_bl < 0.5
    assert e_bl < e_plain / 5


# ---------------------------------------------------------------------------
# Super-resolved front end: nearest and Lanczos-3 upsampling (Sec. 3.2)
# ---------------------------------------------------------------------------

from oracle import upsample as ups  # noqa: E402


@pytest.mark.parametrize("s", [1, 2, 4, 8])
def test_nearest_is_block_repetition(s):
    rng = np.random.default_rng(20 + s)
    hc = rng.uniform(0, 1.2, (13, 13))
    assert np.array_equal(ups.upsample(hc, s, "nearest"), np.kron(hc, np.ones((s, s))))
    g = rng.standard_normal((13 * s, 13 * s))
    blocks = g.reshape(13, s, 13, s).sum(axis=(1, 3))
    assert np.allclose(ups.upsample_adjoint(g, s, "nearest"), blocks, rtol=0, atol=1e-12)


def test_lanczos3_closed_form_values():
    pi2 = np.pi ** 2
    x = np.array([0.0, 0.5, -0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.5])
    want = [1.0, 6 / pi2, 6 / pi2, 0.0, -4 / (3 * pi2), 0.0, 0.24 / pi2, 0.0, 0.0]
    assert np.allclose(ups.lanczos3(x), want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("s", [3, 5, 7])
def test_lanczos_interpolates_coarse_samples_at_odd_factor(s):
    """With pixel centres aligned and s odd, fine sample s*i + (s-1)/2 lies
    on coarse sample i, where every other tap sits at a zero of L."""
    rng = np.random.default_rng(30 + s)
    hc = rng.uniform(0, 1.2, (11, 11))
    hf = ups.upsample(hc, s, "lanczos3")
    c = (s - 1) // 2
    assert np.allclose(hf[c::s, c::s], hc, rtol=0, atol=1e-13)


@pytest.mark.parametrize("s", [1, 2, 4, 8, 16])
def test_lanczos_partition_of_unity_and_mirror(s):
    hf = ups.upsample(np.full((9, 9), 0.7), s, "lanczos3")
    assert np.allclose(hf, 0.7, rtol=0, atol=1e-14)
    rng = np.random.default_rng(40 + s)
    hc = rng.standard_normal((9, 9))
    a = ups.upsample(hc[::-1, ::-1], s, "lanczos3")
    b = ups.upsample(hc, s, "lanczos3")[::-1, ::-1]
    assert np.allclose(a, b, rtol=0, atol=1e-13)


def test_lanczos_reproduces_slow_cosine():
    """A cosine of period 16 coarse samples is reproduced at the fine
    positions (away from the edges) to the kernel's approximation error
    (measured 5.9e-3; a half-pixel misalignment of the fine grid gives 0.17)."""
    s, nc, per = 8, 64, 16.0
    i = np.arange(nc)
    hc = np.cos(2 * np.pi * i[:, None] / per) * np.cos(2 * np.pi * i[None, :] / per)
    hf = ups.upsample(hc, s, "lanczos3")
    u = (np.arange(nc * s) + 0.5) / s - 0.5
    want = np.cos(2 * np.pi * u[:, None] / per) * np.cos(2 * np.pi * u[None, :] / per)
    core = slice(8 * s, (nc - 8) * s)
    assert np.max(np.abs(hf[core, core] - want[core, core])) < 1e-2
    # and the nearest kernel does not
    hn = ups.upsample(hc, s, "nearest")
    assert np.max(np.abs(hn[core, core] - want[core, core])) > 0.1


@pytest.mark.parametrize("kind", ["nearest", "lanczos3"])
@pytest.mark.parametrize("s", [2, 3, 8])
def test_upsample_adjoint_dot_product(kind, s):
    rng = np.random.default_rng(50 + s)
    x = rng.standard_normal((10, 10))
    g = rng.standard_normal((10 * s, 10 * s))
    lhs = np.sum(ups.upsample(x, s, kind) * g)
    rhs = np.sum(x * ups.upsample_adjoint(g, s, kind))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) + 1e-12


@pytest.mark.parametrize("n,m,block", [(48, 128, 16), (100, 256, 64), (64, 64, 1000)])
def test_psf_lowmem_equals_psf(n, m, block):
    """The memory-lean single-wavelength PSF (1-D DFTs over blocks of rows and
    columns) is the same definition: it matches psf() to rounding."""
    h = np.random.default_rng(n).uniform(0, 1.2, (n, n))
    a = oracle.psf(h, 0.5, 300.0, m, [0.55], [1.46])
    b = oracle.psf_lowmem(h, 0.5, 300.0, m, 0.55, 1.46, block=block)
    assert rel(b, a) < 1e-12


# ---------------------------------------------------------------------------
# Chromatic behaviour of the wrapped diffractive lens (scalar diffraction
# theory): at wavelength lam the wrapped phase is alpha times the design
# phase, alpha = lam0 (n(lam) - 1) / (lam (n(lam0) - 1)); its first order
# focuses at f(lam) = f0 lam0 / lam with efficiency sinc^2(1 - alpha), times
# sinc^2(1/L) for L uniform height levels.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("lam", [0.45, 0.65])
def test_wrapped_lens_focus_moves_as_one_over_lambda(lam):
    n, m, dx, f0, lam0 = 512, 1024, 1.0, 5000.0, 0.55
    c = n // 2
    h = wl.fresnel_lens_heights(n, dx, f0)
    nl = float(wl.cauchy_index(lam))
    fl = f0 * lam0 / lam
    zs = fl * (1.0 + np.linspace(-0.08, 0.08, 17))
    on_axis = [oracle.psf(h, dx, z, m, [lam], [nl])[c, c] for z in zs]
    assert abs(zs[int(np.argmax(on_axis))] / fl - 1.0) < 1e-9  # the 1 % grid point at f(lam)


@pytest.mark.parametrize("levels", [0, 16])
@pytest.mark.parametrize("lam", [0.45, 0.55, 0.65])
def test_wrapped_lens_first_order_efficiency(lam, levels):
    """Focal intensity of the wrapped (and quantised) lens over that of an
    ideal lens of focal length f(lam) at lam: sinc^2(1 - alpha) sinc^2(1/L)
    (measured within 0.3 %)."""
    n, m, dx, f0, lam0 = 512, 1024, 1.0, 5000.0, 0.55
    c = n // 2
    h = wl.fresnel_lens_heights(n, dx, f0, levels=levels)
    nl, n0 = float(wl.cauchy_index(lam)), float(wl.cauchy_index(lam0))
    fl = f0 * lam0 / lam
    r = wl.pixel_coords(n, dx)
    r2 = r[:, None] ** 2 + r[None, :] ** 2
    ideal = np.exp(-2j * np.pi / lam * (np.sqrt(r2 + fl * fl) - fl))
    i_ideal = abs(oracle.propagate(ideal, m, dx, lam, fl)[c, c]) ** 2
    i_lens = oracle.psf(h, dx, fl, m, [lam], [nl])[c, c]
    alpha = lam0 * (nl - 1.0) / (lam * (n0 - 1.0))
    eta = np.sinc(1.0 - alpha) ** 2 * (np.sinc(1.0 / levels) ** 2 if levels else 1.0)
    assert abs(i_lens / i_ideal / eta - 1.0) < 0.01


# ---------------------------------------------------------------------------
# Rectangular grids (the paper's largest grid is 128,640 x 85,760): every axis
# is padded and sampled in frequency on its own.  An axis mix-up (fx and fy
# swapped, one axis's M used for the other) fails the brute-force sums and
# the rectangular focal spot below.
# ---------------------------------------------------------------------------

def rand_rect(rng, ny, nx):
    return rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))


@pytest.mark.parametrize("my,mx", [(8, 12), (12, 8), (16, 24), (10, 32)])
def test_rect_fft_path_matches_direct_dft(my, mx):
    rng = np.random.default_rng(my * 100 + mx)
    ep = rand_rect(rng, my, mx)
    dx, lam, z = 0.3, 0.5, 7.0
    h = oracle.transfer_function((my, mx), dx, lam, z)
    assert h.shape == (my, mx)
    want = asm.direct_dft2(asm.direct_dft2(ep) * h, inverse=True)
    got = oracle.propagate_padded(ep, dx, lam, z)
    assert rel(got, want) < 1e-12


@pytest.mark.parametrize("my,mx,ny,nx,dx,lam,z", [
    (8, 12, 5, 7, 0.3, 0.5, 3.0),      # evanescent corners on both axes
    (12, 8, 7, 4, 0.3, 0.5, 4.0),
    (10, 16, 10, 9, 0.27, 0.5, 6.0),   # no padding along y
    (16, 6, 9, 6, 1.0, 0.55, 30.0),    # all bins propagate
])
def test_rect_propagate_matches_brute_force(my, mx, ny, nx, dx, lam, z):
    rng = np.random.default_rng(my + mx + ny + nx)
    u = rand_rect(rng, ny, nx)
    got = oracle.propagate(u, (my, mx), dx, lam, z, out_mode="full")
    want = asm.brute_propagate(u, (my, mx), dx, lam, z)
    assert got.shape == (my, mx)
    assert rel(got, want) < 1e-11
    crop = oracle.propagate(u, (my, mx), dx, lam, z)
    py, px = (my - ny) // 2, (mx - nx) // 2
    assert np.array_equal(crop, got[py:py + ny, px:px + nx])


def test_rect_parseval_z0_and_round_trip():
    ny, nx, my, mx, dx, lam, z = 40, 72, 96, 144, 1.0, 0.55, 3000.0
    rng = np.random.default_rng(21)
    u = rand_rect(rng, ny, nx)
    p = oracle.psf(wl.uniform_heights((ny, nx), seed=22), dx, z, (my, mx), [lam], [1.46],
                   out_mode="full")
    assert p.shape == (my, mx) and abs(p.sum() / (ny * nx) - 1.0) < 1e-12
    assert rel(oracle.propagate(u, (my, mx), dx, lam, 0.0, out_mode="full"),
               oracle.embed(u, (my, mx))) < 1e-14
    fwd = oracle.propagate(u, (my, mx), dx, lam, z, out_mode="full")
    assert rel(oracle.propagate_padded(fwd, dx, lam, -z), oracle.embed(u, (my, mx))) < 1e-12


def test_rect_lens_focus_sinc2():
    """Rectangular pupil Ly x Lx focused at f: peak (Ly Lx/(lam f))^2 and the
    focal profile sinc^2(Lx x/(lam f)) along x, sinc^2(Ly y/(lam f)) along y,
    each with its own width (Fresnel numbers 24 and 54, as the square case)."""
    ny, nx, dx, lam, f, nn = 512, 768, 1.0, 0.55, 5000.0, 1.5
    h = wl.ideal_lens_heights((ny, nx), dx, f, lam, nn).astype(np.float64)
    p = oracle.psf(h, dx, f, (2 * ny, 2 * nx), [lam], [nn])
    cy, cx = ny // 2, nx // 2
    ly, lx = ny * dx, nx * dx
    i0 = (ly * lx / (lam * f)) ** 2
    assert abs(p[cy, cx] / i0 - 1.0) < 0.02
    assert np.unravel_index(np.argmax(p), p.shape) == (cy, cx)
    t = np.arange(-12, 13) * dx
    assert np.max(np.abs(p[cy, cx - 12:cx + 13] - i0 * np.sinc(lx * t / (lam * f)) ** 2)) / i0 < 0.02
    assert np.max(np.abs(p[cy - 12:cy + 13, cx] - i0 * np.sinc(ly * t / (lam * f)) ** 2)) / i0 < 0.02


def test_rect_bandlimit_mask_per_bin():
    """Each axis gets the band limit of its own length."""
    my, mx, dx, lam, z = 24, 40, 0.4, 0.6, 150.0
    hb = oracle.transfer_function((my, mx), dx, lam, z, bandlimit=True)
    fly = 1.0 / (lam * np.sqrt((2.0 * z / (my * dx)) ** 2 + 1.0))
    flx = 1.0 / (lam * np.sqrt((2.0 * z / (mx * dx)) ** 2 + 1.0))
    assert fly != flx
    for fu in range(my):
        for fv in range(mx):
            fy, fx = asm._signed_freq(fu, my, dx), asm._signed_freq(fv, mx, dx)
            keep = ((lam * fx) ** 2 + (lam * fy) ** 2 < 1.0 and abs(fx) < flx and abs(fy) < fly)
            assert (hb[fu, fv] != 0) == keep


def test_rect_gradient_adjoint_dot_product():
    """<J dh, G> = <dh, J^T G> for the rectangular PSF's Jacobian J: finite
    differences of the loss along a random direction against the gradient."""
    ny, nx, my, mx, dx, z = 12, 20, 24, 32, 0.5, 40.0
    lams, nidx = [0.5, 0.62], [1.46, 1.455]
    rng = np.random.default_rng(23)
    h = rng.uniform(0, 1.2, (ny, nx))
    g = rng.standard_normal((ny, nx))
    d = rng.standard_normal((ny, nx))
    grad = oracle.psf_backward(h, dx, z, (my, mx), lams, nidx, g)
    eps = 1e-6
    lp = np.sum(g * oracle.psf(h + eps * d, dx, z, (my, mx), lams, nidx))
    lm = np.sum(g * oracle.psf(h - eps * d, dx, z, (my, mx), lams, nidx))
    fd = (lp - lm) / (2 * eps)
    assert abs(fd - np.sum(grad * d)) < 1e-6 * abs(fd)


def test_rect_psf_lowmem_equals_psf():
    h = np.random.default_rng(24).uniform(0, 1.2, (40, 72))
    a = oracle.psf(h, 0.5, 300.0, (96, 160), [0.55], [1.46])
    b = oracle.psf_lowmem(h, 0.5, 300.0, (96, 160), 0.55, 1.46, block=16)
    assert rel(b, a) < 1e-12


def test_psf_lowmem_rows_mode():
    """Selected rows, the sum and the max of the crop without holding it: the
    same values as the whole-crop result."""
    h = np.random.default_rng(25).uniform(0, 1.2, (40, 72))
    full = oracle.psf_lowmem(h, 0.5, 300.0, (96, 160), 0.55, 1.46, block=16)
    rows = [0, 7, 15, 16, 33, 39]
    got, total, peak = oracle.psf_lowmem(h, 0.5, 300.0, (96, 160), 0.55, 1.46, block=16, rows=rows)
    assert np.array_equal(got, full[rows])
    assert abs(total - full.sum()) < 1e-12 * full.sum() and peak == full.max()


@pytest.mark.parametrize("kind", ["nearest", "lanczos3"])
def test_rect_upsample_separable_and_adjoint(kind):
    """Rectangular designs: the upsampling of an outer product a b^T is the
    outer product of the two one-axis upsamplings (an axis mix-up breaks it),
    nearest is block repetition, and the adjoint identity holds."""
    rng = np.random.default_rng(26)
    s, ncy, ncx = 3, 7, 12
    a, b = rng.standard_normal(ncy), rng.standard_normal(ncx)
    fine = ups.upsample(np.outer(a, b), s, kind)
    assert fine.shape == (ncy * s, ncx * s)
    fa = ups.upsample(np.outer(a, np.ones(1)), s, kind)[:, 0]
    fb = ups.upsample(np.outer(np.ones(1), b), s, kind)[0]
    assert np.allclose(fine, np.outer(fa, fb), rtol=0, atol=1e-13)
    x = rng.standard_normal((ncy, ncx))
    g = rng.standard_normal((ncy * s, ncx * s))
    lhs = np.sum(ups.upsample(x, s, kind) * g)
    rhs = np.sum(x * ups.upsample_adjoint(g, s, kind))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) + 1e-12
    if kind == "nearest":
        assert np.array_equal(ups.upsample(x, s, kind), np.kron(x, np.ones((s, s))))
