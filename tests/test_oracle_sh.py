"""Pins of the Shack-Hartmann oracle (oracle/sh.py): a brute-force direct sum
of the focal field at the half-integer frequencies, Parseval per
subaperture, zero centroids and point-symmetric spots for a flat
wavefront, the tilt response (a tilt of t lambda/d moves the spot by
t M / b focal pixels), binning conservation, and the valid count of the
paper's SCAO SH geometry (Table 2: 160 px pupil, 20 x 20 subapertures, 314)
to within its pixelisation."""

import numpy as np
import pytest

from oracle import pwfs as O
from oracle import sh as SH
from workloads import tilt_opd


def test_brute_force_direct_sum():
    D, n, M, lam = 8, 2, 8, 750.0
    rng = np.random.default_rng(1)
    opd = rng.normal(0, 60.0, (D, D))
    got = SH.spots(opd, D, n, M, 0.0, lam)[0]
    A = O.pupil_amplitude(D, 0.0)
    E = A * np.exp(2j * np.pi * opd / lam)
    b = D // n
    c = np.arange(b) - (b - 1) / 2.0
    f = np.arange(M) - M / 2.0 + 0.5
    for i in range(n):
        for j in range(n):
            blk = E[i * b:(i + 1) * b, j * b:(j + 1) * b]
            F = np.zeros((M, M), complex)
            for v in range(M):
                for u in range(M):
                    F[v, u] = (blk * np.exp(-2j * np.pi * (f[u] * c[None, :] + f[v] * c[:, None]) / M)).sum()
            want = np.abs(F) ** 2 / (M * M * (A * A).sum())
            np.testing.assert_allclose(got[i, j], want, atol=1e-15)


def test_parseval_per_subaperture():
    D, n, M = 32, 4, 24
    rng = np.random.default_rng(2)
    opd = rng.normal(0, 200.0, (2, D, D))
    sp = SH.spots(opd, D, n, M, 0.25, 750.0)
    A = O.pupil_amplitude(D, 0.25)
    b = D // n
    per = (A * A).reshape(n, b, n, b).sum(axis=(1, 3)) / (A * A).sum()
    np.testing.assert_allclose(sp.sum(axis=(-2, -1)), np.broadcast_to(per, (2, n, n)), atol=1e-13)
    pix = SH.detector(sp, 3)
    np.testing.assert_allclose(pix.sum(axis=(-2, -1)), sp.sum(axis=(-2, -1)), atol=1e-14)


@pytest.mark.parametrize("M,rebin", [(16, 2), (21, 3)])
def test_flat_wavefront_centred_and_symmetric(M, rebin):
    D, n = 24, 3
    pix, sl = SH.forward(np.zeros((1, D, D)), D, n, M, rebin, 0.0, 750.0)
    assert np.abs(sl).max() < 1e-12
    # a real aperture function has a point-symmetric spot |F(f)| = |F(-f)|
    # (edge subapertures are not mirror-symmetric per axis)
    sp = SH.spots(np.zeros((D, D)), D, n, M, 0.0, 750.0)[0]
    np.testing.assert_allclose(sp, sp[:, :, ::-1, ::-1], atol=1e-16)


def test_tilt_moves_the_spot_by_t_M_over_b():
    D, n, M, rebin = 64, 4, 64, 4          # b = 16, 4 focal px per lambda/d, detector px = lambda/d
    t = 0.3                                # lambda/d_sub
    opd = tilt_opd(D, t * n, 0.0, 750.0)    # t lambda/d = t n lambda/D
    pix, sl = SH.forward(opd[None], D, n, M, rebin, 0.0, 750.0)
    valid = SH.valid_subapertures(D, n, 0.0)
    want = t * M / (D // n) / rebin
    inner = valid.copy()
    inner[[0, -1], :] = False
    inner[:, [0, -1]] = False                # fully illuminated subapertures
    assert np.abs(sl[0, 0][inner] / want - 1.0).max() < 0.03
    assert np.abs(sl[0, 1][inner]).max() < 1e-10


def test_scao_valid_count():
    # Table 2 gives 314 for this geometry; the half-illumination reading on
    # this pupil pixelisation gives 316 (counts move in steps of 8 by the
    # pupil's symmetry, so 314 is not reachable with it): within 1 %
    nv = SH.valid_subapertures(160, 20, 0.0).sum()
    assert nv == 316 and abs(nv / 314 - 1) < 0.01


# ------------------------------------------------- polychromatic sensor ----

def test_poly_at_the_reference_wavelength_is_the_fft_sensor():
    """One wavelength equal to the reference (s = 1): the matrix products of
    the definition reproduce the FFT-based monochromatic oracle."""
    D, n, M = 24, 3, 20
    rng = np.random.default_rng(21)
    opd = rng.normal(0, 80.0, (2, D, D))
    want = SH.spots(opd, D, n, M, 0.2, 700.0)
    got = SH.spots_poly(opd, D, n, M, 0.2, 700.0, [700.0], [1.0])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * want.max())


def test_poly_is_the_weighted_sum_of_its_wavelengths():
    D, n, M = 16, 2, 16
    rng = np.random.default_rng(22)
    opd = rng.normal(0, 60.0, (D, D))
    lams, ws = [600.0, 750.0, 900.0], [0.2, 0.3, 0.5]
    got = SH.spots_poly(opd, D, n, M, 0.0, 600.0, lams, ws)
    parts = [SH.spots_poly(opd, D, n, M, 0.0, 600.0, [l], [1.0]) for l in lams]
    np.testing.assert_allclose(got, sum(w * p for w, p in zip(ws, parts)), rtol=1e-12, atol=1e-16)


def test_poly_centroid_is_achromatic():
    """A pure tilt moves the spot by the same angle at every wavelength (the
    phase gradient 2 pi t / lambda is sampled at frequencies scaled by
    lambda_ref / lambda), so the centre of gravity agrees at 600, 750 and
    900 nm to within the bias of the grid truncating each spot's wings (the
    spot widens with lambda): 1.11, 1.13, 1.12 px against the geometric 1.2.
    Frequencies left unscaled would give 1.2 x 600 / 900 = 0.8 px at 900 nm.
    At the reference wavelength it equals the monochromatic sensor's."""
    D, n, M, rebin = 32, 4, 32, 2
    opd = tilt_opd(D, 0.6 * n, 0.0, 600.0)     # 0.6 lambda_ref / d of tip (0.6 n lambda_ref / D)
    cents = []
    for lam in (600.0, 750.0, 900.0):
        pix, sl = SH.forward_poly(opd, D, n, M, rebin, 0.0, 600.0, [lam], [1.0])
        cents.append(sl[0, 0][SH.valid_subapertures(D, n, 0.0)].mean())
    _, sl_mono = SH.forward(opd, D, n, M, rebin, 0.0, 600.0)
    assert abs(cents[0] - sl_mono[0, 0][SH.valid_subapertures(D, n, 0.0)].mean()) < 1e-12
    assert 1.0 < cents[0] < 1.2
    for c in cents[1:]:
        assert abs(c / cents[0] - 1) < 2.5e-2


def test_poly_flat_frame_keeps_the_light_on_the_grid():
    """Flat wavefront: at the reference wavelength the spots hold all the
    light (Parseval); at longer wavelengths the s^2 factor keeps each spot's
    energy equal to the fraction that falls on the grid, just below 1 for a
    grid that spans several diffraction widths."""
    D, n, M = 32, 4, 64
    opd = np.zeros((D, D))
    for lam, lo in ((600.0, 1.0 - 1e-12), (900.0, 0.93)):
        tot = SH.spots_poly(opd, D, n, M, 0.0, 600.0, [lam], [1.0]).sum()
        assert lo <= tot <= 1.0 + 1e-12, (lam, tot)


@pytest.mark.parametrize("k", [2, 3])
def test_poly_at_an_integer_fraction_is_the_centre_of_a_finer_fft_sensor(k):
    """At s = 1/k (lambda = k lambda_ref) the frequencies (u - M/2 + 1/2) / (k M)
    are those of the FFT sensor on k M samples at indices u + (k - 1) M / 2, and
    s^2 / M^2 = 1 / (k M)^2: the scaled grid is exactly the central M x M block
    of that finer sensor's spot (an FFT of a zero-padded block, a different
    method), which pins the frequency scale, its sign and the s^2 factor."""
    D, n, M = 24, 3, 12
    rng = np.random.default_rng(30 + k)
    opd = rng.normal(0, 90.0, (2, D, D))
    lam = 600.0 * k
    got = SH.spots_poly(opd, D, n, M, 0.15, 600.0, [lam], [1.0])
    fine = SH.spots(opd, D, n, k * M, 0.15, lam)
    o = (k - 1) * M // 2
    want = fine[..., o:o + M, o:o + M]
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * want.max())
