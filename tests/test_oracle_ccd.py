"""Pins of the detector-stage oracle (oracle/ccd.py) against facts that do
not come from it: numpy's own Philox4x64-10, scipy's Poisson quantile
function and distributions, the variance laws of photon, excess and readout
noise, and the sensor oracle's slopes for a noise-free detector."""

import math

import numpy as np
import pytest
from scipy import stats

from oracle import ccd as C
from oracle import pwfs as O
from workloads import tiny_sensor

M64 = (1 << 64) - 1


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((123, 456), (7, 0, 0, 0)),
                                     ((M64, 5), (M64, 3, 9, 11))])
def test_philox_matches_numpy(key, ctr):
    # numpy's generator returns the block of counter + 1 (carry into word 1)
    bg = np.random.Philox(counter=np.array(ctr, np.uint64), key=np.array(key, np.uint64))
    want = [int(x) for x in bg.random_raw(4)]
    c0 = (ctr[0] + 1) & M64
    c1 = ctr[1] + (1 if c0 == 0 else 0)
    got = C.philox4x64(np.uint64(c0), np.uint64(c1), np.uint64(ctr[2]), np.uint64(ctr[3]), key[0], key[1])
    assert [int(x) for x in got] == want


def test_uniform_and_normal():
    assert C.uniform(np.uint64(0)) == 0.0
    assert C.uniform(np.uint64(M64)) == 1.0 - 2.0 ** -53
    w = C.philox4x64(np.arange(40000, dtype=np.uint64), 1, 2, 3, 99, 0)
    u = C.uniform(w[0])
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    z = C.box_muller(w[1], w[2])
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_exp_neg_against_libm():
    mu = np.concatenate([np.linspace(0, 256, 2001), [1e-9, 0.37, 255.999]])
    assert np.max(np.abs(C.exp_neg(mu) / np.exp(-mu) - 1.0)) < 1e-12


def test_poisson_inversion_is_the_quantile_function():
    rng = np.random.default_rng(3)
    mu = rng.uniform(0.01, 256.0, 5000)
    u = rng.uniform(0.0, 1.0, 5000)
    k = C.poisson_inversion(mu, u)
    ref = stats.poisson.ppf(u, mu).astype(np.int64)
    # away from the CDF steps (where float64 rounding decides) they agree exactly
    F = stats.poisson.cdf(ref, mu)
    Fm = stats.poisson.cdf(ref - 1, mu)
    far = (np.abs(u - F) > 1e-9) & (np.abs(u - Fm) > 1e-9)
    assert far.mean() > 0.99
    np.testing.assert_array_equal(k[far], ref[far])
    assert (C.poisson_inversion(np.array([0.5]), np.array([0.0])) == 0).all()


@pytest.mark.parametrize("lam", [0.3, 3.7, 40.0, 700.0])
def test_poisson_moments(lam):
    n = 40000
    pix = np.arange(n, dtype=np.uint64)
    k = C.poisson(np.full(n, lam), pix, 5, (11, 0))
    assert abs(k.mean() - lam) < 5 * math.sqrt(lam / n)
    assert abs(k.var() / lam - 1.0) < 5 * math.sqrt(2.0 / n) + 0.01
    if lam < 256:
        # one inversion: the first counter block's uniform decides it
        u = C.uniform(C.philox4x64(pix[:200], 5, C.P_PHOTON, 0, 11, 0)[0])
        np.testing.assert_array_equal(k[:200], stats.poisson.ppf(u, lam).astype(np.int64))


@pytest.mark.parametrize("shape", [1.0, 5.0, 60.0])
def test_gamma_distribution(shape):
    n = 20000
    g = C.gamma_mt(np.full(n, shape), np.arange(n, dtype=np.uint64), 2, (7, 0))
    assert stats.kstest(g, stats.gamma(shape).cdf).pvalue > 1e-3


def _flat_intensity(N, seed=1):
    rng = np.random.default_rng(seed)
    I = rng.uniform(0.0, 1.0, (N, N)).astype(np.float32)
    return (I / I.sum()).astype(np.float32)


def test_expected_electrons_conserves_flux_and_noise_free_is_expectation():
    I = _flat_intensity(64)
    lam = C.expected_electrons(I, 12, 4, 1000.0)
    win = I[8:56, 8:56].astype(np.float64)
    assert abs(lam.sum() - 1000.0 * win.sum()) < 1e-9
    assert abs(lam[3, 5] - 1000.0 * win[12:16, 20:24].sum()) < 1e-12
    P = C.detector_frame(I, 12, 4, 1000.0, 0, 0.0, 1, 0)
    np.testing.assert_array_equal(P, lam)


def test_noise_variance_laws():
    # uniform illumination: every pixel has the same mean, so pixel statistics are draw statistics
    N, n_det, r = 256, 64, 4
    I = np.full((N, N), 1.0 / (N * N), np.float32)
    e = 30.0 * N * N / (r * r)          # 30 electrons per detector pixel
    lam = 30.0
    p = C.detector_frame(I, n_det, r, e, C.PHOTON, 0.0, 3, 0)
    assert abs(p.mean() - lam) < 0.5 and abs(p.var() / lam - 1) < 0.1
    assert np.all(p == np.round(p))
    x = C.detector_frame(I, n_det, r, e, C.PHOTON | C.EXCESS, 0.0, 3, 0)
    assert abs(x.mean() - lam) < 0.6 and abs(x.var() / (2 * lam) - 1) < 0.1   # excess factor sqrt(2)
    ro = C.detector_frame(I, n_det, r, e, C.READOUT, 2.5, 3, 0)
    d = ro - lam
    assert abs(d.mean()) < 0.15 and abs(d.std() / 2.5 - 1) < 0.05
    with pytest.raises(ValueError):
        C.detector_frame(I, n_det, r, e, C.EXCESS, 0.0, 3, 0)


def test_frames_and_seeds_key_the_draws():
    I = _flat_intensity(64)[None].repeat(2, axis=0)
    a = C.detector(I, 16, 4, 5e4, C.PHOTON | C.READOUT, 1.0, seed=9, frame0=10)
    b = C.detector(I[:1], 16, 4, 5e4, C.PHOTON | C.READOUT, 1.0, seed=9, frame0=11)
    np.testing.assert_array_equal(a[1], b[0])          # frame index, not position in the batch
    assert not np.array_equal(a[0], a[1])
    c = C.detector(I[:1], 16, 4, 5e4, C.PHOTON | C.READOUT, 1.0, seed=8, frame0=10)
    assert not np.array_equal(a[0], c[0])


def test_noise_free_detector_slopes_equal_sensor_slopes():
    s = tiny_sensor(n_pupil=32, n_fft=64, n_subap=8, n_mod=8, pupil_sep_px=32.0, mod_radius_lod=2.0,
                    obstruction=0.2)
    rng = np.random.default_rng(4)
    opd = rng.normal(0.0, 60.0, (2, 32, 32))
    I = O.forward(opd, s)
    want, _ = O.slopes(I, s)
    P = C.detector(I.astype(np.float32), 16, 4, 1.0, 0, 0.0, 0)
    got, flux = C.detector_slopes(P, s, 16, 4)
    valid = O.valid_subapertures(s)
    assert O.slope_rel_rms(got, want, valid) < 1e-6
    with pytest.raises(ValueError):
        C.detector_geometry(s, 15, 4)


def test_poisson_bounds():
    pix = np.arange(4, dtype=np.uint64)
    k = C.poisson(np.array([-1.0, 0.0, np.inf, 2.0 ** 24 + 1]), pix, 0, (1, 0))
    assert k[0] == 0 and k[1] == 0 and np.isnan(k[2]) and np.isnan(k[3])


def test_basic_operation_elementary_functions():
    """The samplers' log, sqrt and cos(2 pi u), built from + - * / and exact
    power-of-two scalings only, agree with the math library to a few ulp over
    their whole ranges of use (u in (0, 1], Gamma shapes up to 2^24, v^3 of
    the Marsaglia-Tsang step, normals' radius)."""
    x = np.concatenate([np.geomspace(1e-300, 1e300, 20001), np.linspace(0.01, 4.0, 100001),
                        1.0 - np.geomspace(2.0 ** -53, 0.5, 1001)])
    ref = np.log(x)
    big = np.abs(ref) > 1e-3
    assert (np.abs(C.log_basic(x) - ref)[big] / np.abs(ref[big])).max() < 1e-15
    assert np.abs(C.log_basic(x) - ref)[~big].max() < 1e-18
    assert C.log_basic(np.array([1.0]))[0] == 0.0
    y = np.concatenate([[0.0], np.geomspace(1e-300, 1e300, 20001), np.linspace(0.0, 100.0, 100001)])
    r = np.sqrt(y)
    assert (np.abs(C.sqrt_basic(y) - r) / np.maximum(r, 1e-300)).max() < 5e-16
    assert C.sqrt_basic(np.array([4.0, 0.0]))[0] == 2.0
    u = np.linspace(0.0, 1.0, 1_000_001, endpoint=False)
    assert np.abs(C.cos_2pi_basic(u) - np.cos(2.0 * np.pi * u)).max() < 1e-15
    assert C.cos_2pi_basic(np.array([0.0]))[0] == 1.0 and C.cos_2pi_basic(np.array([0.5]))[0] == -1.0
