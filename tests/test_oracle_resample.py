"""Pins of the oracle's non-integer resampling: subapertures that are not a
whole number of pupil pixels (the SOUL pyramid has 40 subapertures on a
220 px pupil, 5.5 px each, Appendix B) and a detector whose pitch is not a
whole number of transform pixels (its 660 transform pixels are read out on
a 120 px CCD, 5.5 each).  Area weighting is checked against a different
route to the same sums: replicate every pixel into an m x m grid of equal
sub-pixels (each holding 1/m^2 of it) so that every edge falls on the finer
grid, then take plain block sums.  On top: flux conservation, the integer
case, the paper's SOUL detector geometry, and the noise-free detector's
slopes equal to the sensor's own (the two binning routes compose)."""

from fractions import Fraction

import numpy as np

from oracle import ccd as C
from oracle import pwfs as O
from workloads import FLAG_REF_SLOPES, tiny_sensor, von_karman_opd


def _replicate(a: np.ndarray, m: int) -> np.ndarray:
    return np.kron(a, np.ones((m, m))) / float(m * m)


def _soul_like():
    # 44 px pupil, 8 subapertures (5.5 px), images 66 px apart on a 128 grid
    return tiny_sensor(n_pupil=44, n_fft=128, n_subap=8, pupil_sep_px=66.0, n_mod=8, mod_radius_lod=2.0,
                       flags=FLAG_REF_SLOPES)


def test_fractional_subaperture_binning_equals_replication():
    s = _soul_like()
    rng = np.random.default_rng(3)
    I = rng.random((2, 128, 128))
    Q = O.bin_images(I, s)
    D, n = s.n_pupil, s.n_subap
    for q, (r0, c0) in enumerate(O.image_origins(s)):
        for f in range(2):
            up = _replicate(I[f, r0:r0 + D, c0:c0 + D], n)     # subaperture = D x D sub-pixels
            want = up.reshape(n, D, n, D).sum(axis=(1, 3))
            np.testing.assert_allclose(Q[f, q], want, rtol=1e-13)
    # flux: the subapertures partition each image
    for q, (r0, c0) in enumerate(O.image_origins(s)):
        np.testing.assert_allclose(Q[:, q].sum(axis=(1, 2)), I[:, r0:r0 + D, c0:c0 + D].sum(axis=(1, 2)),
                                   rtol=1e-13)


def test_integer_subapertures_unchanged_by_the_weights():
    s = tiny_sensor(n_pupil=40, n_fft=128, n_subap=5, pupil_sep_px=48.0)
    rng = np.random.default_rng(4)
    I = rng.random((1, 128, 128))
    Q = O.bin_images(I, s)
    W = O.subaperture_overlaps(40, 5) / 5
    for q, (r0, c0) in enumerate(O.image_origins(s)):
        np.testing.assert_allclose(Q[0, q], W @ I[0, r0:r0 + 40, c0:c0 + 40] @ W.T, rtol=1e-13)


def test_fractional_valid_map_equals_replication():
    for D, n, ob in ((44, 8, 0.0), (220, 40, 0.0), (64, 15, 0.3), (50, 12, 0.12)):
        s = tiny_sensor(n_pupil=D, n_subap=n, obstruction=ob)
        A = O.pupil_amplitude(D, ob)
        lit = np.kron(A, np.ones((n, n))).reshape(n, D, n, D).sum(axis=(1, 3))    # lit sub-pixels
        np.testing.assert_array_equal(O.valid_subapertures(s), 2 * lit >= D * D)
        assert (O.valid_subapertures(s) == O.valid_subapertures(s).T).all()


def test_detector_fractional_pitch_equals_replication():
    rng = np.random.default_rng(5)
    I = rng.random((128, 128)).astype(np.float32)
    lam = C.expected_electrons(I, 20, Fraction(11, 2), 3.0)
    win = I[9:119, 9:119].astype(np.float64)                     # 20 x 5.5 = 110 px, centred
    want = 3.0 * _replicate(win, 2).reshape(20, 11, 20, 11).sum(axis=(1, 3))
    np.testing.assert_allclose(lam, want, rtol=1e-14)
    np.testing.assert_allclose(lam.sum(), 3.0 * win.sum(), rtol=1e-13)
    # a pitch of 8/3 transform pixels: replicate by 3, blocks of 8
    lam = C.expected_electrons(I, 30, Fraction(8, 3), 1.0)
    win = I[24:104, 24:104].astype(np.float64)
    want = _replicate(win, 3).reshape(30, 8, 30, 8).sum(axis=(1, 3))
    np.testing.assert_allclose(lam, want, rtol=1e-14)


def test_detector_integer_pitch_is_the_block_sum_bit_for_bit():
    rng = np.random.default_rng(6)
    I = rng.random((64, 64)).astype(np.float32)
    lam = C.expected_electrons(I, 12, 4, 1.0)
    assert np.array_equal(lam, C.expected_electrons(I, 12, Fraction(8, 2), 1.0))
    win = I[8:56, 8:56].astype(np.float64)
    s = np.zeros((12, 12))
    for i in range(4):
        for j in range(4):
            s = s + win[i::4, j::4]
    assert np.array_equal(lam, s)


def test_soul_detector_geometry():
    # Appendix B: 40 subapertures across a pupil image, pupil centres 48
    # subapertures apart, a 120 x 120 detector; 220 px pupil, 5.5 transform
    # pixels per detector pixel (on a 768 grid here)
    s = tiny_sensor(n_pupil=220, n_fft=768, n_subap=40, pupil_sep_px=264.0)
    org, img, b = C.detector_geometry(s, 120, Fraction(11, 2))
    assert img == 40 and b == 1
    assert sorted(set(r for r, _ in org)) == [16, 64] and sorted(set(c for _, c in org)) == [16, 64]
    assert 64 - 16 == 48


def test_noise_free_detector_slopes_equal_sensor_slopes():
    s = _soul_like()
    opd = von_karman_opd(2, s.n_pupil, 8.0, 0.5, 25.0, seed=8)
    I = O.forward(opd, s)
    want, _ = O.slopes(I, s)
    P = C.detector(I.astype(np.float32), 20, Fraction(11, 2), 1.0e5, 0, 0.0, 0)
    got, _ = C.detector_slopes(P, s, 20, Fraction(11, 2))
    np.testing.assert_allclose(got, want, atol=1e-6)
    assert np.abs(want).max() > 1e-2
