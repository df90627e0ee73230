"""Pins of the square field stop in the oracle (Appendix B names a field of
view, 'fov'; the square shape is the reading, see oracle/pwfs.py): a stop
wider than the grid changes nothing, the flux equals the focal-plane energy
inside the stop computed from the focal field directly (Parseval on the
other side of the mask), a direct 2-D sum on a tiny grid, the sky-angle
scaling with wavelength, the blocking of a modulation circle larger than
the stop, and equal light in both arms of a double roof."""

import numpy as np
import pytest

from oracle import pwfs as O
from workloads import FLAG_DOUBLE_ROOF, FLAG_FULL_PLANE, tiny_sensor, von_karman_opd


def _s(**kw):
    base = dict(n_pupil=16, n_fft=64, n_subap=4, n_mod=8, pupil_sep_px=24.0, mod_radius_lod=2.0,
                obstruction=0.2, flags=FLAG_FULL_PLANE)
    base.update(kw)
    return tiny_sensor(**base)


def test_wide_stop_changes_nothing():
    opd = von_karman_opd(1, 16, 8.0, 0.5, 25.0, seed=1)
    a = O.forward(opd, _s())
    b = O.forward(opd, _s(fov_lod=40.0))            # side 160 samples > 2 N: every sample passes
    assert np.array_equal(a, b)


@pytest.mark.parametrize("fov", [3.0, 6.5, 9.0])
def test_flux_is_the_focal_energy_inside_the_stop(fov):
    s = _s(fov_lod=fov)
    opd = von_karman_opd(1, 16, 8.0, 0.5, 25.0, seed=2)[0].astype(np.float64)
    I = O.forward_frame(opd, s)
    A = O.pupil_amplitude(16, s.obstruction)
    T = O.field_stop(s, s.lambdas_nm[0])
    E0 = A * np.exp(2j * np.pi * opd / s.lambdas_nm[0])
    e = 0.0
    for t in O.modulation_angles(s.n_mod):
        F = O.focal_field(E0 * O.modulation_ramp(16, s.mod_radius_lod, t), 64)
        e += (np.abs(F) ** 2 * (T[:, None] * T[None, :])).sum() / 64 ** 2
    want = e / (s.n_mod * (A * A).sum())
    assert abs(I.sum() - want) < 1e-14
    assert want < 1.0


def test_direct_sum_with_stop():
    s = tiny_sensor(fov_lod=2.5, obstruction=0.0)          # D = 8, N = 16: side 5 samples
    N, D, S = s.n_fft, s.n_pupil, s.pupil_sep_px
    opd = np.random.default_rng(3).standard_normal((D, D)) * 150.0
    got = O.forward_frame(opd, s)
    o = (N - D) // 2
    idx = np.arange(N)
    ub = np.array([u + 0.5 if u < N // 2 else u - N + 0.5 for u in range(N)])
    stop = (2 * np.abs(ub) <= 2.5 * N / D).astype(float)
    M = np.exp(1j * np.pi * S * (np.abs(ub)[None, :] + np.abs(ub)[:, None]) / N) * stop[None, :] * stop[:, None]
    W = np.exp(-2j * np.pi * np.outer(idx, idx) / N)
    A = O.pupil_amplitude(D, 0.0)
    I = np.zeros((N, N))
    for k in range(s.n_mod):
        th = 2 * np.pi * k / s.n_mod
        E = np.zeros((N, N), complex)
        for Y in range(D):
            for X in range(D):
                x, y = X - (D - 1) / 2, Y - (D - 1) / 2
                E[o + Y, o + X] = A[Y, X] * np.exp(2j * np.pi * (opd[Y, X] / s.lambdas_nm[0] + s.mod_radius_lod
                                                              * (x * np.cos(th) + y * np.sin(th)) / D))
        E *= np.exp(-1j * np.pi * (idx[:, None] + idx[None, :]) / N)
        G = (W @ E @ W.T) * M
        e = np.conj(W) @ G @ np.conj(W).T / N ** 2
        I += np.abs(e) ** 2
    I /= s.n_mod * (A * A).sum()
    assert np.abs(got - I).max() <= 1e-12 * np.abs(I).max()


def test_stop_is_a_sky_angle():
    opd = von_karman_opd(1, 16, 8.0, 0.5, 25.0, seed=4).astype(np.float32).astype(np.float64)
    a = O.forward(opd, _s(fov_lod=5.0, lambdas_nm=(750.0,), lambda_ref_nm=750.0))
    b = O.forward(opd * 2.0, _s(fov_lod=5.0, lambdas_nm=(1500.0,), lambda_ref_nm=1500.0))
    assert np.abs(a - b).max() < 1e-15
    # given at 750 nm and sensed at 1500 nm, stop and modulation radius are
    # both half as many lambda/D as at 750: the same as giving them at 1500
    c = O.forward(opd, _s(fov_lod=5.0, mod_radius_lod=2.0, lambdas_nm=(1500.0,), lambda_ref_nm=750.0))
    d = O.forward(opd, _s(fov_lod=2.5, mod_radius_lod=1.0, lambdas_nm=(1500.0,), lambda_ref_nm=1500.0))
    assert np.abs(c - d).max() < 1e-15
    assert np.abs(c - O.forward(opd, _s(mod_radius_lod=1.0, lambdas_nm=(1500.0,), lambda_ref_nm=1500.0))).max() > 1e-6


def test_modulation_outside_the_stop_is_blocked():
    flat = np.zeros((1, 16, 16))
    small = O.forward(flat, _s(mod_radius_lod=4.0, fov_lod=2.0)).sum()
    large = O.forward(flat, _s(mod_radius_lod=4.0, fov_lod=14.0)).sum()
    assert small < 0.15 and large > 0.9


def test_double_roof_arms_get_equal_light_through_the_stop():
    s = _s(fov_lod=6.0, flags=FLAG_FULL_PLANE | FLAG_DOUBLE_ROOF)
    opd = von_karman_opd(1, 16, 8.0, 0.5, 25.0, seed=5)[0]
    I = O.forward_frame(opd, s)
    plain = O.forward_frame(opd, _s(fov_lod=6.0)).sum()
    np.testing.assert_allclose(I.sum(axis=(1, 2)), [0.5 * plain, 0.5 * plain], rtol=1e-13)
