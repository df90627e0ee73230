"""Pins of the closed-loop oracle (oracle/loop.py): bilinear periodic sampling
against np.roll and exact linear functions, frozen-flow translation, the
integrator's closed form, the delay line, and the loop's physics: a static
aberration inside the mirror's modal space is driven to zero, the commands
converge to its modal coefficients, and nothing moves before the delay."""

import numpy as np
import pytest

from oracle import loop as L
from oracle import pwfs as O
from workloads import tiny_sensor
from workloads.modes import kl_modes


def test_bilinear_integer_shift_is_roll_and_half_pixel_is_mean():
    rng = np.random.default_rng(0)
    S = rng.normal(size=(16, 20))
    y, x = np.mgrid[0:16, 0:20].astype(float)
    np.testing.assert_allclose(L.bilinear_periodic(S, x + 3, y - 2), np.roll(S, (2, -3), axis=(0, 1)), atol=1e-15)
    h = L.bilinear_periodic(S, x + 0.5, y)
    np.testing.assert_allclose(h, 0.5 * (S + np.roll(S, -1, axis=1)), atol=1e-15)
    # wrap: coordinate n_c - 0.25 mixes the last and the first column
    v = L.bilinear_periodic(S, np.array([19.75]), np.array([4.0]))
    assert abs(v[0] - (0.25 * S[4, 19] + 0.75 * S[4, 0])) < 1e-15


def test_bilinear_reproduces_linear_functions():
    y, x = np.mgrid[0:32, 0:32].astype(float)
    S = 0.3 * x - 1.7 * y + 2.0
    X = np.array([3.2, 10.75, 20.5])
    Y = np.array([7.9, 1.25, 30.0])
    np.testing.assert_allclose(L.bilinear_periodic(S, X, Y), 0.3 * X - 1.7 * Y + 2.0, atol=1e-12)


def test_frozen_flow_translation_and_linearity():
    rng = np.random.default_rng(1)
    scr = rng.normal(size=(2, 40, 40))
    a = L.layers_opd(scr, [1.0, 0.0], [(2, 3), (0, 0)], [(1.0, 0.0), (0, 0)], 4, 8)
    b = L.layers_opd(scr, [1.0, 0.0], [(6, 3), (0, 0)], [(0.0, 0.0), (0, 0)], 0, 8)
    np.testing.assert_allclose(a, b, atol=1e-15)
    both = L.layers_opd(scr, [0.5, 2.0], [(2, 3), (5, 1)], [(0.3, 0.1), (-0.2, 0.7)], 7, 8)
    one = L.layers_opd(scr[:1], [0.5], [(2, 3)], [(0.3, 0.1)], 7, 8)
    two = L.layers_opd(scr[1:], [2.0], [(5, 1)], [(-0.2, 0.7)], 7, 8)
    np.testing.assert_allclose(both, one + two, atol=1e-13)


@pytest.mark.parametrize("ff", [1.0, 0.97])
def test_integrator_closed_form(ff):
    g = np.array([0.4, 0.55])
    f = np.array([ff, ff])
    m = np.array([2.0, -1.0])
    c = np.zeros(2)
    for t in range(25):
        c = L.integrator_step(c, m, g, f)
    want = g * m * (25 if ff == 1.0 else (1 - ff ** 25) / (1 - ff))
    np.testing.assert_allclose(c, want, rtol=1e-12)
    np.testing.assert_array_equal(L.group_vector([0.5, 0.2], [2, 3]), [0.5, 0.5, 0.2, 0.2, 0.2])


def _small_loop_parts(n_modes=10):
    s = tiny_sensor(n_pupil=32, n_fft=64, n_subap=8, n_mod=8, pupil_sep_px=32.0, mod_radius_lod=3.0,
                    obstruction=0.0)
    Z, _ = kl_modes(32, 0.0, 8.0, 25.0, n_modes)
    B = Z.T.copy()                                   # nm per unit command, unit RMS modes
    delta = 5.0
    cols = []
    for j in range(n_modes):
        sp, _ = O.slopes(O.forward((delta * Z[j]).reshape(1, 32, 32), s), s)
        sm, _ = O.slopes(O.forward((-delta * Z[j]).reshape(1, 32, 32), s), s)
        cols.append(((sp - sm) / (2 * delta)).ravel())
    IM = np.array(cols).T                            # [slopes][modes]
    R = np.linalg.pinv(IM)
    return s, Z, B, IM, R


def test_static_aberration_is_corrected():
    s, Z, B, IM, R = _small_loop_parts()
    np.testing.assert_allclose(R @ IM, np.eye(10), atol=1e-9)
    a = np.array([12.0, -8.0, 5.0, 3.0, -4.0, 2.0, 1.5, -1.0, 2.5, -2.0])      # nm RMS per mode
    scr = (Z.T @ a).reshape(1, 32, 32)
    r = L.run(s, scr, [1.0], [(0, 0)], [(0, 0)], B, R, np.full(10, 0.5), np.ones(10), 2, 30)
    rms = r["residual_rms"]
    assert rms[0] == rms[1]                          # nothing applied before the delay
    assert rms[2] < 0.7 * rms[1]
    assert rms[-1] < 0.02 * rms[0]
    np.testing.assert_allclose(r["commands"][-1], a, rtol=0.02, atol=0.2)
