"""Pins of the double-roof sensor in the oracle (Table 4: ModulatedDoubleRoof
and DoubleRoofSlopec; arms and slope form are readings, stated in
oracle/pwfs.py): a direct 2-D sum of each arm with no FFT, Parseval (half
the light per arm), the zero-separation limit (each arm images the pupil),
mirror symmetry and zero reference-subtracted slopes for a flat wavefront,
a signed linear tilt response on the right axis only, and the
geometric-optics gain 2 / (pi r) of a large modulation, the same as the
pyramid's."""

import math

import numpy as np
import pytest

from oracle import pwfs as O
from workloads import FLAG_DOUBLE_ROOF, FLAG_FULL_PLANE, FLAG_REF_SLOPES, tiny_sensor, tilt_opd


def _roof(**kw):
    base = dict(flags=FLAG_DOUBLE_ROOF | FLAG_REF_SLOPES)
    base.update(kw)
    return tiny_sensor(**base)


def _brute_arm(opd, s, axis):
    """One arm by direct sums over the padded grid: modulation and half-pixel
    tilts, DFT, the roof phase pi S |u_bar| / N along one axis only, inverse
    DFT; |e|^2 averaged over the points, over sum(A^2)."""
    N, D, S = s.n_fft, s.n_pupil, s.pupil_sep_px
    o = (N - D) // 2
    idx = np.arange(N)
    K = np.exp(-2j * np.pi * (idx[None, :, None, None] * idx[None, None, None, :]
                              + idx[:, None, None, None] * idx[None, None, :, None]) / N)
    ub = np.array([u + 0.5 if u < N // 2 else u - N + 0.5 for u in range(N)])
    ph = np.pi * S * np.abs(ub) / N
    M = np.exp(1j * (ph[None, :] if axis == 0 else ph[:, None])) * np.ones((N, N))
    E0 = np.zeros((N, N), complex)
    area = 0.0
    for Y in range(D):
        for X in range(D):
            r = math.hypot(X - (D - 1) / 2, Y - (D - 1) / 2)
            a = 1.0 if (s.obstruction * D / 2 <= r <= D / 2) else 0.0
            area += a
            E0[o + Y, o + X] = a * np.exp(2j * np.pi * opd[Y, X] / s.lambdas_nm[0])
    I = np.zeros((N, N))
    for k in range(s.n_mod):
        t = 2 * np.pi * k / s.n_mod
        E = E0.copy()
        for Y in range(N):
            for X in range(N):
                y, x = Y - o - (D - 1) / 2, X - o - (D - 1) / 2
                E[Y, X] *= np.exp(2j * np.pi * s.mod_radius_lod * (x * math.cos(t) + y * math.sin(t)) / D)
                E[Y, X] *= np.exp(-1j * np.pi * (X + Y) / N)
        G = np.einsum("vuYX,YX->vu", K, E) * M
        e = np.einsum("vuYX,vu->YX", np.conj(K), G) / (N * N)
        I += np.abs(e) ** 2
    return I / (s.n_mod * area)


@pytest.mark.parametrize("kw", [dict(), dict(obstruction=0.3, mod_radius_lod=2.0, n_mod=8)])
def test_arms_match_direct_sum(kw):
    s = _roof(**kw)
    opd = np.random.default_rng(11).standard_normal((s.n_pupil, s.n_pupil)) * 120.0
    I = O.forward_frame(opd, s)
    assert I.shape == (2, s.n_fft, s.n_fft)
    for axis in (0, 1):
        want = 0.5 * _brute_arm(opd, s, axis)
        assert np.abs(I[axis] - want).max() <= 1e-12 * np.abs(want).max()


def test_each_arm_carries_half_the_light():
    s = _roof(n_pupil=32, n_fft=128, n_subap=8, pupil_sep_px=48.0, n_mod=12, obstruction=0.2,
              flags=FLAG_DOUBLE_ROOF | FLAG_FULL_PLANE)
    opd = np.random.default_rng(12).standard_normal((32, 32)) * 300.0
    I = O.forward_frame(opd, s)
    np.testing.assert_allclose(I.sum(axis=(1, 2)), [0.5, 0.5], atol=1e-14)


def test_zero_separation_images_the_pupil():
    s = _roof(n_pupil=16, n_fft=32, n_subap=4, pupil_sep_px=0.0, n_mod=8, mod_radius_lod=2.0)
    opd = np.random.default_rng(13).standard_normal((16, 16)) * 200.0
    I = O.forward_frame(opd, s)
    A = O.pupil_amplitude(16, 0.0)
    want = np.zeros((32, 32))
    want[8:24, 8:24] = 0.5 * A * A / (A * A).sum()
    for arm in (0, 1):
        np.testing.assert_allclose(I[arm], want, atol=1e-15)


def test_flat_wavefront_mirror_images_and_zero_slopes():
    s = _roof(n_pupil=32, n_fft=96, n_subap=8, pupil_sep_px=40.0, n_mod=16, mod_radius_lod=3.0, obstruction=0.2)
    I = O.forward(np.zeros((1, 32, 32)), s)
    Q = O.bin_images(I, s)[0]
    np.testing.assert_allclose(Q[0], Q[1][:, ::-1], atol=1e-15)       # arm x: left = mirrored right
    np.testing.assert_allclose(Q[2], Q[3][::-1, :], atol=1e-15)       # arm y: top = mirrored bottom
    raw, _ = O.raw_slopes_roof(Q[None], O.valid_subapertures(s))
    np.testing.assert_allclose(raw[0, 0], -raw[0, 0][:, ::-1], atol=1e-14)
    assert abs(raw[0, 0].mean()) < 1e-14 and abs(raw[0, 1].mean()) < 1e-14
    sl, _ = O.slopes(I, s)
    assert np.abs(sl).max() < 1e-13


@pytest.mark.parametrize("theta,axis", [(0.0, 0), (math.pi / 2, 1)])
def test_tilt_response_signed_linear_and_on_its_own_axis(theta, axis):
    s = _roof(n_pupil=32, n_fft=128, n_subap=8, pupil_sep_px=48.0, n_mod=16, mod_radius_lod=3.0)
    valid = O.valid_subapertures(s)
    gains = []
    for t in (0.01, 0.03):
        sl, _ = O.slopes(O.forward(tilt_opd(32, t, theta)[None], s), s)
        gains.append(sl[0, axis][valid].mean() / t)
        assert abs(sl[0, 1 - axis][valid].mean()) < 1e-12
    assert min(gains) > 0 and abs(gains[0] / gains[1] - 1.0) < 5e-3


def test_geometric_gain_equals_the_pyramids():
    kw = dict(n_pupil=32, n_fft=128, n_subap=4, n_mod=64, pupil_sep_px=48.0, mod_radius_lod=10.0)
    t = 0.1
    opd = tilt_opd(32, t)[None]
    roof = _roof(**kw)
    pyr = tiny_sensor(flags=FLAG_REF_SLOPES, **kw)
    valid = O.valid_subapertures(pyr)
    g_roof = O.slopes(O.forward(opd, roof), roof)[0][0, 0][valid].mean() / t
    g_pyr = O.slopes(O.forward(opd, pyr), pyr)[0][0, 0][valid].mean() / t
    geo = 2.0 / (math.pi * 10.0)
    assert abs(g_roof / geo - 1.0) < 0.05
    assert abs(g_roof / g_pyr - 1.0) < 0.03
