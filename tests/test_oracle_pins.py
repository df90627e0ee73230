"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test names the property it relies on: direct-sum DFTs on tiny grids,
Parseval's identity, the shift theorem, mirror symmetry of the flat-wavefront
sensor, the linear small-tilt response, and bookkeeping identities of the
binning.  A plausible mistake in the oracle (a dropped half-pixel term, a
wrong face sign, a transposed ramp, a lost 1/N^2) fails at least one of them.
"""

import math

import numpy as np
import pytest

from oracle import pwfs as O
from workloads import tiny_sensor, tilt_opd, workload


def _rand_opd(D, seed, rms_nm=120.0):
    return np.random.default_rng(seed).standard_normal((D, D)) * rms_nm


# -------------------------------------------------- direct-sum brute force --

def _brute_forward(opd, s):
    """Whole forward chain by direct 2-D sums on the padded grid (no FFT, no
    separability): pupil from pixel-centre radii, modulation tilt, half-pixel
    tilt, DFT, 4-face pyramid phase pi S (|u_bar| + |v_bar|) / N, inverse DFT."""
    N, D, S = s.n_fft, s.n_pupil, s.pupil_sep_px
    o = (N - D) // 2
    idx = np.arange(N)
    # 4-index kernels K[v, u, Y, X] = exp(-2 pi i (u X + v Y) / N)
    ph = (idx[None, :, None, None] * idx[None, None, None, :]
          + idx[:, None, None, None] * idx[None, None, :, None])
    K = np.exp(-2j * np.pi * ph / N)
    ubar = np.array([u + 0.5 if u < N // 2 else u - N + 0.5 for u in range(N)])
    M = np.exp(1j * np.pi * S * (np.abs(ubar)[None, :] + np.abs(ubar)[:, None]) / N)
    I = np.zeros((N, N))
    area = 0.0
    Epad0 = np.zeros((N, N), complex)
    for Y in range(D):
        for X in range(D):
            y, x = Y - (D - 1) / 2, X - (D - 1) / 2
            r = math.hypot(x, y)
            a = 1.0 if (s.obstruction * D / 2 <= r <= D / 2) else 0.0
            area += a * a
            Epad0[o + Y, o + X] = a * np.exp(2j * np.pi * opd[Y, X] / s.lambdas_nm[0])
    for k in range(s.n_mod):
        t = 2 * np.pi * k / s.n_mod
        E = Epad0.copy()
        for Y in range(N):
            for X in range(N):
                y, x = Y - o - (D - 1) / 2, X - o - (D - 1) / 2
                E[Y, X] *= np.exp(2j * np.pi * s.mod_radius_lod * (x * math.cos(t) + y * math.sin(t)) / D)
                E[Y, X] *= np.exp(-1j * np.pi * (X + Y) / N)
        F = np.einsum("vuYX,YX->vu", K, E)
        G = F * M
        e = np.einsum("vuYX,vu->YX", np.conj(K), G) / (N * N)
        I += np.abs(e) ** 2
    return I / (s.n_mod * area)


@pytest.mark.parametrize("kw", [dict(), dict(obstruction=0.3, mod_radius_lod=2.0, n_mod=8),
                                dict(n_fft=20, pupil_sep_px=10.0, n_pupil=8)])
def test_forward_matches_direct_sum(kw):
    s = tiny_sensor(**kw)
    opd = _rand_opd(s.n_pupil, 3)
    a = O.forward_frame(opd, s)
    b = _brute_forward(opd, s)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


# ------------------------------------------------------- Parseval / flux --

@pytest.mark.parametrize("name", ["cfg1", "tiny", "poly"])
def test_parseval_flux_is_one(name):
    """The pyramid mask is phase only, so each frame's intensity sums to 1."""
    if name == "cfg1":
        s = workload("cfg1").sensors[0]
    elif name == "tiny":
        s = tiny_sensor(obstruction=0.25)
    else:
        s = tiny_sensor(lambdas_nm=(600.0, 900.0), lambda_weights=(0.25, 0.75))
    I = O.forward(_rand_opd(s.n_pupil, 5, 400.0)[None], s)
    assert abs(I.sum() - 1.0) < 1e-12


# ----------------------------------------------- mask identity / one face --

def test_unit_mask_returns_pupil():
    """S = 0 makes the mask 1: the chain is an FFT round trip, so |e|^2 is the
    padded |A|^2 whatever the phase and the modulation (Parseval per point)."""
    s = tiny_sensor(pupil_sep_px=0.0, obstruction=0.3)
    D, N = s.n_pupil, s.n_fft
    I = O.forward_frame(_rand_opd(D, 7, 500.0), s)
    A = O.pupil_amplitude(D, s.obstruction)
    ref = np.zeros((N, N))
    o = (N - D) // 2
    ref[o:o + D, o:o + D] = A / A.sum()
    assert np.abs(I - ref).max() < 1e-14


@pytest.mark.parametrize("S", [4, 8, 10])
def test_one_face_mask_is_a_shift(S):
    """A single face exp(i pi S u_bar / N) (no |.|) over the whole focal plane
    is a linear phase: by the shift theorem the pupil image moves by -S/2 in
    both axes.  Pins the half-integer focal coordinates and the image origin
    of the face that sees positive focal coordinates."""
    s = tiny_sensor(n_fft=24, pupil_sep_px=float(S))
    N, D = s.n_fft, s.n_pupil
    ub = O.focal_coords(N)
    m = np.exp(1j * np.pi * S * ub / N)
    I = O.forward(_rand_opd(D, 11, 300.0)[None], s, mask=m)[0]
    A = O.pupil_amplitude(D, 0.0)
    ref = np.zeros((N, N))
    o = (N - D) // 2 - S // 2
    ref[o:o + D, o:o + D] = A / A.sum()
    assert np.abs(I - ref).max() < 1e-14
    (r0, c0) = O.image_origins(s)[0]
    assert (r0, c0) == (o, o)


# ------------------------------------------------ modulation ramp pinning --

@pytest.mark.parametrize("theta,axis", [(0.0, 1), (math.pi / 2, 0), (math.pi, 1)])
def test_modulation_ramp_moves_focal_spot(theta, axis):
    """A tilt of r lambda/D shifts the focal field by r N / D bins along
    (cos t, sin t) (shift theorem; here r N / D = 4 bins)."""
    D, N, r = 16, 32, 2.0
    A = O.pupil_amplitude(D, 0.0)
    F0 = np.abs(O.focal_field(A, N)) ** 2
    F1 = np.abs(O.focal_field(A * O.modulation_ramp(D, r, theta), N)) ** 2
    shift = int(round(r * N / D * (math.cos(theta) if axis == 1 else math.sin(theta))))
    assert np.abs(F1 - np.roll(F0, shift, axis=axis)).max() < 1e-9 * F0.max()


# -------------------------------------------------- flat-wavefront symmetry --

@pytest.mark.parametrize("name", ["cfg1", "tiny_obs"])
def test_flat_wavefront_mirror_symmetry(name):
    """A flat wavefront, a centred pupil, a mask with its apex between the
    four central pixels and a modulation circle closed under x -> -x and
    y -> -y make the intensity mirror-symmetric about both array midlines."""
    s = workload("cfg1").sensors[0] if name == "cfg1" else tiny_sensor(obstruction=0.3, n_mod=8)
    I = O.forward(np.zeros((1, s.n_pupil, s.n_pupil)), s)[0]
    assert np.abs(I - I[:, ::-1]).max() < 1e-14
    assert np.abs(I - I[::-1, :]).max() < 1e-14
    valid = O.valid_subapertures(s)
    raw, _ = O.raw_slopes(O.bin_images(I, s), valid)
    sx, sy = raw[0]
    assert np.abs(sx + sx[:, ::-1]).max() < 1e-13
    assert np.abs(sy + sy[::-1, :]).max() < 1e-13
    assert abs(sx[valid].mean()) < 1e-14 and abs(sy[valid].mean()) < 1e-14
    # not trivially zero before the reference is subtracted
    assert np.sqrt((sx[valid] ** 2).mean()) > 1e-3
    sl, _ = O.slopes(I[None], s)
    assert np.abs(sl).max() < 1e-13


# ------------------------------------------------------- tip/tilt response --

def test_tip_response_linear_signed_and_uncoupled():
    """Small tilts give a slope proportional to the tilt (linear regime of the
    modulated sensor), positive for a phase increasing along +x, and no mean
    slope on the other axis (mirror symmetry in y)."""
    s = workload("cfg1").sensors[0]
    valid = O.valid_subapertures(s)
    gains = []
    for t in (0.005, 0.02, 0.05):
        sl, _ = O.slopes(O.forward(tilt_opd(s.n_pupil, t)[None], s), s)
        gains.append(sl[0, 0][valid].mean() / t)
        assert abs(sl[0, 1][valid].mean()) < 1e-12
    gains = np.array(gains)
    assert gains.min() > 0.0
    assert np.ptp(gains) / gains.mean() < 2e-3
    # the same tilt along y gives the transposed response
    sl, _ = O.slopes(O.forward(tilt_opd(s.n_pupil, 0.02, math.pi / 2)[None], s), s)
    assert abs(sl[0, 1][valid].mean() / 0.02 - gains[1]) < 1e-9
    assert abs(sl[0, 0][valid].mean()) < 1e-12


def test_large_modulation_geometric_limit():
    """With a modulation radius much larger than the tilt, a modulated pyramid
    sees the fraction of the circle on each side: mean s_x -> (2/pi) asin(t/r),
    i.e. gain 2/(pi r) per lambda/D (geometric-optics limit; 1.5 % off at r = 10)."""
    s = tiny_sensor(n_pupil=32, n_fft=128, n_subap=4, n_mod=64, pupil_sep_px=48.0,
                    mod_radius_lod=10.0)
    valid = O.valid_subapertures(s)
    t = 0.1
    sl, _ = O.slopes(O.forward(tilt_opd(s.n_pupil, t)[None], s), s)
    g = sl[0, 0][valid].mean() / t
    geo = 2.0 / (math.pi * s.mod_radius_lod)
    assert abs(g - geo) / geo < 0.05


# ------------------------------------------------- separable operator form --

@pytest.mark.parametrize("name", ["cfg1", "tiny_obs", "tiny_poly"])
def test_separable_form_equals_fft_route(name):
    if name == "cfg1":
        s = workload("cfg1").sensors[0]
    elif name == "tiny_obs":
        s = tiny_sensor(obstruction=0.3, n_fft=24, pupil_sep_px=12.0)
    else:
        s = tiny_sensor(lambdas_nm=(600.0, 900.0), lambda_weights=(0.5, 0.5))
    opd = _rand_opd(s.n_pupil, 13, 250.0)
    a = O.forward_frame(opd, s)
    b = O.forward_frame_separable(opd, s)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


# ------------------------------------------------------- binning / slopes --

def test_binning_conserves_window_flux_and_slopes_scale_free():
    s = workload("cfg1").sensors[0]
    I = O.forward(_rand_opd(s.n_pupil, 17, 300.0)[None], s)
    Q = O.bin_images(I, s)
    tot = sum(I[0, r:r + s.n_pupil, c:c + s.n_pupil].sum() for r, c in O.image_origins(s))
    assert abs(Q.sum() - tot) < 1e-13
    # S = D = N/2: the four images tile the plane, so they hold all the flux
    assert abs(Q.sum() - 1.0) < 1e-12
    s1, f1 = O.slopes(I, s)
    s2, f2 = O.slopes(7.5 * I, s)
    assert np.abs(s1 - s2).max() < 1e-13
    assert abs(f2[0] / f1[0] - 7.5) < 1e-13


def test_local_norm_bounds():
    """Per-subaperture normalisation bounds each raw slope by 1 in modulus
    (a difference of non-negative parts over their sum)."""
    s = tiny_sensor(n_pupil=16, n_fft=32, n_subap=4, pupil_sep_px=16.0, flags=4)
    I = O.forward(_rand_opd(16, 19, 600.0)[None], s)
    raw, _ = O.raw_slopes(O.bin_images(I, s), O.valid_subapertures(s), local_norm=True)
    assert np.abs(raw).max() <= 1.0 + 1e-12


def test_valid_map_symmetry_and_counts():
    for s in (workload("cfg1").sensors[0], workload("cfg2").sensors[0]):
        v = O.valid_subapertures(s)
        assert (v == v[::-1]).all() and (v == v[:, ::-1]).all() and (v == v.T).all()
        n = s.n_subap
        assert v[n // 2, n // 2 - 1] or s.obstruction > 0
        assert not v[0, 0]


def test_polychromatic_is_weighted_sum():
    base = tiny_sensor(obstruction=0.2)
    opd = _rand_opd(base.n_pupil, 23, 200.0)
    s1 = base.with_(lambdas_nm=(600.0,), lambda_weights=(1.0,))
    s2 = base.with_(lambdas_nm=(900.0,), lambda_weights=(1.0,))
    sp = base.with_(lambdas_nm=(600.0, 900.0), lambda_weights=(0.3, 0.7))
    I = O.forward_frame(opd, sp)
    ref = 0.3 * O.forward_frame(opd, s1) + 0.7 * O.forward_frame(opd, s2)
    assert np.abs(I - ref).max() < 1e-15
    # the modulation circle is a fixed sky angle: at 600 nm it is 750/600 wider
    s3 = base.with_(lambdas_nm=(600.0,), lambda_weights=(1.0,), lambda_ref_nm=750.0)
    s4 = base.with_(lambdas_nm=(600.0,), lambda_weights=(1.0,), lambda_ref_nm=600.0,
                    mod_radius_lod=base.mod_radius_lod * 750.0 / 600.0)
    assert np.abs(O.forward_frame(opd, s3) - O.forward_frame(opd, s4)).max() < 1e-15


def test_error_metrics():
    a = np.ones((2, 4, 4))
    b = a * (1 + 1e-3)
    e = O.intensity_rel_error(b, a)
    assert np.allclose(e, 1e-3)
    v = np.ones((4, 4), bool)
    assert abs(O.slope_rel_rms(b[:, None].repeat(2, 1), a[:, None].repeat(2, 1), v) - 1e-3) < 1e-12
