"""Pins of the extended-source form of the sensor oracle: the source sampling
(count, symmetry, second moment of the rings), equality with the average of
point-source images each seen through an OPD tilt (the already-pinned point
source path with the tilt put in the wavefront instead of the modulation),
a zero radius reducing to the point source, and the physics of an extended
source (less tip response than a point source, as with more modulation)."""

import numpy as np
import pytest

from oracle import pwfs as O
from workloads import tiny_sensor, tilt_opd


def _sensor(**kw):
    base = dict(n_pupil=16, n_fft=64, n_subap=4, n_mod=8, pupil_sep_px=32.0, mod_radius_lod=1.5,
                obstruction=0.0)
    base.update(kw)
    return tiny_sensor(**base)


@pytest.mark.parametrize("R", [0, 1, 2, 3])
def test_source_sampling(R):
    s = _sensor(src_rings=R, src_radius_lod=2.0)
    p = O.source_points(s)
    assert len(p) == 1 + 3 * R * (R + 1)
    assert np.abs(p.mean(axis=0)).max() < 1e-14
    if R:
        want = (2.0 / R) ** 2 * 3 * (R * (R + 1) / 2) ** 2 / (1 + 3 * R * (R + 1))
        assert abs((p[:, 0] ** 2).mean() - want) < 1e-12
        assert abs((p[:, 0] ** 2).mean() - (p[:, 1] ** 2).mean()) < 1e-12


@pytest.mark.parametrize("lams", [(750.0,), (600.0, 900.0)])
def test_extended_source_is_mean_of_tilted_point_sources(lams):
    w = tuple([1.0 / len(lams)] * len(lams))
    s = _sensor(src_rings=2, src_radius_lod=1.2, lambdas_nm=lams, lambda_weights=w)
    pt = _sensor(lambdas_nm=lams, lambda_weights=w)
    rng = np.random.default_rng(8)
    opd = rng.normal(0.0, 40.0, (16, 16))
    got = O.forward(opd, s)[0]
    want = np.zeros_like(got)
    for dx, dy in O.source_points(s):
        t = np.hypot(dx, dy)
        th = np.arctan2(dy, dx)
        ramp = tilt_opd(16, t, th, s.lambda_ref_nm) if t > 0 else 0.0
        want += O.forward(opd + ramp, pt)[0]
    want /= len(O.source_points(s))
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max() + 1e-16


def test_zero_radius_is_the_point_source_and_flux_is_conserved():
    s0 = _sensor()
    s1 = _sensor(src_rings=2, src_radius_lod=0.0)
    opd = np.random.default_rng(9).normal(0.0, 30.0, (16, 16))
    I0 = O.forward(opd, s0)[0]
    I1 = O.forward(opd, s1)[0]
    assert np.abs(I0 - I1).max() < 1e-14
    assert abs(O.forward(opd, _sensor(src_rings=2, src_radius_lod=2.5))[0].sum() - 1.0) < 1e-12


def test_extended_source_lowers_the_tip_response():
    gains = []
    for rho in (0.0, 1.0, 2.0):
        s = _sensor(n_pupil=32, n_subap=8, n_fft=128, pupil_sep_px=64.0, src_rings=2, src_radius_lod=rho)
        ref = O.reference_slopes(s)
        valid = O.valid_subapertures(s)
        t = 0.05
        sl, _ = O.slopes(O.forward(tilt_opd(32, t, 0.0, 750.0), s), s, ref)
        gains.append(sl[0, 0][valid].mean() / t)
    assert gains[0] > gains[1] > gains[2] > 0
