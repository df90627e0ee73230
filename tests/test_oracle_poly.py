"""Pins of the oracle's wavelength handling for finely sampled polychromatic
sensors (Table 4: PolyCromPyramid), beyond the weighted-sum and the
fixed-sky-angle modulation pins of the core tests:

* similarity: the sensor sees OPD / lambda and the modulation radius in
  lambda/D at the sensing wavelength only, so a sensor at 1500 nm fed twice
  the OPD with the same radius in its own lambda/D gives exactly the 750 nm
  result (pins the phase scale 2 pi OPD / lambda);
* geometric optics: with a modulation radius large against the tilt, the
  sensor responds to the tilt angle over the modulation angle, both fixed on
  the sky, so the tilt gain is the same at every wavelength (a radius not
  rescaled by lambda_ref / lambda would change it by that ratio);
* the midpoint sampling of a smooth band converges quadratically: doubling
  the number of samples divides the error by about four."""

import math

import numpy as np

from oracle import pwfs as O
from workloads import band_sampling, tiny_sensor, tilt_opd, von_karman_opd


def test_band_sampling_midpoints():
    lams, ws = band_sampling(750.0, 300.0, 6)
    assert np.allclose(lams, [625.0, 675.0, 725.0, 775.0, 825.0, 875.0])
    assert abs(sum(ws) - 1.0) < 1e-15 and len(set(ws)) == 1


def test_intensity_depends_on_opd_over_lambda_only():
    base = tiny_sensor(n_pupil=16, n_fft=64, n_subap=4, n_mod=8, pupil_sep_px=24.0, mod_radius_lod=2.0,
                       obstruction=0.2)
    # OPD as float32 values (the sensor's input type); the factor 2 keeps them exact
    opd = von_karman_opd(2, 16, 8.0, 0.5, 25.0, seed=9).astype(np.float32).astype(np.float64)
    s750 = base.with_(lambdas_nm=(750.0,), lambda_weights=(1.0,), lambda_ref_nm=750.0)
    s1500 = base.with_(lambdas_nm=(1500.0,), lambda_weights=(1.0,), lambda_ref_nm=1500.0)
    a = O.forward(opd, s750)
    b = O.forward(opd * 2.0, s1500)
    assert np.abs(a - b).max() < 1e-15
    # and the same OPD at 1500 nm is a different (weaker) phase
    assert np.abs(O.forward(opd, s1500) - a).max() > 1e-4


def test_geometric_tilt_gain_is_wavelength_independent():
    # 32 px pupil, 4 px per lambda/D, radius 6 lambda/D at 750 nm sampled by
    # 64 points (under one lambda/D apart at every wavelength used)
    s0 = tiny_sensor(n_pupil=32, n_fft=128, n_subap=4, n_mod=64, pupil_sep_px=48.0, mod_radius_lod=6.0)
    valid = O.valid_subapertures(s0)
    t = 0.1                                  # lambda/D at 750 nm: a fixed sky angle
    opd = tilt_opd(32, t)[None]
    gain = {}
    for lam in (600.0, 750.0, 900.0):
        s = s0.with_(lambdas_nm=(lam,), lambda_weights=(1.0,))
        sl, _ = O.slopes(O.forward(opd, s), s)
        gain[lam] = sl[0, 0][valid].mean() / t
    assert abs(gain[750.0] / (2.0 / (math.pi * 6.0)) - 1.0) < 0.05
    for lam in (600.0, 900.0):
        assert abs(gain[lam] / gain[750.0] - 1.0) < 0.03
    # a radius held at 6 lambda/D of the sensing wavelength would move the
    # gain by about lambda / 750: the check above tells the two apart
    s = s0.with_(lambdas_nm=(600.0,), lambda_weights=(1.0,), lambda_ref_nm=600.0)
    sl, _ = O.slopes(O.forward(opd, s), s)
    assert abs(sl[0, 0][valid].mean() / t / gain[750.0] - 1.0) > 0.15


def test_band_sampling_converges_quadratically():
    s = tiny_sensor(n_pupil=16, n_fft=64, n_subap=4, n_mod=8, pupil_sep_px=24.0, mod_radius_lod=2.0)
    opd = von_karman_opd(1, 16, 8.0, 0.5, 25.0, seed=3)
    lams, ws = band_sampling(750.0, 300.0, 64)
    ref = O.forward(opd, s.with_(lambdas_nm=lams, lambda_weights=ws))
    err = []
    for n in (2, 4, 8):
        lams, ws = band_sampling(750.0, 300.0, n)
        err.append(np.linalg.norm(O.forward(opd, s.with_(lambdas_nm=lams, lambda_weights=ws)) - ref))
    for a, b in zip(err, err[1:]):
        assert 3.5 < a / b < 5.0
