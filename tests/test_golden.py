"""The 160 px workload takes its pupil-separation ratio, modulation radius and
wavelength from the paper's SOUL pyramid block (Appendix B listing)."""

import os

from workloads import workload

HERE = os.path.dirname(os.path.abspath(__file__))


def _soul():
    out = {}
    with open(os.path.join(HERE, "golden", "soul_pyramid.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v)
    return out


def test_160px_sensor_follows_soul_ratios():
    g = _soul()
    s = workload("cfg2").sensors[0]
    assert s.pupil_sep_px / s.n_pupil == g["pup_dist_subaps"] / g["pup_diam_subaps"]
    assert s.mod_radius_lod == g["mod_amp_lambda_over_d"]
    assert s.lambdas_nm == (g["wavelength_nm"],)
    assert s.n_subap == g["pup_diam_subaps"]
