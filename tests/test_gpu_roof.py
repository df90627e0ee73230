"""Double-roof sensor on the GPU (PWFS_F_DOUBLE_ROOF) against the oracle
(oracle/pwfs.py): both arms' planes and the per-arm slopes element by element
on small sensors (full plane and image windows, global and local
normalisation, the radix-3 plan, two wavelengths, an extended source, a
field stop, subapertures that cut pixels), the 160 px / N=512 / 48-point sensor on
sampled frames of a full 1000-frame launch, and the modes it does not take."""

import numpy as np
import pytest

import parity
from oracle import pwfs as O
from workloads import FLAG_DOUBLE_ROOF, FLAG_FULL_PLANE, FLAG_LOCAL_NORM, FLAG_REF_SLOPES, tiny_sensor, workload
from workloads import von_karman_opd, workload_opd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

INT_TOL = 1e-5
SLOPE_TOL = 1e-4


def _P():
    from paper_2602_06688_amd import pwfs as P
    return P


def _windows(I, s):
    D = s.n_pupil
    return np.stack([I[:, pl, r:r + D, c:c + D] for pl, r, c in O.image_origins(s)], axis=1)


def _check(s, opd, label, frames=None):
    P = _P()
    F = opd.shape[0]
    print(f"[gpu] roof {label}: D={s.n_pupil} N={s.n_fft} n_mod={s.n_mod} flags={s.flags} F={F}", flush=True)
    plan = P.Plan([s], max_frames=F)
    x = torch.from_numpy(np.ascontiguousarray(opd, dtype=np.float32)).cuda()
    I, sl, flux = plan.step(x)
    torch.cuda.synchronize()
    idx = list(range(F)) if frames is None else frames
    I = I.cpu().numpy().astype(np.float64)[idx]
    sl = sl.cpu().numpy().astype(np.float64)[idx]
    flux = flux.cpu().numpy()[idx, 0].astype(np.float64)
    assert I.shape[1:] == (2, s.n_fft, s.n_fft)
    I_ref = O.forward(opd[idx].astype(np.float32).astype(np.float64), s)
    s_ref, f_ref = O.slopes(I_ref, s)
    valid = O.valid_subapertures(s)
    if s.flags & FLAG_FULL_PLANE:
        err = parity.errors(I, I_ref, sl, s_ref, valid)
        np.testing.assert_allclose(I.sum(axis=(2, 3)), I_ref.sum(axis=(2, 3)), rtol=2e-6)
    else:
        err = parity.errors(_windows(I, s), _windows(I_ref, s), sl, s_ref, valid)
    fe = np.abs(flux / f_ref - 1).max()
    print(f"      {parity.fmt(err)}; flux {fe:.2e}", flush=True)
    parity.check(err, parity.FP32)
    assert fe <= 1e-5
    assert (sl[:, :, ~valid] == 0).all()
    return plan


CASES = {
    "N128_full": tiny_sensor(n_pupil=48, n_fft=128, n_subap=12, pupil_sep_px=56.0, n_mod=8, mod_radius_lod=2.0,
                             obstruction=0.2, flags=FLAG_DOUBLE_ROOF | FLAG_REF_SLOPES | FLAG_FULL_PLANE),
    "N128_windows": tiny_sensor(n_pupil=48, n_fft=128, n_subap=12, pupil_sep_px=56.0, n_mod=8,
                                mod_radius_lod=2.0, flags=FLAG_DOUBLE_ROOF | FLAG_REF_SLOPES),
    "local_norm_no_ref": tiny_sensor(n_pupil=64, n_fft=128, n_subap=16, pupil_sep_px=64.0, n_mod=12,
                                     mod_radius_lod=3.0, flags=FLAG_DOUBLE_ROOF | FLAG_LOCAL_NORM),
    "N64_unmodulated": tiny_sensor(n_pupil=32, n_fft=64, n_subap=4, pupil_sep_px=32.0, n_mod=1, mod_radius_lod=0.0,
                                   flags=FLAG_DOUBLE_ROOF | FLAG_REF_SLOPES),
    "N384_radix3": tiny_sensor(n_pupil=120, n_fft=384, n_subap=30, pupil_sep_px=144.0, n_mod=8, obstruction=0.28,
                               mod_radius_lod=3.0, flags=FLAG_DOUBLE_ROOF | FLAG_REF_SLOPES),
    "poly2_N256": tiny_sensor(n_pupil=80, n_fft=256, n_subap=20, pupil_sep_px=96.0, n_mod=6, mod_radius_lod=2.0,
                              lambdas_nm=(650.0, 850.0), lambda_weights=(0.4, 0.6),
                              flags=FLAG_DOUBLE_ROOF | FLAG_REF_SLOPES | FLAG_FULL_PLANE),
    "extended": tiny_sensor(n_pupil=64, n_fft=128, n_subap=16, pupil_sep_px=64.0, n_mod=8, mod_radius_lod=2.0,
                            src_rings=1, src_radius_lod=1.5, flags=FLAG_DOUBLE_ROOF | FLAG_REF_SLOPES),
    "field_stop": tiny_sensor(n_pupil=48, n_fft=128, n_subap=12, pupil_sep_px=56.0, n_mod=8, mod_radius_lod=2.0,
                              fov_lod=9.0, flags=FLAG_DOUBLE_ROOF | FLAG_REF_SLOPES | FLAG_FULL_PLANE),
    "subap_5p5": tiny_sensor(n_pupil=44, n_fft=128, n_subap=8, pupil_sep_px=66.0, n_mod=8, mod_radius_lod=2.0,
                             flags=FLAG_DOUBLE_ROOF | FLAG_REF_SLOPES),
}


@pytest.mark.parametrize("name", list(CASES))
def test_small_double_roofs_match_oracle(name):
    s = CASES[name]
    rng = np.random.default_rng(sum(name.encode()))
    opd = von_karman_opd(3, s.n_pupil, 8.0, 0.5, 25.0, seed=int(rng.integers(1000)))
    _check(s, opd, name)


def test_flat_wavefront_zero_slopes():
    P = _P()
    s = CASES["N128_windows"]
    plan = P.Plan([s], max_frames=2)
    _, sl, _ = plan.step(torch.zeros((2, s.n_pupil, s.n_pupil), device="cuda"))
    assert float(sl.abs().max()) < 1e-5


def test_full_size_launch_sampled_frames():
    """160 px pupil, N = 512, 48 points, 40 x 40: the plain path's workload as
    a double roof, all 1000 frames in one call, three of them checked."""
    w = workload("cfg2")
    s = w.sensors[0].with_(flags=FLAG_DOUBLE_ROOF | FLAG_REF_SLOPES)
    _check(s, workload_opd(w), "160 px, 1000 frames", frames=[0, 517, 999])


def test_modes_it_does_not_take():
    P = _P()
    s = CASES["N384_radix3"]
    plan = P.Plan([s], max_frames=2)
    with pytest.raises(P.PwfsError) as e:
        plan.set_tuning(mode=P.MODE_PERSISTENT)
    assert e.value.code == P.PWFS_EUNSUPPORTED
    I = plan.forward(torch.zeros((2, s.n_pupil, s.n_pupil), device="cuda"))
    with pytest.raises(P.PwfsError) as e:
        plan.ccd(I, P.ccd_desc(96, 4, 1e4, P.CCD_PHOTON))
    assert e.value.code == P.PWFS_EUNSUPPORTED
