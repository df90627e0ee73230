"""Detector stage on the GPU (pwfs_ccd, pwfs_ccd_slopes) against the oracle
(oracle/ccd.py) on the same float32 intensity planes, which the oracle's
sensor model produces: every detector value bit for bit -- Poisson counts,
Gaussian readout and Gamma excess draws alike, since both sides evaluate
the samplers' exp, ln, sqrt and cos with the same basic operations in the
same order, so no accept/reject decision depends on a math library --,
slopes on detector pixels; batching invariance in the benchmark's launch
configuration; the noise-free detector reproduces the intensity slopes;
argument errors."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import ccd as C
from oracle import pwfs as O
from workloads import FLAG_FULL_PLANE, FLAG_REF_SLOPES, tiny_sensor, workload, workload_opd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _P():
    from paper_2602_06688_amd import pwfs as P
    return P


def _small(full=True):
    return tiny_sensor(n_pupil=32, n_fft=64, n_subap=8, n_mod=8, pupil_sep_px=32.0, mod_radius_lod=2.0,
                       obstruction=0.2, flags=FLAG_REF_SLOPES | (FLAG_FULL_PLANE if full else 0))


def _window_mask(s):
    m = np.zeros((s.n_fft, s.n_fft), bool)
    D = s.n_pupil
    for r0, c0 in O.image_origins(s):
        m[r0:r0 + D, c0:c0 + D] = True
    return m


FLAGS = [("none", 0), ("photon", 1), ("readout", 2), ("photon+readout", 3), ("photon+excess+readout", 7)]


@pytest.mark.parametrize("electrons", [60.0, 7.0e4, 2.0e6])
@pytest.mark.parametrize("label,flags", FLAGS)
def test_detector_matches_oracle_small(label, flags, electrons):
    P = _P()
    s = _small()
    rng = np.random.default_rng(21)
    I = O.forward(rng.normal(0.0, 80.0, (3, 32, 32)), s).astype(np.float32)
    plan = P.Plan([s], max_frames=3)
    d = P.ccd_desc(16, 4, electrons, flags, readout_e=0.7, seed=1234)
    print(f"[gpu] ccd small {label} electrons={electrons:g}", flush=True)
    got = plan.ccd(torch.from_numpy(I).cuda(), d, frame0=5).cpu().numpy()
    want = C.detector(I, 16, 4, electrons, flags, 0.7, 1234, frame0=5).astype(np.float32)
    np.testing.assert_array_equal(got, want)


def test_window_mode_counts_only_the_pupil_images():
    P = _P()
    s = _small(full=False)
    rng = np.random.default_rng(22)
    I = O.forward(rng.normal(0.0, 80.0, (2, 32, 32)), s).astype(np.float32)   # full plane, light everywhere
    plan = P.Plan([s], max_frames=2)
    d = P.ccd_desc(16, 4, 5e4, P.CCD_PHOTON, seed=3)
    print("[gpu] ccd window mode", flush=True)
    got = plan.ccd(torch.from_numpy(I).cuda(), d).cpu().numpy()
    want = C.detector(I * _window_mask(s)[None], 16, 4, 5e4, C.PHOTON, 0.0, 3).astype(np.float32)
    np.testing.assert_array_equal(got, want)


def _cfg2():
    w = workload("cfg2")
    return w, w.sensors[0]


def test_full_size_sampled_frames_and_detector_slopes():
    """160 px / N=512 sensor, 120 px detector (rebin 4): six sampled frames
    of the 1000-frame workload through the oracle's sensor model, then the
    GPU's and the oracle's detector (photon, excess and readout noise: equal
    bit for bit) and detector slopes."""
    P = _P()
    w, s = _cfg2()
    idx = [0, 1, 250, 517, 998, 999]
    opd = workload_opd(w, frames=idx)
    I = O.forward(opd, s).astype(np.float32)
    Iw = I * _window_mask(s)[None]
    plan = P.Plan([s], max_frames=1000)
    d = P.ccd_desc(120, 4, 9.0e4, P.CCD_PHOTON | P.CCD_EXCESS | P.CCD_READOUT, readout_e=0.4, seed=77)
    for j, f in enumerate(idx):
        print(f"[gpu] ccd full size frame {f}", flush=True)
        got = plan.ccd(torch.from_numpy(I[j:j + 1]).cuda(), d, frame0=f)
        want = C.detector(Iw[j:j + 1], 120, 4, 9.0e4, 7, 0.4, 77, frame0=f)
        np.testing.assert_array_equal(got.cpu().numpy(), want.astype(np.float32))
        sl, fl = plan.ccd_slopes(got, d)
        ws, wf = C.detector_slopes(want, s, 120, 4)
        valid = O.valid_subapertures(s)
        assert O.slope_rel_rms(sl.cpu().numpy(), ws, valid) < 1e-5
        assert abs(fl.item() / wf[0] - 1.0) < 1e-6


def test_full_batch_launch_equals_single_frames_and_noise_free_slopes():
    """The benchmark's launch (1000 frames in one call after the GPU forward
    model) gives each frame exactly what a one-frame launch keyed by its
    index gives; with no noise the detector slopes equal the intensity
    slopes."""
    P = _P()
    w, s = _cfg2()
    x = torch.from_numpy(workload_opd(w)).cuda()
    plan = P.Plan([s], max_frames=w.n_frames)
    I = plan.forward(x)
    d = P.ccd_desc(120, 4, 9.0e4, P.CCD_PHOTON | P.CCD_EXCESS | P.CCD_READOUT, readout_e=0.4, seed=5)
    print("[gpu] ccd full batch", flush=True)
    full = plan.ccd(I, d)
    for f in (0, 517, 999):
        one = plan.ccd(I[f:f + 1].contiguous(), d, frame0=f)
        assert torch.equal(full[f:f + 1], one)
    assert torch.isfinite(full).all()
    d0 = P.ccd_desc(120, 4, 9.0e4, 0, seed=5)
    P0 = plan.ccd(I[:16].contiguous(), d0)
    s_det, f_det = plan.ccd_slopes(P0, d0)
    s_int, f_int = plan.slopes(I[:16].contiguous())
    valid = torch.from_numpy(plan.valid_map(0)).cuda()
    a = s_det.reshape(16, 2, -1)[:, :, valid.reshape(-1)]
    b = s_int.reshape(16, 2, -1)[:, :, valid.reshape(-1)]
    assert float((a - b).norm() / b.norm()) < 1e-5
    assert torch.allclose(f_det / 9.0e4, f_int[:, 0], rtol=1e-5)


def test_huge_or_nonfinite_expectation_gives_nan():
    P = _P()
    s = _small()
    I = np.zeros((1, 64, 64), np.float32)
    I[0, 10, 10] = 1.0
    I[0, 30, 30] = np.inf
    plan = P.Plan([s], max_frames=1)
    d = P.ccd_desc(16, 4, 2.0 ** 25, P.CCD_PHOTON, seed=1)
    print("[gpu] ccd bounds", flush=True)
    got = plan.ccd(torch.from_numpy(I).cuda(), d).cpu().numpy()[0]
    want = C.detector(I, 16, 4, 2.0 ** 25, C.PHOTON, 0.0, 1)[0]
    assert np.isnan(got[2, 2]) and np.isnan(got[7, 7]) and np.isnan(want[2, 2]) and np.isnan(want[7, 7])
    ok = ~np.isnan(want)
    np.testing.assert_array_equal(got[ok], want[ok].astype(np.float32))


def test_errors():
    P = _P()
    w, s = _cfg2()
    plan = P.Plan([s], max_frames=2)
    I = torch.zeros((2, 512, 512), device="cuda")
    with pytest.raises(P.PwfsError) as e:
        plan.ccd(I, P.ccd_desc(120, 4, 1e4, P.CCD_EXCESS))
    assert e.value.code == P.PWFS_EINVAL
    with pytest.raises(P.PwfsError) as e:
        plan.ccd(I, P.ccd_desc(119, 4, 1e4, P.CCD_PHOTON))          # images not on whole detector pixels
    assert e.value.code == P.PWFS_EINVAL
    with pytest.raises(P.PwfsError) as e:
        plan.ccd(I, P.ccd_desc(130, 4, 1e4, P.CCD_PHOTON))          # larger than the plane
    assert e.value.code == P.PWFS_EINVAL
    bad = P.ccd_desc(120, 4, 1e4, P.CCD_PHOTON)
    bad.rebin_den = 65
    with pytest.raises(P.PwfsError):
        plan.ccd(I, bad)
    with pytest.raises(P.PwfsError) as e:
        plan.ccd(I, P.ccd_desc(120, Fraction(3, 4), 1e4, P.CCD_PHOTON))   # pixels finer than the plane's
    assert e.value.code == P.PWFS_EINVAL
    with pytest.raises(P.PwfsError) as e:
        plan.ccd(I, P.ccd_desc(121, Fraction(7, 2), 1e4, P.CCD_PHOTON))   # 423.5 px: not whole pixels
    assert e.value.code == P.PWFS_EINVAL
    with pytest.raises(P.PwfsError) as e:
        plan.ccd(torch.zeros((3, 512, 512), device="cuda"), P.ccd_desc(120, 4, 1e4, P.CCD_PHOTON))
    assert e.value.code == P.PWFS_ESTATE


def _soul_like(full):
    # 44 px pupil, 8 subapertures of 5.5 px, images 66 px apart on a 128 grid;
    # a 20 px detector of 5.5 transform pixels: one detector pixel per subaperture
    return tiny_sensor(n_pupil=44, n_fft=128, n_subap=8, pupil_sep_px=66.0, n_mod=8, mod_radius_lod=2.0,
                       flags=FLAG_REF_SLOPES | (FLAG_FULL_PLANE if full else 0))


@pytest.mark.parametrize("full", [True, False])
@pytest.mark.parametrize("label,flags", FLAGS)
def test_fractional_pitch_matches_oracle(label, flags, full):
    P = _P()
    s = _soul_like(full)
    r = Fraction(11, 2)
    rng = np.random.default_rng(23)
    I = O.forward(rng.normal(0.0, 80.0, (3, 44, 44)), s).astype(np.float32)
    Iw = I if full else I * _window_mask(s)[None]
    plan = P.Plan([s], max_frames=3)
    d = P.ccd_desc(20, r, 3.0e4, flags, readout_e=0.7, seed=99)
    print(f"[gpu] ccd pitch 11/2 {label} full={full}", flush=True)
    got = plan.ccd(torch.from_numpy(I).cuda(), d, frame0=2)
    want = C.detector(Iw, 20, r, 3.0e4, flags, 0.7, 99, frame0=2)
    np.testing.assert_array_equal(got.cpu().numpy(), want.astype(np.float32))
    sl, fl = plan.ccd_slopes(got, d)
    ws, wf = C.detector_slopes(want, s, 20, r)
    valid = O.valid_subapertures(s)
    np.testing.assert_allclose(sl.cpu().numpy(), ws, atol=2e-5 if flags else 1e-5)
    np.testing.assert_allclose(fl.cpu().numpy(), wf, rtol=1e-5)
    assert (sl.cpu().numpy()[:, :, ~valid] == 0).all()


# the listing's 2.0 arcsec field of view as lambda/D at 750 nm on the 8.222 m pupil
SOUL_FOV_LOD = 2.0 / (750e-9 / 8.222 * 206264.806)


def test_soul_geometry_chain():
    """The SOUL pyramid of Appendix B: 220 px pupil, 40 subapertures of 5.5 px,
    pupils 48 subapertures apart, 3 lambda/D modulation at 750 nm with 24
    points (Table 2: 24 transforms per step) behind a 2.0 arcsec square
    field stop, read out on a 120 x 120 detector of 5.5 transform pixels (on
    a 768 grid here).  Two frames:
    intensity, the sensor's own slopes (fractional subapertures), detector
    pixels and detector slopes, all against the oracle."""
    P = _P()
    from workloads import von_karman_opd
    s = tiny_sensor(n_pupil=220, n_fft=768, n_subap=40, pupil_sep_px=264.0, n_mod=24, mod_radius_lod=3.0,
                    diameter_m=8.222, fov_lod=SOUL_FOV_LOD, flags=FLAG_REF_SLOPES)
    opd = von_karman_opd(2, 220, 8.222, 0.126, 40.0, seed=31)
    x = torch.from_numpy(opd.astype(np.float32)).cuda()
    plan = P.Plan([s], max_frames=2)
    print("[gpu] SOUL geometry: forward + slopes", flush=True)
    I, sl, fl = plan.step(x)
    I_ref = O.forward(opd.astype(np.float32).astype(np.float64), s)
    m = _window_mask(s)
    Ig = I.cpu().numpy().astype(np.float64) * m[None]
    e = np.linalg.norm((Ig - I_ref * m[None]).reshape(2, -1), axis=1) / np.linalg.norm((I_ref * m[None]).reshape(2, -1), axis=1)
    assert e.max() < 1e-5
    s_ref, f_ref = O.slopes(I_ref, s)
    valid = O.valid_subapertures(s)
    assert np.array_equal(plan.valid_map(0), valid)
    assert O.slope_rel_rms(sl.cpu().numpy(), s_ref, valid) < 1e-4
    r = Fraction(11, 2)
    d = P.ccd_desc(120, r, 2.0e5, P.CCD_PHOTON | P.CCD_READOUT, readout_e=0.4, seed=8)
    print("[gpu] SOUL geometry: detector 120 px, pitch 11/2", flush=True)
    Iin = I_ref.astype(np.float32)
    got = plan.ccd(torch.from_numpy(Iin).cuda(), d)
    want = C.detector(Iin * m[None], 120, r, 2.0e5, 3, 0.4, 8)
    np.testing.assert_array_equal(got.cpu().numpy(), want.astype(np.float32))
    dsl, dfl = plan.ccd_slopes(got, d)
    ws, wf = C.detector_slopes(want, s, 120, r)
    assert O.slope_rel_rms(dsl.cpu().numpy(), ws, valid) < 1e-5


def test_soul_chain_in_the_benchmark_launch():
    """The SOUL chain exactly as the benchmark runs it: 1000 frames (200
    distinct screens repeated) in one plan call, the 120 px detector with
    photon and readout noise, detector slopes; frames 0 and 999 against the
    oracle (frame 999 repeats frame 199's screen but draws its own noise)."""
    P = _P()
    from workloads import von_karman_opd
    from workloads.configs import photo_electrons
    s = tiny_sensor(n_pupil=220, n_fft=768, n_subap=40, pupil_sep_px=264.0, n_mod=24, mod_radius_lod=3.0,
                    diameter_m=8.222, fov_lod=SOUL_FOV_LOD, flags=FLAG_REF_SLOPES)
    scr = von_karman_opd(200, 220, 8.222, 0.126, 40.0, seed=70, grid=512)
    opd = np.ascontiguousarray(np.tile(scr, (5, 1, 1)))
    x = torch.from_numpy(opd).cuda()
    plan = P.Plan([s], max_frames=1000)
    el = photo_electrons(8.0, 8.222, 0.0, 300.0, 0.000588, 0.32)
    r = Fraction(11, 2)
    d = P.ccd_desc(120, r, el, P.CCD_PHOTON | P.CCD_READOUT, 0.4, seed=12)
    print("[gpu] SOUL chain, 1000-frame launch", flush=True)
    I = plan.forward(x)
    pix = plan.ccd(I, d)
    sl, fl = plan.ccd_slopes(pix, d)
    torch.cuda.synchronize()
    m = _window_mask(s)
    valid = O.valid_subapertures(s)
    for f in (0, 999):
        I_ref = O.forward(opd[f:f + 1].astype(np.float64), s)
        Ig = I[f:f + 1].cpu().numpy().astype(np.float64) * m[None]
        e = np.linalg.norm(Ig - I_ref * m[None]) / np.linalg.norm(I_ref * m[None])
        print(f"      frame {f}: intensity rel err {e:.2e}", flush=True)
        assert e < 1e-5
        # detector and slopes of the GPU's own intensity, as the chain feeds them
        want = C.detector(Ig.astype(np.float32), 120, r, el, 3, 0.4, 12, frame0=f)
        np.testing.assert_array_equal(pix[f:f + 1].cpu().numpy(), want.astype(np.float32))
        ws, _ = C.detector_slopes(want, s, 120, r)
        assert O.slope_rel_rms(sl[f:f + 1].cpu().numpy(), ws, valid) < 1e-5
