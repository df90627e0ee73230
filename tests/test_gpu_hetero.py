"""Heterogeneous batch: six sensors of different pupil, FFT size, modulation
and three wavelengths in one plan; the persistent launch must give exactly
the per-sensor launches' results, and both match the FP64 oracle."""

import numpy as np
import pytest

import parity
from oracle import pwfs as O
from workloads import tiny_sensor, von_karman_opd, workload, workload_opd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LAMS = dict(lambdas_nm=(600.0, 750.0, 900.0), lambda_weights=(1 / 3, 1 / 3, 1 / 3))


def _windows(I, s):
    D = s.n_pupil
    return np.stack([I[:, r:r + D, c:c + D] for r, c in O.image_origins(s)], axis=1)


def _small_hetero():
    spec = [(80, 256, 2.0, 8), (120, 384, 3.0, 8), (160, 512, 3.0, 4), (160, 512, 4.0, 4),
            (240, 768, 5.0, 4), (240, 768, 5.0, 4)]
    return [tiny_sensor(n_pupil=d, n_fft=n, n_subap=d // 4, n_mod=k, pupil_sep_px=1.2 * d, mod_radius_lod=r,
                        obstruction=0.28, diameter_m=38.5, **LAMS) for d, n, r, k in spec]


def _packed(opds):
    F = opds[0].shape[0]
    return np.concatenate([o.reshape(F, -1) for o in opds], axis=1)


def _unpack(plan, arr, which):
    out = []
    for s, info in zip(plan.sensors, plan.info):
        if which == "I":
            N = s.n_fft
            out.append(arr[:, info.intensity_offset:info.intensity_offset + N * N].reshape(-1, N, N))
        else:
            n = s.n_subap
            out.append(arr[:, info.slope_offset:info.slope_offset + 2 * n * n].reshape(-1, 2, n, n))
    return out


def test_persistent_equals_launches_and_oracle():
    from paper_2602_06688_amd import pwfs as P
    sensors = _small_hetero()
    F = 2
    opds = [von_karman_opd(F, s.n_pupil, 38.5, 0.157, 25.0, seed=40 + i) for i, s in enumerate(sensors)]
    x = torch.from_numpy(_packed(opds)).cuda()
    plan = P.Plan(sensors, max_frames=F)
    print("[gpu] hetero small: per-sensor launches", flush=True)
    I0, S0, F0 = plan.step(x)
    torch.cuda.synchronize()
    for chunk in sorted({1, plan.get_tuning()["max_chunk"]}):
        for w in (1, 2):
            print(f"[gpu] hetero small: persistent chunk={chunk} wg_per_cu={w}", flush=True)
            plan.set_tuning(mode=P.MODE_PERSISTENT, chunk=chunk, wg_per_cu=w)
            I1, S1, F1 = plan.step(x)
            torch.cuda.synchronize()
            assert torch.equal(I0, I1) and torch.equal(S0, S1) and torch.equal(F0, F1)
    Is = _unpack(plan, I0.cpu().numpy().astype(np.float64), "I")
    Ss = _unpack(plan, S0.cpu().numpy().astype(np.float64), "S")
    for s, o, Ig, Sg in zip(sensors, opds, Is, Ss):
        I_ref = O.forward(o, s)
        s_ref, _ = O.slopes(I_ref, s)
        err = parity.errors(_windows(Ig, s), _windows(I_ref, s), Sg, s_ref, O.valid_subapertures(s))
        print(f"      D={s.n_pupil} N={s.n_fft}: {parity.fmt(err)}", flush=True)
        parity.check(err, parity.FP32)


def test_full_heterogeneous_workload_sampled():
    """The six-instance, three-wavelength workload at full size (first 8
    timesteps): persistent == launches; sensors 0 and 2 against the oracle."""
    from paper_2602_06688_amd import pwfs as P
    w = workload("cfg4")
    F = 8
    opds = [workload_opd(w, i, frames=range(F)) for i in range(len(w.sensors))]
    x = torch.from_numpy(_packed(opds)).cuda()
    plan = P.Plan(list(w.sensors), max_frames=F)
    print("[gpu] hetero full: launches", flush=True)
    I0, S0, _ = plan.step(x)
    plan.set_tuning(mode=P.MODE_PERSISTENT)
    print("[gpu] hetero full: persistent", flush=True)
    I1, S1, _ = plan.step(x)
    torch.cuda.synchronize()
    assert torch.equal(I0, I1) and torch.equal(S0, S1)
    Is = _unpack(plan, I0.cpu().numpy().astype(np.float64), "I")
    Ss = _unpack(plan, S0.cpu().numpy().astype(np.float64), "S")
    for i in (0, 2):
        s = w.sensors[i]
        I_ref = O.forward(opds[i][:1], s)
        s_ref, _ = O.slopes(I_ref, s)
        err = parity.errors(_windows(Is[i][:1], s), _windows(I_ref, s), Ss[i][:1], s_ref, O.valid_subapertures(s))
        print(f"      sensor {i}: {parity.fmt(err)}", flush=True)
        parity.check(err, parity.FP32)


def test_persistent_mode_rejected_when_ineligible():
    from paper_2602_06688_amd import pwfs as P
    plan = P.Plan([workload("cfg1").sensors[0]], max_frames=2)     # N = 128
    with pytest.raises(P.PwfsError) as ei:
        plan.set_tuning(mode=P.MODE_PERSISTENT)
    assert ei.value.code == P.PWFS_EUNSUPPORTED
    with pytest.raises(P.PwfsError):
        plan.set_tuning(chunk=10 ** 6)


def test_persistent_wait_timeout_is_reported():
    """A dependency wait that gives up must not pass silently: forced from the
    host (a negative spin limit makes every wait give up at once, without
    polling), the persistent launch skips the waiting items and still ends;
    pwfs_device_status then reports PWFS_EHIP once and clears the flag, and the plan
    runs correctly again with the default limit."""
    from paper_2602_06688_amd import pwfs as P
    sensors = _small_hetero()[:3]
    F = 2
    opds = [von_karman_opd(F, s.n_pupil, 38.5, 0.157, 25.0, seed=40 + i) for i, s in enumerate(sensors)]
    x = torch.from_numpy(_packed(opds)).cuda()
    plan = P.Plan(sensors, max_frames=F)
    I0, S0, _ = [t.clone() for t in plan.step(x)]
    plan.status()                                        # nothing to report
    print("[gpu] hetero: persistent pass with every dependency wait forced to give up", flush=True)
    plan.set_tuning(mode=P.MODE_PERSISTENT, spin_limit=-1)
    plan.forward(x)
    with pytest.raises(P.PwfsError) as ei:
        plan.status()
    assert ei.value.code == P.PWFS_EHIP and "gave up" in str(ei.value)
    plan.status()                                        # reported once, then cleared
    print("[gpu] hetero: default spin limit again", flush=True)
    plan.set_tuning(spin_limit=0)
    I1, S1, _ = plan.step(x)
    plan.status()
    assert torch.equal(I0, I1) and torch.equal(S0, S1)


def test_row_tiles_give_identical_bits_in_both_modes():
    """Every compiled row tile (8 or 16 rows per row-pass workgroup, chosen
    per sensor) gives the default tile's bits, with per-sensor launches and
    in the persistent launch; tiles that are not compiled for a sensor's N
    are refused."""
    from paper_2602_06688_amd import pwfs as P
    sensors = _small_hetero()
    F = 2
    opds = [von_karman_opd(F, s.n_pupil, 38.5, 0.157, 25.0, seed=40 + i) for i, s in enumerate(sensors)]
    x = torch.from_numpy(_packed(opds)).cuda()
    plan = P.Plan(sensors, max_frames=F)
    assert [plan.row_tile(i) for i in range(6)] == [8, 16, 8, 8, 8, 8]
    I0, S0, _ = [t.clone() for t in plan.step(x)]
    alt = [16, 8, 16, 16, 16, 16]
    for mode in (P.MODE_LAUNCHES, P.MODE_PERSISTENT):
        for pick in ([1, 1, 1, 1, 1, 1], [0, 1, 0, 1, 0, 1]):
            tiles = [a if p else 0 for a, p in zip(alt, pick)]
            print(f"[gpu] hetero small: mode {mode} row tiles {tiles}", flush=True)
            for i, r in enumerate(tiles):
                plan.set_row_tile(i, r)
            plan.set_tuning(mode=mode)
            I1, S1, _ = plan.step(x)
            torch.cuda.synchronize()
            assert torch.equal(I0, I1) and torch.equal(S0, S1)
    for i in range(6):
        plan.set_row_tile(i, 0)
    assert [plan.row_tile(i) for i in range(6)] == [8, 16, 8, 8, 8, 8]
    for bad in (4, 12, 32):
        with pytest.raises(P.PwfsError) as ei:
            plan.set_row_tile(2, bad)
        assert ei.value.code == P.PWFS_EINVAL
    with pytest.raises(P.PwfsError):
        plan.set_row_tile(6, 8)
