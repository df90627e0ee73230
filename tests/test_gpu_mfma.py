"""Matrix-core (DFT-as-GEMM) precision form against the FP64 oracle.

The split forms carry ~16 (bf16 x3) or ~22 (fp16 x3) significand bits per
operand with fp32 accumulation; the one-term forms carry 8 (bf16) or 11
(fp16).  Every
comparison bounds the normwise figures and every pixel and subaperture on its
own (tests/parity.py), at a small multiple of what each form reaches, so that
a split that lost one of its three products (an error near the one-term
form's ~1e-3) fails:
  bf16 x3: intensity normwise 2e-5, pixel 5e-5; slopes pooled 1e-5, subap 5e-5
  fp16 x3: intensity normwise 1e-6, pixel 5e-6; slopes pooled 1e-6, subap 5e-6
  bf16:    intensity normwise 5e-3, pixel 2e-2; slopes pooled 3e-3, subap 2e-2
  fp16:    intensity normwise 1e-3, pixel 3e-3; slopes pooled 4e-4, subap 1.5e-3
Both one-term forms are held to the 1e-3 slope target of the matrix-core
forms on the 160 px sensor in the benchmark's 1000-frame launch.  On the 64 px
sensor the bf16 form reaches ~1.1e-3, above that target, and is reported as
such; the fp16 form reaches ~1.3e-4 there and meets it by its parity bound.
"""

import numpy as np
import pytest

import parity
from oracle import pwfs as O
from workloads import PREC_BF16, PREC_BF16X3, PREC_FP16, PREC_FP16X3, band_sampling, tiny_sensor, workload, workload_opd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BOUNDS = {PREC_BF16X3: parity.BF16X3, PREC_FP16X3: parity.FP16X3, PREC_BF16: parity.BF16, PREC_FP16: parity.FP16}
NAMES = {PREC_BF16X3: "bf16x3", PREC_FP16X3: "fp16x3", PREC_BF16: "bf16", PREC_FP16: "fp16"}


def _windows(I, s):
    D = s.n_pupil
    return np.stack([I[:, r:r + D, c:c + D] for r, c in O.image_origins(s)], axis=1)


def _run(s, opd, frames=None):
    from paper_2602_06688_amd import pwfs as P
    plan = P.Plan([s], max_frames=opd.shape[0])
    I, sl, fl = plan.step(torch.from_numpy(np.ascontiguousarray(opd, np.float32)).cuda())
    torch.cuda.synchronize()
    return I.cpu().numpy().astype(np.float64), sl.cpu().numpy().astype(np.float64), fl.cpu().numpy()[:, 0]


@pytest.mark.parametrize("prec", [PREC_BF16X3, PREC_FP16X3, PREC_BF16, PREC_FP16])
def test_64px_all_frames(prec):
    w = workload("cfg1")
    s = w.sensors[0].with_(precision=prec)
    opd = workload_opd(w)
    print(f"[gpu] mfma {NAMES[prec]} 64px 100 frames", flush=True)
    I, sl, fl = _run(s, opd)
    I_ref = O.forward(opd, w.sensors[0])
    s_ref, f_ref = O.slopes(I_ref, w.sensors[0])
    err = parity.errors(_windows(I, s), _windows(I_ref, s), sl, s_ref, O.valid_subapertures(s))
    print(f"      {parity.fmt(err)}; flux {np.abs(fl / f_ref - 1).max():.2e}", flush=True)
    parity.check(err, BOUNDS[prec])


@pytest.mark.parametrize("prec", [PREC_BF16X3, PREC_FP16X3])
def test_edge_sensors_mfma(prec):
    from workloads import von_karman_opd
    cases = [tiny_sensor(n_pupil=40, n_fft=128, n_subap=5, pupil_sep_px=48.0, n_mod=5, obstruction=0.3,
                         mod_radius_lod=3.0, precision=prec),
             tiny_sensor(n_pupil=48, n_fft=128, n_subap=12, pupil_sep_px=56.0, n_mod=8, precision=prec,
                         lambdas_nm=(600.0, 750.0, 900.0), lambda_weights=(0.2, 0.3, 0.5), flags=3),
             tiny_sensor(n_pupil=80, n_fft=256, n_subap=20, pupil_sep_px=96.0, n_mod=16, obstruction=0.28,
                         mod_radius_lod=2.0, precision=prec),
             # a 300 nm band in 16 samples
             tiny_sensor(n_pupil=48, n_fft=128, n_subap=12, pupil_sep_px=56.0, n_mod=8, precision=prec,
                         lambdas_nm=band_sampling(750.0, 300.0, 16)[0],
                         lambda_weights=band_sampling(750.0, 300.0, 16)[1]),
             # D not a multiple of 4: stage 1 stores element by element
             tiny_sensor(n_pupil=42, n_fft=128, n_subap=6, pupil_sep_px=48.0, n_mod=8, obstruction=0.2,
                         mod_radius_lod=3.0, precision=prec)]
    for s in cases:
        opd = von_karman_opd(3, s.n_pupil, 8.0, 0.5, 25.0, seed=7)
        print(f"[gpu] mfma {NAMES[prec]} D={s.n_pupil} N={s.n_fft} flags={s.flags}", flush=True)
        I, sl, _ = _run(s, opd)
        ref_s = s.with_(precision=0)
        I_ref = O.forward(opd, ref_s)
        s_ref, _ = O.slopes(I_ref, ref_s)
        if s.flags & 2:
            err = parity.errors(I, I_ref, sl, s_ref, O.valid_subapertures(s))
        else:
            err = parity.errors(_windows(I, s), _windows(I_ref, s), sl, s_ref, O.valid_subapertures(s))
        print(f"      {parity.fmt(err)}", flush=True)
        parity.check(err, BOUNDS[prec])


@pytest.mark.parametrize("prec", [PREC_BF16, PREC_FP16])
def test_edge_sensors_one_term(prec):
    """The one-term forms run K steps of 64, so a pupil whose 2D is not a
    multiple of 64 exercises the zero padding of both operands; D = 42 also
    takes stage 1's element-by-element stores."""
    from workloads import von_karman_opd
    cases = [tiny_sensor(n_pupil=40, n_fft=128, n_subap=5, pupil_sep_px=48.0, n_mod=5, obstruction=0.3,
                         mod_radius_lod=3.0, precision=prec),
             tiny_sensor(n_pupil=48, n_fft=128, n_subap=12, pupil_sep_px=56.0, n_mod=8, precision=prec,
                         lambdas_nm=(600.0, 750.0, 900.0), lambda_weights=(0.2, 0.3, 0.5), flags=3),
             # D not a multiple of 4, and K padding (128 - 84) longer than D
             tiny_sensor(n_pupil=42, n_fft=128, n_subap=6, pupil_sep_px=48.0, n_mod=8, obstruction=0.2,
                         mod_radius_lod=3.0, precision=prec)]
    for s in cases:
        opd = von_karman_opd(3, s.n_pupil, 8.0, 0.5, 25.0, seed=7)
        print(f"[gpu] mfma {NAMES[prec]} D={s.n_pupil} N={s.n_fft} flags={s.flags}", flush=True)
        I, sl, _ = _run(s, opd)
        ref_s = s.with_(precision=0)
        I_ref = O.forward(opd, ref_s)
        s_ref, _ = O.slopes(I_ref, ref_s)
        if s.flags & 2:
            err = parity.errors(I, I_ref, sl, s_ref, O.valid_subapertures(s))
        else:
            err = parity.errors(_windows(I, s), _windows(I_ref, s), sl, s_ref, O.valid_subapertures(s))
        print(f"      {parity.fmt(err)}", flush=True)
        parity.check(err, BOUNDS[prec])


def test_160px_sampled_bf16x3():
    w = workload("cfg2")
    s = w.sensors[0].with_(precision=PREC_BF16X3)
    opd = workload_opd(w, frames=range(64))
    print("[gpu] mfma bf16x3 160px 64 frames", flush=True)
    I, sl, _ = _run(s, opd)
    valid = O.valid_subapertures(s)
    for f in (0, 63):
        I_ref = O.forward(opd[f:f + 1], w.sensors[0])
        s_ref, _ = O.slopes(I_ref, w.sensors[0])
        err = parity.errors(_windows(I[f:f + 1], s), _windows(I_ref, s), sl[f:f + 1], s_ref, valid)
        print(f"      frame {f}: {parity.fmt(err)}", flush=True)
        parity.check(err, parity.BF16X3)


@pytest.mark.parametrize("prec", [PREC_BF16X3, PREC_FP16X3, PREC_BF16, PREC_FP16])
def test_160px_full_size_in_the_benchmark_launch(prec):
    """All 1000 frames in one plan, as the bench launches the matrix-core
    forms.  A frame's 320 image columns are 2.5 column tiles, so odd frames
    start in the middle of a tile shared with the frame before; frames 0, 1
    (the first straddling tile), 517 and 999 against the oracle, every frame
    finite with its flux in range.  The one-term bf16 form is held here to
    the 1e-3 relative slope RMS target of the matrix-core forms."""
    w = workload("cfg2")
    s = w.sensors[0].with_(precision=prec)
    print(f"[gpu] mfma {NAMES[prec]} 160px 1000 frames: inputs", flush=True)
    opd = workload_opd(w)
    print(f"[gpu] mfma {NAMES[prec]} 160px 1000 frames: forward + slopes", flush=True)
    I, sl, fl = _run(s, opd)
    assert np.isfinite(I).all() and np.isfinite(sl).all()
    assert (fl > 0.5).all() and (fl < 1.0 + 1e-3).all()
    valid = O.valid_subapertures(s)
    frames = (0, 1, 517, 999)
    refs = []
    for f in frames:
        I_ref = O.forward(opd[f:f + 1], w.sensors[0])
        refs.append(O.slopes(I_ref, w.sensors[0]) + (I_ref,))
    for f, (s_ref, f_ref, I_ref) in zip(frames, refs):
        err = parity.errors(_windows(I[f:f + 1], s), _windows(I_ref, s), sl[f:f + 1], s_ref, valid)
        print(f"      frame {f}: {parity.fmt(err)}", flush=True)
        parity.check(err, BOUNDS[prec])
        assert abs(fl[f] / f_ref[0] - 1) <= (1e-3 if prec in (PREC_BF16, PREC_FP16) else 1e-5)
    if prec in (PREC_BF16, PREC_FP16):
        pooled = parity.slope_rms_error(np.concatenate([sl[f:f + 1] for f in frames]),
                                        np.concatenate([r[0] for r in refs]), valid)
        print(f"      {NAMES[prec]} one-term, pooled slope rms over the sampled frames {pooled:.2e}", flush=True)
        assert pooled <= 1e-3


@pytest.mark.parametrize("prec", [PREC_BF16X3, PREC_FP16X3, PREC_BF16, PREC_FP16])
def test_pass_split_gives_the_same_bits(prec):
    """Column tiles run across the frames of a pass, so where a tile straddles
    two frames, and which tile is ragged, depend on the pass size.  Each output
    element still sees the same products in the same order: 12 frames in one
    pass and in passes of 5, 5, 2 (and of 1) give identical intensities and
    slopes.  D = 40 gives Nc = 80 image columns per frame, 0.625 of a tile."""
    from workloads import von_karman_opd
    from paper_2602_06688_amd import pwfs as P
    s = tiny_sensor(n_pupil=40, n_fft=128, n_subap=5, pupil_sep_px=48.0, n_mod=5, obstruction=0.3,
                    mod_radius_lod=3.0, precision=prec)
    opd = von_karman_opd(12, s.n_pupil, 8.0, 0.5, 25.0, seed=11)
    x = torch.from_numpy(np.ascontiguousarray(opd, np.float32)).cuda()
    plan = P.Plan([s], max_frames=12)
    print(f"[gpu] mfma {NAMES[prec]} pass split: one pass of {plan.get_tuning()['chunk']}", flush=True)
    I0, S0, F0 = [t.clone() for t in plan.step(x)]
    for chunk in (5, 1):
        print(f"[gpu] mfma {NAMES[prec]} pass split: passes of {chunk}", flush=True)
        plan.set_tuning(chunk=chunk)
        I1, S1, F1 = plan.step(x)
        torch.cuda.synchronize()
        assert torch.equal(I0, I1) and torch.equal(S0, S1) and torch.equal(F0, F1)
