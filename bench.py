"""Throughput of the pyramid-sensor path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

A step is one pass of the whole path (forward model + binning/slopes) over
the 1000-frame batch of the 160 px pupil / 512 px transform / 48-point
modulation / 40 x 40 subaperture workload, with the synthetic von Karman
inputs already resident in HBM.  The step is captured once as a HIP graph;
the timed region is K replays of it (events around each replay give the
median), bracketed by device synchronisations.  Kernel durations for the
roofline come from HIP events around every launch of K eager steps of the
same batch, run right after.  Every form's error is measured against the
FP64 oracle on the frames of the CPU baseline.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PWFS frames/s @160px pupil,48 mod pts: plain vs MFMA/surrogate at stated error"
def poly_form(P, torch, dev, x, s, steps: int, n_lambda: int = 16, frames: int = 200):
    """The 160 px sensor sampling a 300 nm band around 750 nm with 16
    wavelengths (midpoint rule, equal weights): the plain FP32 path, 16 times
    the work of one wavelength per frame."""
    from workloads import band_sampling
    lams, ws = band_sampling(750.0, 300.0, n_lambda)
    sp = s.with_(lambdas_nm=lams, lambda_weights=ws)
    plan = P.Plan([sp], max_frames=frames, device=dev)
    xi = x[:frames].contiguous()
    out = plan.step(xi)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.step(xi, *out)
    torch.cuda.synchronize(dev)
    fs = frames * steps / (time.perf_counter() - t0)
    fl = nominal_flops(sp)["path"]
    a = fl * fs / 1e12
    print(f"# polychromatic {n_lambda} wavelengths: {fs:.0f} frames/s ({a:.1f} TFLOP/s nominal)",
          file=sys.stderr, flush=True)
    return {"value": round(fs, 1), "unit": "frames/s",
            "workload": f"160 px sensor, {n_lambda} wavelengths over 600-900 nm, {frames} frames per step",
            "roofline_path": {"bound": "alu", "achieved": round(a, 2), "peak": FP32_PEAK_TFLOPS,
                              "unit": "TFLOP/s", "frac": round(a / FP32_PEAK_TFLOPS, 4),
                              "flops_per_frame": fl}}


FP32_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0}   # MI355X dense matrix peaks
HBM_PEAK_GBS = 8000.0        # MI355X published HBM3E bandwidth


def nominal_flops(s) -> dict:
    """Nominal work per frame of the plain method (5 M log2 M per complex
    M-point FFT).  Whole path: per wavelength and modulation point one forward
    and one inverse N x N transform, the mask product (6 flops/px), the |e|^2
    accumulation (3 flops/px) and the complex modulation/phase product
    (6 flops per pupil px); the column pass owns the column halves of both
    2-D transforms plus mask and accumulation."""
    N, D = s.n_fft, s.n_pupil
    K = s.n_mod * len(s.lambdas_nm)
    fft2d = 5.0 * N * N * math.log2(N * N)
    path = K * (2 * fft2d + 9.0 * N * N + 6.0 * D * D)
    cols = K * (2 * 5.0 * N * N * math.log2(N) + 9.0 * N * N)
    return {"path": path, "cols": cols}


def mfma_flops(s, terms: int) -> dict:
    """Executed matrix-core flops per frame of the DFT-as-GEMM form: stage 1
    (2 Nc x D x Kp per distinct cosine) and stage 2 (2 Nc x Nc x Kp per point),
    2 flops per MAC, times the number of split products."""
    D, N = s.n_pupil, s.n_fft
    Nc = N if (s.flags & 2) else 2 * D
    Kp = (2 * D + 31) // 32 * 32
    L = len(s.lambdas_nm)
    n_a = min(s.n_mod // 2 + 1, s.n_mod)
    g1 = L * n_a * 2 * Nc * D * Kp * 2.0 * terms
    g2 = L * s.n_mod * 2 * Nc * Nc * Kp * 2.0 * terms
    return {"stage1": g1, "stage2": g2}


def time_form(P, torch, s, x, n_frames, steps, warmup, ref_I, ref_S, dev, stream, label, terms, dtype, refs=None):
    """frames/s of one precision form (median of graph replays of the batch),
    its error against the FP64 oracle on the oracle's frames (refs) and
    against the FP32 path's outputs (ref_I, ref_S) on all frames, and its
    matrix-core roofline (HIP events over eager steps)."""
    plan = P.Plan([s], max_frames=n_frames, device=dev, stream=stream)
    I = plan.new_intensity(n_frames)
    S = plan.new_slopes(n_frames)
    Fl = torch.zeros((n_frames, 1), dtype=torch.float32, device=dev)
    import numpy as np
    for _ in range(warmup):
        plan.step(x, I, S, Fl, stream=stream)
    torch.cuda.synchronize(dev)
    wall, ms = graph_replays(torch, dev, lambda st: plan.step(x, I, S, Fl, stream=st), steps)
    med = float(np.median(ms)) / 1e3
    plan.profile(4096)
    torch.cuda.synchronize(dev)
    for _ in range(steps):
        plan.step(x, I, S, Fl, stream=stream)
    torch.cuda.synchronize(dev)
    g2_ms, g2_n = plan.profile_read("mfma")
    g1_ms, g1_n = plan.profile_read("rows")
    plan.profile(0)
    valid = torch.from_numpy(plan.valid_map(0)).to(dev)
    D = s.n_pupil
    win = [(r, c) for r in (s.n_fft // 2 - int(s.pupil_sep_px) // 2 - D // 2,
                            s.n_fft // 2 + int(s.pupil_sep_px) // 2 - D // 2)
           for c in (s.n_fft // 2 - int(s.pupil_sep_px) // 2 - D // 2,
                     s.n_fft // 2 + int(s.pupil_sep_px) // 2 - D // 2)]
    a = torch.stack([I[:, r:r + D, c:c + D] for r, c in win], 1).reshape(n_frames, -1).double()
    b = torch.stack([ref_I[:, r:r + D, c:c + D] for r, c in win], 1).reshape(n_frames, -1).double()
    ie = ((a - b).norm(dim=1) / b.norm(dim=1)).max().item()
    sa = S.double()[:, :, valid]
    sb = ref_S.double()[:, :, valid]
    se = ((sa - sb).norm() / sb.norm()).item()
    fl = mfma_flops(s, terms)
    frames = n_frames * steps
    ach = fl["stage2"] * frames / (g2_ms / 1e3) / 1e12 if g2_ms > 0 else None
    peak = MFMA_PEAK_TFLOPS[dtype]
    ev = oracle_errors(torch, I, S, s, refs) if refs is not None else None
    out = {"value": round(n_frames / med, 2), "unit": "frames/s", "median_step_ms": round(med * 1e3, 4),
           "mean_step_ms": round(wall / steps * 1e3, 4), "replays": steps,
           "errors_vs_oracle": ev,
           "at_stated_error": (ev["slope_rel_rms"] <= 1e-3) if ev else None,
           "intensity_rel_err_max_vs_fp32": ie, "slope_rel_rms_vs_fp32": se,
           "roofline": {"kernel": "k_mfma_cols_ws (stage 2: e_k = Qy_k T, |e|^2 accumulate)", "bound": "mfma",
                        "achieved": round(ach, 2) if ach else None, "peak": peak, "unit": "TFLOP/s",
                        "frac": round(ach / peak, 4) if ach else None, "traffic": None,
                        "avg_launch_ms": round(g2_ms / max(1, g2_n), 4), "flops_per_frame": fl["stage2"]},
           "stage1_ms_per_step": round(g1_ms / steps, 3), "stage2_ms_per_step": round(g2_ms / steps, 3)}
    plan.close()
    print(f"# {label}: {out['value']:.0f} frames/s, vs fp32: intensity {ie:.2e}, slopes {se:.2e}; vs oracle: "
          f"{ev}", file=sys.stderr, flush=True)
    return out


def surrogate_form(torch, dev, n_train, n_test, epochs, reps):
    """Learned surrogate of the 160 px sensor: trained on n_train samples of
    the plain kernels, timed on n_test held-out samples; errors are against
    the plain path (the reference), next to the linear interaction-matrix method."""
    from paper_2602_06688_amd.surrogate import SurrogatePipeline
    from workloads import workload
    from workloads.modes import coefficient_sigmas, kl_modes
    w = workload("cfg5")
    s = w.sensors[0]
    ex = w.extra
    t0 = time.perf_counter()
    modes, ev = kl_modes(s.n_pupil, s.obstruction, s.diameter_m, w.L0_m, ex["n_modes"])
    sig = coefficient_sigmas(ev, ex["residual_rms_nm"], s.lambdas_nm[0])
    pipe = SurrogatePipeline(s, modes, sig, device=dev)
    z, S = pipe.generate(n_train, seed=w.seeds[0])
    zt, St = pipe.generate(n_test, seed=ex["test_seed"])
    torch.cuda.synchronize(dev)
    t_data = time.perf_counter() - t0
    pipe.interaction_matrix()
    e_lin = pipe.rel_error(pipe.linear_predict(zt), St)
    rep = pipe.train(z, S, hidden=(ex["hidden"], ex["hidden"]), epochs=epochs, batch=1024, lr=1e-3)
    out = torch.empty_like(St)
    pipe.predict(zt, out=out)
    e_nn = pipe.rel_error(out, St)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(reps):
        pipe.predict(zt, out=out)
    torch.cuda.synchronize(dev)
    dt = (time.perf_counter() - t0) / reps
    sizes = [ex["n_modes"], ex["hidden"], ex["hidden"], 2 * s.n_subap ** 2]
    # matrix-core flops per frame: the network (one bf16 product per layer)
    # and the linear part IM z (one bf16 product)
    fl = 2.0 * sum(a * b for a, b in zip(sizes[:-1], sizes[1:])) + 2.0 * sizes[0] * sizes[-1]
    ach = fl * n_test / dt / 1e12
    print(f"# surrogate: {n_test / dt:.0f} frames/s, error {e_nn:.3e} (linear IM {e_lin:.3e}), "
          f"train {rep.seconds:.1f} s", file=sys.stderr, flush=True)
    return {"value": round(n_test / dt, 1), "unit": "frames/s",
            "slope_rel_rms_vs_plain": e_nn, "linear_im_slope_rel_rms_vs_plain": e_lin,
            "train_samples": n_train, "test_samples": n_test, "epochs": epochs,
            "train_seconds": round(rep.seconds, 2), "data_seconds": round(t_data, 2),
            "loss_first_last": [rep.losses[0], rep.losses[-1]],
            "form": "IM z + r_rms * net(z): push-pull interaction matrix plus the trained correction",
            "roofline": {"kernel": "k_gemm_ws (inference products: network and folded linear part, bf16, fp32 accumulation)", "bound": "mfma",
                         "achieved": round(ach, 2), "peak": MFMA_PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                         "frac": round(ach / MFMA_PEAK_TFLOPS["bf16"], 4), "flops_per_frame": fl,
                         "traffic": None}}


def surrogate_study(torch, dev, n_max: int, n_test: int, configs) -> dict:
    """Error of the learned surrogate against the plain path as the training
    set, the width of the hidden layers and the epochs grow: one pool of
    n_max training samples (seed of the workload) and one held-out test set,
    the push-pull interaction matrix built once, then one network per
    (samples, width, epochs) trained on the first `samples` of the pool."""
    from paper_2602_06688_amd.surrogate import SurrogatePipeline
    from workloads import workload
    from workloads.modes import coefficient_sigmas, kl_modes
    w = workload("cfg5")
    s = w.sensors[0]
    ex = w.extra
    modes, ev = kl_modes(s.n_pupil, s.obstruction, s.diameter_m, w.L0_m, ex["n_modes"])
    sig = coefficient_sigmas(ev, ex["residual_rms_nm"], s.lambdas_nm[0])
    pipe = SurrogatePipeline(s, modes, sig, device=dev)
    t0 = time.perf_counter()
    z, S = pipe.generate(n_max, seed=w.seeds[0])
    zt, St = pipe.generate(n_test, seed=ex["test_seed"])
    torch.cuda.synchronize(dev)
    t_data = time.perf_counter() - t0
    pipe.interaction_matrix()
    e_lin = pipe.rel_error(pipe.linear_predict(zt), St)
    print(f"# study: {n_max} + {n_test} samples in {t_data:.1f} s, linear IM error {e_lin:.4e}", file=sys.stderr,
          flush=True)
    rows = []
    for n, width, epochs in configs:
        rep = pipe.train(z[:n], S[:n], hidden=(width, width), epochs=epochs, batch=1024, lr=1e-3)
        e = pipe.rel_error(pipe.predict(zt), St)
        e_train = pipe.rel_error(pipe.predict(z[:n_test]), S[:n_test])
        rows.append({"train_samples": n, "hidden": width, "epochs": epochs, "test_error": e,
                     "train_error": e_train, "train_seconds": round(rep.seconds, 1),
                     "loss_last": rep.losses[-1]})
        print(f"# study: n={n} width={width} epochs={epochs}: test {e:.4e} train {e_train:.4e} "
              f"({rep.seconds:.1f} s)", file=sys.stderr, flush=True)
    return {"linear_im_error": e_lin, "test_samples": n_test, "data_seconds": round(t_data, 1), "runs": rows}


def detector_form(P, torch, dev, stream, x, plan, I, s, steps: int):
    """The plain path followed by the detector (120 x 120, photon + excess +
    readout noise, magnitude-8 source) and the slopes on detector pixels:
    frames/s over the 1000-frame batch, and the detector kernel against the
    HBM roof (it reads the four pupil images and writes the detector frame)."""
    from workloads.configs import soul_detector
    F = int(x.shape[0])
    det = soul_detector(s)
    flags = P.CCD_PHOTON | P.CCD_EXCESS | P.CCD_READOUT
    d = P.ccd_desc(det["n_det"], det["rebin"], det["electrons"], flags, det["readout_e"], seed=11)
    pix = torch.empty((F, det["n_det"], det["n_det"]), dtype=torch.float32, device=dev)
    sl = torch.empty((F, 2, s.n_subap, s.n_subap), dtype=torch.float32, device=dev)
    fl = torch.zeros(F, dtype=torch.float32, device=dev)

    def one(k):
        plan.forward(x, I, stream=stream)
        plan.ccd(I, d, frame0=k * F, out=pix, stream=stream)
        plan.ccd_slopes(pix, d, out=sl, flux=fl, stream=stream)

    one(0)
    torch.cuda.synchronize(dev)
    plan.profile(4096)
    t0 = time.perf_counter()
    for k in range(steps):
        one(k + 1)
    torch.cuda.synchronize(dev)
    dt = (time.perf_counter() - t0) / steps
    ccd_ms, ccd_n = plan.profile_read("ccd")
    plan.profile(0)
    byts = 4.0 * (4 * s.n_pupil ** 2 + det["n_det"] ** 2)        # image pixels read + detector pixels written
    ach = byts * F * steps / (ccd_ms / 1e3) / 1e9
    print(f"# detector: {F / dt:.0f} frames/s, k_ccd {ccd_ms / max(1, ccd_n):.3f} ms per launch", file=sys.stderr,
          flush=True)
    return {"value": round(F / dt, 1), "unit": "frames/s", "ms_per_step": round(dt * 1e3, 4),
            "detector": {"n_det": det["n_det"], "rebin": det["rebin"], "electrons_per_frame": round(det["electrons"], 1),
                         "readout_e": det["readout_e"], "noise": "photon+excess+readout"},
            "roofline": {"kernel": "k_ccd (rebin, Poisson, Gamma, Gaussian per detector pixel)", "bound": "hbm",
                         "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_frame": byts,
                         "avg_launch_ms": round(ccd_ms / max(1, ccd_n), 4), "traffic": None,
                         "note": "bytes are reported for reference; the kernel is bound by its float64 "
                                 "sampling arithmetic (Philox, Poisson inversion, Gamma), not by HBM"}}


def roof_form(P, torch, dev, x, s, steps: int):
    """The 160 px sensor as a double roof (two arms, one roof edge each) over
    the same 1000 frames: forward + slopes.  Nominal flops: each arm needs a
    1-D transform pair along its roof axis over the N x N plane per point,
    so the two arms together count as one 2-D pair, the pyramid's figure
    (the kernels also run the flat-mask axis, which is work the method does
    not need)."""
    from workloads import FLAG_DOUBLE_ROOF, FLAG_REF_SLOPES
    sr = s.with_(flags=FLAG_DOUBLE_ROOF | FLAG_REF_SLOPES)
    F = int(x.shape[0])
    plan = P.Plan([sr], max_frames=F, device=dev)
    out = plan.step(x)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.step(x, *out)
    torch.cuda.synchronize(dev)
    fs = F * steps / (time.perf_counter() - t0)
    fl = nominal_flops(s)["path"]
    a = fl * fs / 1e12
    print(f"# double roof: {fs:.0f} frames/s ({a:.1f} TFLOP/s nominal)", file=sys.stderr, flush=True)
    return {"value": round(fs, 1), "unit": "frames/s",
            "workload": "160 px double roof, N=512, 48 points, 40x40, 1000 frames per step",
            "roofline_path": {"bound": "alu", "achieved": round(a, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": round(a / FP32_PEAK_TFLOPS, 4), "flops_per_frame": fl}}


def soul_form(P, torch, dev, stream, steps: int, frames: int = 1000, distinct: int = 200):
    """The SOUL pyramid of Appendix B as one chain: 220 px pupil (8.22 m),
    40 x 40 subapertures of 5.5 px, pupils 48 subapertures apart, 3 lambda/D
    modulation at 750 nm sampled by 24 points (Table 2: 24 transforms per
    step), a 2.0 arcsec field stop, on a 768 grid (the paper pads to 660); a
    120 x 120 detector of 5.5
    transform pixels per pixel with photon and readout noise (magnitude 8,
    300 nm, 0.588 ms, QE 0.32, 0.4 e-); slopes on detector pixels.
    frames/s of the chain over `frames` frames (`distinct` screens at 0.8
    arcsec seeing, repeated)."""
    import numpy as np
    from fractions import Fraction
    from workloads import FLAG_REF_SLOPES, tiny_sensor, von_karman_opd
    from workloads.configs import photo_electrons
    # field stop: the listing's 2.0 arcsec as lambda/D at 750 nm on 8.222 m
    fov = 2.0 / (750e-9 / 8.222 * 206264.806)
    s = tiny_sensor(n_pupil=220, n_fft=768, n_subap=40, pupil_sep_px=264.0, n_mod=24, mod_radius_lod=3.0,
                    diameter_m=8.222, fov_lod=fov, flags=FLAG_REF_SLOPES)
    scr = von_karman_opd(distinct, 220, 8.222, 0.126, 40.0, seed=70, grid=512)
    x = torch.from_numpy(np.ascontiguousarray(np.tile(scr, (frames // distinct, 1, 1)))).to(dev)
    plan = P.Plan([s], max_frames=frames, device=dev)
    el = photo_electrons(8.0, 8.222, 0.0, 300.0, 0.000588, 0.32)
    d = P.ccd_desc(120, Fraction(11, 2), el, P.CCD_PHOTON | P.CCD_READOUT, 0.4, seed=12)
    I = plan.forward(x, stream=stream)
    pix = torch.empty((frames, 120, 120), dtype=torch.float32, device=dev)
    sl = torch.empty((frames, 2, 40, 40), dtype=torch.float32, device=dev)
    fl = torch.zeros(frames, dtype=torch.float32, device=dev)

    def one(k):
        plan.forward(x, I, stream=stream)
        plan.ccd(I, d, frame0=k * frames, out=pix, stream=stream)
        plan.ccd_slopes(pix, d, out=sl, flux=fl, stream=stream)

    one(0)
    torch.cuda.synchronize(dev)
    plan.profile(4096)
    t0 = time.perf_counter()
    for k in range(steps):
        one(k + 1)
    torch.cuda.synchronize(dev)
    dt = (time.perf_counter() - t0) / steps
    kms = {k: round(plan.profile_read(k)[0] / steps, 3) for k in ("field", "rows", "cols", "ccd", "slopes")}
    plan.profile(0)
    assert bool(torch.isfinite(sl).all())
    fs = frames / dt
    fl_frame = nominal_flops(s)["path"]
    a = fl_frame * fs / 1e12
    print(f"# SOUL chain: {fs:.0f} frames/s ({a:.1f} TFLOP/s nominal), ms per step {kms}", file=sys.stderr,
          flush=True)
    return {"value": round(fs, 1), "unit": "frames/s", "ms_per_step": round(dt * 1e3, 4),
            "workload": "SOUL pyramid: 220 px, 40x40 subap (5.5 px), 24 points at 3 lambda/D, 2.0 arcsec "
                        "square field stop, N=768; "
                        "120 px detector at 11/2 transform px per px, photon + readout noise; detector slopes",
            "frames_per_step": frames, "electrons_per_frame": round(el, 1), "kernel_ms_per_step": kms,
            "roofline_path": {"bound": "alu", "achieved": round(a, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": round(a / FP32_PEAK_TFLOPS, 4), "flops_per_frame": fl_frame}}


def loop_form(torch, dev, steps: int = 2000):
    """Closed AO loop of the SOUL configuration around the 160 px sensor
    (500 KL modes, four frozen-flow layers, the listing's integrator and
    delay): calibrated by push-pull, one timestep captured in a HIP graph,
    `steps` replays timed; then the residual wavefront over 200 more steps."""
    import numpy as np
    from paper_2602_06688_amd import pwfs as P
    from paper_2602_06688_amd.loop import ClosedLoop
    from workloads import workload
    from workloads.configs import soul_loop
    from workloads.modes import kl_modes
    from workloads.screens import periodic_layer
    s = workload("cfg2").sensors[0]
    cfg = soul_loop(s)
    t0 = time.perf_counter()
    Z, _ = kl_modes(s.n_pupil, s.obstruction, s.diameter_m, cfg["L0_m"], cfg["n_modes"])
    screens = np.stack([periodic_layer(cfg["screen_px"], cfg["pixel_m"], cfg["r0_m"], cfg["L0_m"], sd)
                        for sd in cfg["seeds"]])
    params = [(float(np.sqrt(c)), o[0], o[1], v[0], v[1])
              for c, o, v in zip(cfg["cn2"], cfg["origins_px"], cfg["velocities_px"])]
    g = np.concatenate([np.full(n, v) for v, n in zip(cfg["gains"], cfg["groups"])])
    ff = np.concatenate([np.full(n, v) for v, n in zip(cfg["ff"], cfg["groups"])])
    loop = ClosedLoop(s, Z.T.copy(), screens, params, g, ff, cfg["delay"], device=dev)
    loop.calibrate(delta_nm=10.0)
    t_setup = time.perf_counter() - t0
    loop.reset()
    loop.capture()
    loop.run(50)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    loop.run(steps)
    torch.cuda.synchronize(dev)
    dt = (time.perf_counter() - t0) / steps
    # residual and open-loop wavefront (telemetry, outside the timed region)
    c = np.arange(s.n_pupil) - (s.n_pupil - 1) / 2.0
    r2 = c[None, :] ** 2 + c[:, None] ** 2
    rad = s.n_pupil / 2.0
    pupil = (r2 <= rad * rad) & (r2 >= (s.obstruction * rad) ** 2)
    closed = []
    loop.run(200, record=lambda lp: closed.append(lp.residual_rms(pupil)))
    st = torch.zeros(1, dtype=torch.int64, device=dev)
    opn = []
    for t in range(0, steps + 250, 250):
        st.fill_(t)
        o = P.layers(loop.screens, loop.layer_params, s.n_pupil, st).cpu().numpy()[pupil]
        opn.append(float(np.sqrt(np.mean((o - o.mean()) ** 2))))
    fl = nominal_flops(s)["path"]
    ach = fl / dt / 1e12
    print(f"# closed loop: {1.0 / dt:.0f} timesteps/s ({dt * 1e3:.3f} ms), residual {np.mean(closed):.0f} nm "
          f"(open loop {np.mean(opn):.0f} nm)", file=sys.stderr, flush=True)
    return {"value": round(1.0 / dt, 1), "unit": "timesteps/s", "ms_per_timestep": round(dt * 1e3, 4),
            "steps_timed": steps, "setup_seconds": round(t_setup, 2),
            "residual_rms_nm": round(float(np.mean(closed)), 1), "open_loop_rms_nm": round(float(np.mean(opn)), 1),
            "what": "layers + mirror GEMM + sensor (1 frame) + slopes + reconstructor GEMM + integrator, "
                    "one HIP graph replay per timestep",
            "roofline": {"kernel": "whole timestep (sensor flops at one frame per launch)", "bound": "alu",
                         "achieved": round(ach, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(ach / FP32_PEAK_TFLOPS, 4), "flops_per_timestep": fl, "traffic": None}}


def sh_form(P, torch, dev, x, steps: int):
    """Shack-Hartmann sensor: the paper's SCAO SH shape (Table 2: 160 px, 20 x 20
    subapertures, 56 x 56 focal samples, 8 x 8 pixels each) over the 1000
    160 px frames, a MORFEO-LGS-like shape (68 x 68 subapertures of 7 px,
    240 x 240 samples, 16 x 16 pixels) over 100 frames (six LGS sensors per
    timestep), and the SCAO shape as a polychromatic sensor (Table 4) over
    three wavelengths.  Centre-of-gravity slopes; flops are those the kernel executes
    (two complex products per subaperture, |F|^2)."""
    import numpy as np
    from workloads import von_karman_opd

    def one(desc, opd, reps):
        sh = P.SH(desc, max_frames=int(opd.shape[0]), device=dev)
        sl = torch.empty((int(opd.shape[0]), 2, sh.n, sh.n), dtype=torch.float32, device=dev)
        sh.forward(opd, slopes=sl)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(reps):
            sh.forward(opd, slopes=sl)
        torch.cuda.synchronize(dev)
        dt = (time.perf_counter() - t0) / reps
        b, M = desc.n_pupil // desc.n_subap, desc.n_fft
        fl = (8.0 * b * b * M + 8.0 * b * M * M + 3.0 * M * M) * sh.n_valid
        return int(opd.shape[0]) / dt, fl, sh.n_valid

    fs1, fl1, nv1 = one(P.sh_desc(160, 20, 56, 7, 0.0, 750.0), x, steps)
    lgs = torch.from_numpy(von_karman_opd(100, 476, 38.5, 0.157, 25.0, seed=61)).to(dev)
    fs2, fl2, nv2 = one(P.sh_desc(476, 68, 240, 15, 0.28, 750.0), lgs, max(2, steps // 4))
    band = ([600.0, 750.0, 900.0], [1 / 3, 1 / 3, 1 / 3])
    fs3, fl3, _ = one(P.sh_desc(160, 20, 56, 7, 0.0, 600.0, lambdas_nm=band[0], lambda_weights=band[1]), x,
                      max(2, steps // 2))
    fl3 *= len(band[0])
    a1 = fl1 * fs1 / 1e12
    a2 = fl2 * fs2 / 1e12
    a3 = fl3 * fs3 / 1e12
    print(f"# shack-hartmann: SCAO {fs1:.0f} frames/s ({a1:.1f} TFLOP/s), LGS-like {fs2:.0f} frames/s "
          f"= {fs2 / 6:.0f} six-sensor timesteps/s ({a2:.1f} TFLOP/s), SCAO over 3 wavelengths "
          f"{fs3:.0f} frames/s ({a3:.1f} TFLOP/s)", file=sys.stderr, flush=True)
    return {"value": round(fs1, 1), "unit": "frames/s", "workload": "SCAO SH 160 px, 20x20 subap, 56x56, 8x8 px",
            "valid_subapertures": nv1,
            "roofline": {"kernel": "k_sh (per-subaperture focal DFT in LDS, |F|^2, binning, centroid)",
                         "bound": "alu", "achieved": round(a1, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(a1 / FP32_PEAK_TFLOPS, 4), "flops_per_frame": fl1, "traffic": None},
            "lgs_like": {"frames_per_s": round(fs2, 1), "six_sensor_timesteps_per_s": round(fs2 / 6, 1),
                         "workload": "68x68 subap of 7 px (476 px pupil), 240x240 focal samples, 16x16 px",
                         "valid_subapertures": nv2, "achieved_tflops": round(a2, 2),
                         "frac": round(a2 / FP32_PEAK_TFLOPS, 4), "flops_per_frame": fl2},
            "polychromatic": {"frames_per_s": round(fs3, 1),
                              "workload": "SCAO SH shape over 600/750/900 nm (equal weights, grid fixed at 600 nm)",
                              "achieved_tflops": round(a3, 2), "frac": round(a3 / FP32_PEAK_TFLOPS, 4),
                              "flops_per_frame": fl3}}


def hetero_form(P, torch, dev, stream, steps: int, graph_reps: int = 200):
    """Six sensors (80-240 px pupils, FFT 256-768, 16-96 points, 3 wavelengths)
    in one plan: autotuned execution, timesteps/s over the 500-frame batch, and
    the per-timestep latency of a HIP graph holding one timestep."""
    import numpy as np
    from paper_2602_06688_amd.autotune import autotune
    from workloads import workload, workload_opd
    w = workload("cfg4")
    F = w.n_frames
    opds = [workload_opd(w, i) for i in range(len(w.sensors))]
    x = torch.from_numpy(np.concatenate([o.reshape(F, -1) for o in opds], axis=1)).to(dev)
    plan = P.Plan(list(w.sensors), max_frames=F, device=dev, stream=stream)
    I = plan.new_intensity(F)
    S = plan.new_slopes(F)
    Fl = torch.zeros((F, len(w.sensors)), dtype=torch.float32, device=dev)
    tune = autotune(plan, lambda: plan.forward(x, I, stream=stream), F, reps=2)
    best_by_mode = {}
    for c in tune.get("tried", []):
        name = {P.MODE_LAUNCHES: "launches", P.MODE_PERSISTENT: "persistent"}.get(c["mode"], str(c["mode"]))
        best_by_mode[name] = round(min(best_by_mode.get(name, c["ms"]), c["ms"]), 3)
    path = sum(nominal_flops(s)["path"] for s in w.sensors)

    def timed():
        """Timesteps/s over ``steps`` steps, then the kernel durations of one
        more step with every launch timed (a run of its own: the events would
        slow the timed steps)."""
        plan.step(x, I, S, Fl, stream=stream)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.step(x, I, S, Fl, stream=stream)
        torch.cuda.synchronize(dev)
        dt = time.perf_counter() - t0
        plan.profile(1 << 16)
        plan.step(x, I, S, Fl, stream=stream)
        torch.cuda.synchronize(dev)
        kms = {k: plan.profile_read(k) for k in ("field", "rows", "cols", "slopes", "hetero")}
        plan.profile(0)
        gpu_ms = sum(v[0] for v in kms.values())
        return dt, kms, path * F / (gpu_ms / 1e3) / 1e12

    # the best persistent setting the tuner found, measured as a form of its
    # own (one persistent launch per pass for all six sensors), then the tuned one
    persistent = None
    pers = [c for c in tune.get("tried", []) if c["mode"] == P.MODE_PERSISTENT]
    if pers:
        pb = min(pers, key=lambda c: c["ms"])
        plan.set_tuning(**{k: pb[k] for k in ("mode", "chunk", "wg_per_cu", "row_groups")})
        for i, r in enumerate(pb.get("row_tiles", [])):
            plan.set_row_tile(i, r)
        pdt, pkms, pach = timed()
        persistent = {"value": round(F * steps / pdt, 2), "unit": "timesteps/s",
                      "tuning": {k: pb[k] for k in ("chunk", "wg_per_cu", "row_groups", "row_tiles") if k in pb},
                      "roofline_frac": round(pach / FP32_PEAK_TFLOPS, 4),
                      "kernel_ms_per_step": {k: round(v[0], 3) for k, v in pkms.items() if v[1]},
                      "launches_per_step": sum(v[1] for v in pkms.values())}
        plan.set_tuning(**{k: tune[k] for k in ("mode", "chunk", "wg_per_cu", "row_groups")})
        for i, r in enumerate(tune.get("row_tiles", [])):
            plan.set_row_tile(i, r)
    dt, kms, ach = timed()
    # one timestep (frame 0 of every sensor) captured in a graph, replayed
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream(device=dev)
    x1, I1, S1, F1 = x[:1], I[:1], S[:1], Fl[:1]
    with torch.cuda.stream(side):
        plan.step(x1, I1, S1, F1, stream=side)
    side.synchronize()
    ref = S1.clone()
    with torch.cuda.graph(g, stream=side):
        plan.step(x1, I1, S1, F1, stream=side)
    g.replay()
    torch.cuda.synchronize(dev)
    same = bool(torch.equal(S1, ref))
    t0 = time.perf_counter()
    for _ in range(graph_reps):
        g.replay()
    torch.cuda.synchronize(dev)
    lat = (time.perf_counter() - t0) / graph_reps * 1e3
    if persistent:
        print(f"# hetero persistent: {persistent['value']:.1f} timesteps/s, frac {persistent['roofline_frac']:.3f}",
              file=sys.stderr, flush=True)
    print(f"# hetero: {F * steps / dt:.1f} timesteps/s ({tune.get('mode')}, chunk {tune.get('chunk')}), "
          f"graph timestep {lat:.3f} ms", file=sys.stderr, flush=True)
    return {"value": round(F * steps / dt, 2), "unit": "timesteps/s",
            "workload": w.name, "frames": F, "ms_per_step": round(dt / steps * 1e3, 3),
            "tuning": {k: tune[k] for k in ("mode", "chunk", "wg_per_cu", "row_groups", "row_tiles") if k in tune},
            "best_ms_by_mode": best_by_mode,
            "persistent": persistent,
            "graph_timestep_ms": round(lat, 4), "graph_replay_matches_eager": same,
            "roofline": {"bound": "alu", "achieved": round(ach, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(ach / FP32_PEAK_TFLOPS, 4), "flops_per_timestep": path, "traffic": None,
                         "kernel_ms_per_step": {k: round(v[0], 3) for k, v in kms.items() if v[1]},
                         "launches_per_step": sum(v[1] for v in kms.values())}}


def measured_traffic(kernel: str, frames_per_launch: float):
    """HBM bytes per launch from the committed counter summary, or None when
    the kernel sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)[kernel]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for p in rec["sources"]:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sha256"]:
        return None
    return rec["hbm_bytes_per_frame"] * frames_per_launch


_ORACLE = {}


def _oracle_init(s, ref):
    _ORACLE["s"], _ORACLE["ref"] = s, ref


def _oracle_frame(opd):
    """One frame through the oracle: (the four pupil images [4][D][D], slopes
    [2][n][n], flux), float64."""
    import numpy as np
    from oracle import pwfs as O
    s = _ORACLE["s"]
    I = O.forward(opd[None], s)
    sl, fl = O.slopes(I, s, ref=_ORACLE["ref"])
    D = s.n_pupil
    win = np.stack([I[0, r:r + D, c:c + D] for r, c in O.image_origins(s)])
    return win, sl[0], float(fl[0])


def cpu_baseline(s, opd, n_frames: int, cores: int):
    """The FP64 oracle on the host cores, frames split over a process pool;
    the reference slopes (a flat wavefront through the same oracle) are
    computed once, as a plan does.  Returns the baseline record and the
    oracle's results on those frames (the reference of every form's error)."""
    import multiprocessing as mp
    import numpy as np
    from oracle import pwfs as O
    ref = O.reference_slopes(s)
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores, initializer=_oracle_init, initargs=(s, ref)) as pool:
        pool.map(_oracle_frame, [opd[i] for i in range(min(cores, n_frames))])   # warm the workers
        t0 = time.perf_counter()
        res = pool.map(_oracle_frame, [opd[i] for i in range(n_frames)], chunksize=1)
        dt = time.perf_counter() - t0
    refs = {"windows": np.stack([r[0] for r in res]), "slopes": np.stack([r[1] for r in res]),
            "flux": np.array([r[2] for r in res]), "valid": O.valid_subapertures(s)}
    rec = {"value": n_frames / dt, "unit": "frames/s", "cores": cores, "kind": "oracle",
           "sample": f"{n_frames} of the {opd.shape[0]} frames, forward+slopes in complex128 numpy "
                     f"(reference slopes computed once), {cores} worker processes, {dt:.1f} s wall"}
    return rec, refs


def oracle_errors(torch, I, S, s, refs) -> dict:
    """Errors of a form's outputs (device intensity [F][N][N], slopes
    [F][2][n][n]) against the oracle on the oracle's frames: per-frame
    normwise intensity (worst frame), every pixel against (|I_ref| + frame
    mean) (worst), pooled slope RMS, every valid subaperture against
    (|s_ref| + frame RMS) (worst)."""
    import numpy as np
    from oracle import pwfs as O
    F = refs["windows"].shape[0]
    D = s.n_pupil
    Ih = I[:F].cpu().numpy()
    a = np.stack([Ih[:, r:r + D, c:c + D] for r, c in O.image_origins(s)], axis=1).reshape(F, -1).astype(np.float64)
    b = refs["windows"].reshape(F, -1)
    v = refs["valid"]
    sa = S[:F].cpu().numpy().astype(np.float64)[:, :, v].reshape(F, -1)
    sb = refs["slopes"][:, :, v].reshape(F, -1)
    rms = np.sqrt((sb ** 2).mean(axis=1, keepdims=True))
    return {"frames": F,
            "intensity_normwise_max": float((np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)).max()),
            "intensity_pixel_max": float((np.abs(a - b) / (np.abs(b) + np.abs(b).mean(axis=1, keepdims=True))).max()),
            "slope_rel_rms": float(np.linalg.norm(sa - sb) / np.linalg.norm(sb)),
            "slope_subap_max": float((np.abs(sa - sb) / (np.abs(sb) + rms)).max())}


def graph_replays(torch, dev, fn, reps: int):
    """Captures fn(stream) once as a HIP graph and replays it `reps` times,
    with events around each replay on the replay stream.  Returns (wall
    seconds over all replays between two device synchronisations, per-replay
    ms from the events)."""
    side = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(side):
        fn(side)                      # warm on the capture stream
    side.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        fn(side)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    with torch.cuda.stream(side):
        g.replay()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    with torch.cuda.stream(side):
        for a, b in ev:
            a.record(side)
            g.replay()
            b.record(side)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in ev]
    del g
    return wall, ms


def host_info(torch, dev) -> dict:
    """Hardware and software the numbers were taken on."""
    cpu = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    rocm = None
    for path in ("/opt/rocm/.info/version", "/opt/rocm/.info/version-dev"):
        try:
            with open(path) as f:
                rocm = f.read().strip()
                break
        except OSError:
            pass
    props = torch.cuda.get_device_properties(dev)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": cpu, "cpu_logical": os.cpu_count(), "cpu_available": avail,
            "gpu": torch.cuda.get_device_name(dev), "gpu_arch": getattr(props, "gcnArchName", None),
            "compute_units": props.multi_processor_count, "rocm": rocm, "hip_runtime": torch.version.hip,
            "torch": torch.__version__}


def small_sensor_forms(P, torch, dev, stream, reps: int) -> dict:
    """The 64 px sensor (N=128, 16 points, 16 x 16, 100 frames): the plain
    FP32 path and its precision forms (bf16 x3, fp16 x3, bf16, fp16) on the same
    shapes and inputs.  frames/s from the median of graph replays of the
    100-frame batch, errors against the oracle on all 100 frames, kernel
    durations from HIP events over eager steps."""
    import numpy as np
    from oracle import pwfs as O
    from workloads import PREC_BF16, PREC_BF16X3, PREC_FP16, PREC_FP16X3, workload, workload_opd
    w = workload("cfg1")
    s = w.sensors[0]
    F = w.n_frames
    opd = workload_opd(w)
    t0 = time.perf_counter()
    I_ref = O.forward(opd, s)
    s_ref, f_ref = O.slopes(I_ref, s)
    D = s.n_pupil
    refs = {"windows": np.stack([I_ref[:, r:r + D, c:c + D] for r, c in O.image_origins(s)], axis=1),
            "slopes": s_ref, "flux": f_ref, "valid": O.valid_subapertures(s)}
    t_oracle = time.perf_counter() - t0
    x = torch.from_numpy(opd).to(dev)
    out = {"workload": w.name, "frames_per_batch": F, "oracle_seconds_single_process": round(t_oracle, 2)}
    for label, prec in (("fp32", 0), ("fp32_fused", 0), ("mfma_bf16x3", PREC_BF16X3),
                        ("mfma_fp16x3", PREC_FP16X3), ("mfma_bf16", PREC_BF16), ("mfma_fp16", PREC_FP16)):
        sp = s.with_(precision=prec)
        plan = P.Plan([sp], max_frames=F, device=dev, stream=stream)
        if label == "fp32_fused":
            plan.set_tuning(mode=P.MODE_FUSED)
        I = plan.new_intensity(F)
        S = plan.new_slopes(F)
        Fl = torch.zeros((F, 1), dtype=torch.float32, device=dev)
        wall, ms = graph_replays(torch, dev, lambda st: plan.step(x, I, S, Fl, stream=st), reps)
        med = float(np.median(ms))
        err = oracle_errors(torch, I, S, sp, refs)
        # kernel durations over eager steps
        plan.profile(4096)
        for _ in range(reps):
            plan.step(x, I, S, Fl, stream=stream)
        torch.cuda.synchronize(dev)
        kern = {k: plan.profile_read(k) for k in ("field", "rows", "cols", "fused", "mfma", "slopes")}
        plan.profile(0)
        rec = {"value": round(F / (med / 1e3), 1), "unit": "frames/s", "median_batch_ms": round(med, 4),
               "replays": reps, "mean_batch_ms": round(wall / reps * 1e3, 4), "errors_vs_oracle": err,
               "kernel_ms_per_batch": {k: round(v[0] / reps, 4) for k, v in kern.items() if v[1]}}
        if label == "fp32_fused":
            fl = nominal_flops(sp)
            fms, fn = kern["fused"]
            ach = fl["path"] * F * reps / (fms / 1e3) / 1e12 if fms > 0 else None
            rec["roofline"] = {"kernel": "k_fused (field, rows, columns, |e|^2 of one frame per workgroup)",
                               "bound": "alu", "achieved": round(ach, 2) if ach else None, "peak": FP32_PEAK_TFLOPS,
                               "unit": "TFLOP/s", "frac": round(ach / FP32_PEAK_TFLOPS, 4) if ach else None,
                               "flops_per_frame": fl["path"], "avg_launch_ms": round(fms / max(1, fn), 4),
                               "traffic": measured_traffic("k_fused", F),
                               "traffic_unit": "bytes per 100-frame launch (HBM, copy-calibrated rocprofv3 "
                                               "FETCH_SIZE/WRITE_SIZE)",
                               "algorithmic_bytes": 4.0 * F * (sp.n_pupil ** 2 + 4 * sp.n_pupil ** 2)}
        elif prec == 0:
            fl = nominal_flops(sp)
            cms, cn = kern["cols"]
            fpl = F * reps / max(1, cn)
            ach = fl["cols"] * fpl / (cms / max(1, cn) / 1e3) / 1e12 if cms > 0 else None
            rec["roofline"] = {"kernel": "k_cols (column pass)", "bound": "alu", "achieved": round(ach, 2),
                               "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / FP32_PEAK_TFLOPS, 4),
                               "flops_per_frame": fl["cols"], "frames_per_launch": fpl,
                               "avg_launch_ms": round(cms / max(1, cn), 4), "traffic": None}
            gpu_ms = sum(v[0] for v in kern.values()) / reps
            rec["roofline_path"] = {"achieved": round(fl["path"] * F / (gpu_ms / 1e3) / 1e12, 2),
                                    "frac": round(fl["path"] * F / (gpu_ms / 1e3) / 1e12 / FP32_PEAK_TFLOPS, 4),
                                    "flops_per_frame": fl["path"], "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s"}
        else:
            terms = 1 if prec in (PREC_BF16, PREC_FP16) else 3
            fl = mfma_flops(sp, terms)
            g2, n2 = kern["mfma"]
            fpl = F * reps / max(1, n2)
            ach = fl["stage2"] * fpl / (g2 / max(1, n2) / 1e3) / 1e12 if g2 > 0 else None
            rec["roofline"] = {"kernel": "k_mfma_cols_ws (stage 2)", "bound": "mfma",
                               "achieved": round(ach, 2) if ach else None, "peak": MFMA_PEAK_TFLOPS["bf16"],
                               "unit": "TFLOP/s", "frac": round(ach / MFMA_PEAK_TFLOPS["bf16"], 4) if ach else None,
                               "flops_per_frame": fl["stage2"], "traffic": None}
            rec["at_stated_error"] = err["slope_rel_rms"] <= 1e-3
        out[label] = rec
        plan.close()
        print(f"# 64 px {label}: {rec['value']:.0f} frames/s (median of {reps} replays of {F} frames), "
              f"slope err vs oracle {err['slope_rel_rms']:.2e}", file=sys.stderr, flush=True)
    base = out["fp32"]["value"]
    for label in ("fp32_fused", "mfma_bf16x3", "mfma_fp16x3", "mfma_bf16", "mfma_fp16"):
        out[label]["vs_fp32_plain"] = round(out[label]["value"] / base, 3)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-frames", type=int, default=192,
                    help="frames of the oracle CPU baseline (about 10 s on 16 host processes)")
    ap.add_argument("--no-forms", action="store_true", help="time only the plain FP32 path")
    ap.add_argument("--no-small", action="store_true", help="skip the 64 px sensor and its precision forms")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-surrogate form")
    ap.add_argument("--no-detector", action="store_true", help="skip the path with the detector stage")
    ap.add_argument("--no-loop", action="store_true", help="skip the closed AO loop")
    ap.add_argument("--no-sh", action="store_true", help="skip the Shack-Hartmann sensor")
    ap.add_argument("--no-hetero", action="store_true", help="skip the heterogeneous six-sensor batch")
    ap.add_argument("--no-poly", action="store_true", help="skip the 16-wavelength sensor")
    ap.add_argument("--no-soul", action="store_true", help="skip the SOUL pyramid + detector chain")
    ap.add_argument("--no-roof", action="store_true", help="skip the double-roof sensor")
    ap.add_argument("--surrogate-train", type=int, default=200_000)
    ap.add_argument("--surrogate-epochs", type=int, default=20)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed region, run one plain device copy of this many MiB "
                         "(calibrates the HBM byte counters of a profiler run)")
    ap.add_argument("--surrogate-study", action="store_true",
                    help="instead of the benchmark: the surrogate's error against training samples, width and "
                         "epochs (prints one JSON line)")
    args = ap.parse_args()
    if args.surrogate_study:
        import torch
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        cfgs = [(200_000, 1024, 20), (800_000, 1024, 20), (1_600_000, 1024, 20), (200_000, 2048, 20),
                (1_600_000, 2048, 20), (1_600_000, 1024, 60)]
        print(json.dumps({"surrogate_study": surrogate_study(torch, dev, 1_600_000, 20_000, cfgs)}), flush=True)
        return 0
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the sensor path is measured at its single-GPU shape "
              "(sharding over GPUs is described in DESIGN.md, not run).", file=sys.stderr)
        return 2

    import numpy as np
    from workloads import workload, workload_opd

    w = workload("cfg2")
    s = w.sensors[0]
    t0 = time.perf_counter()
    opd = workload_opd(w)
    print(f"# inputs: {w.n_frames} frames generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)

    cpu, refs = None, None
    if not args.no_cpu:
        cores = max(1, min(16, os.cpu_count() or 1))
        cpu, refs = cpu_baseline(s, opd, args.cpu_frames, cores)
        print(f"# cpu baseline: {cpu['value']:.2f} frames/s on {cores} processes", file=sys.stderr, flush=True)

    import torch
    from paper_2602_06688_amd import pwfs as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    plan = P.Plan([s], max_frames=w.n_frames, device=dev, stream=stream)
    x = torch.from_numpy(opd).to(dev)
    I = plan.new_intensity(w.n_frames)
    S = plan.new_slopes(w.n_frames)
    Fl = torch.zeros((w.n_frames, 1), dtype=torch.float32, device=dev)

    for _ in range(args.warmup):
        plan.step(x, I, S, Fl, stream=stream)
    torch.cuda.synchronize(dev)
    # the timed region: K replays of the step captured as a HIP graph
    dt, replay_ms = graph_replays(torch, dev, lambda st: plan.step(x, I, S, Fl, stream=st), args.steps)
    median_ms = float(np.median(replay_ms))
    # kernel durations: HIP events around every launch of K eager steps, on the launch stream
    plan.profile(4096)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.step(x, I, S, Fl, stream=stream)
    torch.cuda.synchronize(dev)
    eager_dt = time.perf_counter() - t0
    kern = {k: plan.profile_read(k) for k in ("field", "rows", "cols", "slopes")}
    plan.profile(0)
    fp32_err = oracle_errors(torch, I, S, s, refs) if refs is not None else None
    if fp32_err:
        print(f"# fp32 vs oracle: {fp32_err}", file=sys.stderr, flush=True)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize(dev)
        dst.copy_(src)
        torch.cuda.synchronize(dev)
        del src, dst

    # per-timestep latency: one frame's forward + slopes captured in a HIP graph
    lat_plan = P.Plan([s], max_frames=1, device=dev, stream=stream)
    x1 = x[:1]
    I1 = lat_plan.new_intensity(1)
    S1 = lat_plan.new_slopes(1)
    F1 = torch.zeros((1, 1), dtype=torch.float32, device=dev)
    lat_wall, lat_ms = graph_replays(torch, dev, lambda st: lat_plan.step(x1, I1, S1, F1, stream=st), 200)
    graph_ok = bool(torch.equal(S1, S[:1]))
    graph_ms = float(np.median(lat_ms))

    forms = {}
    if not args.no_forms:
        from workloads import PREC_BF16, PREC_BF16X3, PREC_FP16, PREC_FP16X3
        for label, prec, terms, dt_name in (("mfma_bf16x3", PREC_BF16X3, 3, "bf16"),
                                            ("mfma_fp16x3", PREC_FP16X3, 3, "fp16"),
                                            ("mfma_bf16", PREC_BF16, 1, "bf16"),
                                            ("mfma_fp16", PREC_FP16, 1, "fp16")):
            forms[label] = time_form(P, torch, s.with_(precision=prec), x, w.n_frames, max(20, args.steps // 2),
                                     1, I, S, dev, stream, label, terms, dt_name, refs)
    if not args.no_small:
        forms["pwfs64"] = small_sensor_forms(P, torch, dev, stream, max(20, args.steps))
    if not args.no_detector:
        forms["detector"] = detector_form(P, torch, dev, stream, x, plan, I, s, max(2, args.steps // 2))
    if not args.no_surrogate:
        forms["surrogate"] = surrogate_form(torch, dev, args.surrogate_train, 20_000, args.surrogate_epochs, 5)
    if not args.no_sh:
        forms["shack_hartmann"] = sh_form(P, torch, dev, x, max(2, args.steps // 2))
    if not args.no_roof:
        forms["double_roof"] = roof_form(P, torch, dev, x, s, max(2, args.steps // 4))
    if not args.no_soul:
        forms["soul_chain"] = soul_form(P, torch, dev, stream, max(2, args.steps // 4))
    if not args.no_poly:
        forms["polychromatic16"] = poly_form(P, torch, dev, x, s, max(2, args.steps // 4))
    if not args.no_loop:
        forms["closed_loop"] = loop_form(torch, dev)
    if not args.no_hetero:
        forms["hetero6_poly3"] = hetero_form(P, torch, dev, stream, max(2, args.steps // 5))

    frames = w.n_frames * args.steps
    value = frames / dt
    flops = nominal_flops(s)
    host = host_info(torch, dev)
    cols_ms, cols_n = kern["cols"]
    frames_per_launch = w.n_frames * args.steps / max(1, cols_n)
    achieved = flops["cols"] * frames_per_launch / (cols_ms / max(1, cols_n) / 1e3) / 1e12
    gpu_ms = sum(v[0] for v in kern.values())
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "median_step_ms": round(median_ms, 4),
        "timing": f"{args.steps} replays of the 1000-frame step captured as one HIP graph, between two device "
                  f"synchronisations (value); median of per-replay events {median_ms:.3f} ms; kernel durations "
                  f"from HIP events around every launch of {args.steps} eager steps "
                  f"({eager_dt / args.steps * 1e3:.3f} ms per step)",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic von Karman screens (r0 0.12 m, L0 40 m) + 5 mas tip/tilt jitter, seeds 2/12",
        "errors_vs_oracle": fp32_err,
        "host": host,
        "config": {"workload": w.name, "frames_per_step": w.n_frames, "n_pupil": s.n_pupil, "n_fft": s.n_fft,
                   "n_mod": s.n_mod, "n_subap": s.n_subap, "obstruction": s.obstruction,
                   "lambda_nm": s.lambdas_nm[0], "precision": "fp32", "intensity": "pupil-image windows"},
        "roofline": {
            "kernel": "k_cols (column pass: column FFT, mask, column IFFT, |e|^2 accumulate)",
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
            "traffic": measured_traffic("k_cols", frames_per_launch),
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
            "launches": cols_n,
            "avg_launch_ms": round(cols_ms / max(1, cols_n), 4),
            "frames_per_launch": frames_per_launch,
            "flops_per_frame": flops["cols"],
        },
        "roofline_path": {
            "achieved": round(flops["path"] * frames / (gpu_ms / 1e3) / 1e12, 3),
            "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(flops["path"] * frames / (gpu_ms / 1e3) / 1e12 / FP32_PEAK_TFLOPS, 4),
            "flops_per_frame": flops["path"],
            "kernel_ms": {k: round(v[0], 3) for k, v in kern.items()},
        },
        "graph_timestep": {"ms": round(graph_ms, 4), "frames_per_s": round(1e3 / graph_ms, 1),
                           "replay_matches_batched": graph_ok,
                           "what": "one frame (forward + slopes) per HIP graph replay, median of 200"},
        "forms": forms,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
