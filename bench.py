"""Throughput of the pyramid-sensor path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

A step is one pass of the whole path (forward model + binning/slopes) over
the 1000-frame batch of the 160 px pupil / 512 px transform / 48-point
modulation / 40 x 40 subaperture workload, with the synthetic von Karman
inputs already resident in HBM.  Prints one JSON line.
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
FP32_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0}   # MI355X dense matrix peaks


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


def time_form(P, torch, s, x, n_frames, steps, warmup, ref_I, ref_S, dev, stream, label, terms, dtype):
    """frames/s of one precision form, its error against the FP32 path's
    outputs (ref_I, ref_S) on the same frames, and its matrix-core roofline."""
    plan = P.Plan([s], max_frames=n_frames, device=dev, stream=stream)
    I = plan.new_intensity(n_frames)
    S = plan.new_slopes(n_frames)
    Fl = torch.zeros((n_frames, 1), dtype=torch.float32, device=dev)
    for _ in range(warmup):
        plan.step(x, I, S, Fl, stream=stream)
    torch.cuda.synchronize(dev)
    plan.profile(4096)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.step(x, I, S, Fl, stream=stream)
    torch.cuda.synchronize(dev)
    dt = time.perf_counter() - t0
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
    out = {"value": round(frames / dt, 2), "unit": "frames/s", "ms_per_step": round(dt / steps * 1e3, 4),
           "intensity_rel_err_max_vs_fp32": ie, "slope_rel_rms_vs_fp32": se,
           "roofline": {"kernel": "k_mfma_cols (stage 2: e_k = Qy_k T, |e|^2 accumulate)", "bound": "mfma",
                        "achieved": round(ach, 2) if ach else None, "peak": peak, "unit": "TFLOP/s",
                        "frac": round(ach / peak, 4) if ach else None, "traffic": None,
                        "avg_launch_ms": round(g2_ms / max(1, g2_n), 4), "flops_per_frame": fl["stage2"]},
           "stage1_ms_per_step": round(g1_ms / steps, 3), "stage2_ms_per_step": round(g2_ms / steps, 3)}
    plan.close()
    print(f"# {label}: {out['value']:.0f} frames/s, intensity err {ie:.2e}, slope err {se:.2e}",
          file=sys.stderr, flush=True)
    return out


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


def _oracle_frame(args):
    import numpy as np
    from oracle import pwfs as O
    opd, s = args
    I = O.forward(opd[None], s)
    O.slopes(I, s)
    return 0


def cpu_baseline(s, opd, n_frames: int, cores: int) -> dict:
    """The FP64 oracle on the host cores, frames split over a process pool."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    sample = [(opd[i], s) for i in range(n_frames)]
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_frame, sample[:cores])          # warm the workers
        t0 = time.perf_counter()
        pool.map(_oracle_frame, sample, chunksize=1)
        dt = time.perf_counter() - t0
    return {"value": n_frames / dt, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_frames} of the 1000 frames, forward+slopes in complex128 numpy, "
                      f"{cores} worker processes, {dt:.1f} s wall"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-frames", type=int, default=32)
    ap.add_argument("--no-forms", action="store_true", help="time only the plain FP32 path")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed region, run one plain device copy of this many MiB "
                         "(calibrates the HBM byte counters of a profiler run)")
    args = ap.parse_args()
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

    cpu = None
    if not args.no_cpu:
        cores = max(1, min(16, os.cpu_count() or 1))
        cpu = cpu_baseline(s, opd, args.cpu_frames, cores)
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
    # per-kernel HIP events on the launch stream over the timed region
    plan.profile(4096)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.step(x, I, S, Fl, stream=stream)
    torch.cuda.synchronize(dev)
    dt = time.perf_counter() - t0
    kern = {k: plan.profile_read(k) for k in ("field", "rows", "cols", "slopes")}
    plan.profile(0)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize(dev)
        dst.copy_(src)
        torch.cuda.synchronize(dev)
        del src, dst

    forms = {}
    if not args.no_forms:
        from workloads import PREC_BF16, PREC_BF16X3, PREC_FP16X3
        for label, prec, terms, dt_name in (("mfma_bf16x3", PREC_BF16X3, 3, "bf16"),
                                            ("mfma_fp16x3", PREC_FP16X3, 3, "fp16"),
                                            ("mfma_bf16", PREC_BF16, 1, "bf16")):
            forms[label] = time_form(P, torch, s.with_(precision=prec), x, w.n_frames, max(2, args.steps // 2),
                                     1, I, S, dev, stream, label, terms, dt_name)

    frames = w.n_frames * args.steps
    value = frames / dt
    flops = nominal_flops(s)
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
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic von Karman screens (r0 0.12 m, L0 40 m) + 5 mas tip/tilt jitter, seeds 2/12",
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
        "forms": forms,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
