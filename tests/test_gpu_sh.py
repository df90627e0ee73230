"""Shack-Hartmann sensor on the GPU (pwfs_sh_*) against the oracle
(oracle/sh.py): detector pixels and centre-of-gravity slopes element by
element on small sensors covering every way the kernel shares a pixel
between threads, the paper's SCAO SH shape (Table 2: 160 px, 20 x 20
subapertures, 56 x 56 focal samples) on sampled frames of a full 1000-frame
launch, and a MORFEO-LGS-like shape (68 x 68 subapertures of 7 px, 240 x 240
focal samples) on one frame."""

import numpy as np
import pytest

from oracle import sh as SH
from workloads import von_karman_opd, workload, workload_opd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _P():
    from paper_2602_06688_amd import pwfs as P
    return P


def _compare(D, n, M, r, ob, opd, label, frames=None):
    P = _P()
    F = opd.shape[0]
    print(f"[gpu] sh {label}: D={D} n={n} M={M} rebin={r} F={F}", flush=True)
    sh = P.SH(P.sh_desc(D, n, M, r, ob, 750.0), max_frames=F)
    x = torch.from_numpy(np.ascontiguousarray(opd, np.float32)).cuda()
    sl, pix = sh.forward(x, want_pixels=True)
    torch.cuda.synchronize()
    idx = list(range(F)) if frames is None else frames
    want_pix, want_sl = SH.forward(opd[idx].astype(np.float32).astype(np.float64), D, n, M, r, ob, 750.0)
    gp = pix.cpu().numpy()[idx]
    gs = sl.cpu().numpy()[idx]
    valid = SH.valid_subapertures(D, n, ob)
    assert (gp[:, ~valid] == 0).all()              # invalid subapertures: zero pixels (and slopes)
    pe = np.abs(gp[:, valid] - want_pix[:, valid]).max() / np.abs(want_pix[:, valid]).max()
    se = np.abs(gs - want_sl).max()
    print(f"      pixels max rel {pe:.2e}, slopes max abs {se:.2e} px, valid {sh.n_valid}", flush=True)
    assert pe < 1e-5
    assert se < 1e-5
    assert sh.n_valid == SH.valid_subapertures(D, n, ob).sum()
    return sh, sl, pix


@pytest.mark.parametrize("D,n,M,r,ob", [
    (32, 4, 24, 3, 0.2),     # 8 pixels across, 4 threads per pixel
    (24, 3, 21, 3, 0.0),     # odd sample count, 7 pixels across
    (32, 4, 64, 2, 0.0),     # 32 pixels across: more pixels than threads
    (28, 4, 60, 15, 0.1),    # b = 7, 4 pixels across of 15 x 15 samples each
    (16, 2, 8, 1, 0.0),      # one sample per pixel
    (32, 8, 16, 2, 0.0),     # b = 4
    (20, 4, 20, 4, 0.0),     # b = 5: run-time width
    (64, 4, 48, 4, 0.1),     # b = 16
    (16, 2, 48, 4, 0.0),     # b = 8, one thread per pixel: four focal columns per register group
    (16, 2, 60, 5, 0.1),     # b = 8, 5 columns: a group of four and one with a single live column
    (16, 4, 64, 4, 0.0),     # b = 4, four columns per register group
])
def test_small_sensors_match_oracle(D, n, M, r, ob):
    rng = np.random.default_rng(D * M + r)
    opd = von_karman_opd(3, D, 2.0, 0.3, 25.0, seed=int(rng.integers(1000)))
    _compare(D, n, M, r, ob, opd, "small")


def test_flat_wavefront_zero_slopes():
    P = _P()
    sh = P.SH(P.sh_desc(40, 5, 32, 4, 0.3), max_frames=2)
    sl, _ = sh.forward(torch.zeros((2, 40, 40), device="cuda"))
    assert float(sl.abs().max()) < 1e-5


def test_scao_shape_full_launch_sampled_frames():
    w = workload("cfg2")
    opd = workload_opd(w)                    # 1000 frames of 160 px screens
    _compare(160, 20, 56, 7, 0.0, opd, "SCAO 1000 frames", frames=[0, 517, 999])


def test_morfeo_lgs_like_shape():
    opd = von_karman_opd(1, 476, 38.5, 0.157, 25.0, seed=61)
    _compare(476, 68, 240, 15, 0.28, opd, "LGS-like 68x68 / 240")


def test_errors():
    P = _P()
    sh = P.SH(P.sh_desc(160, 20, 56, 7), max_frames=2)
    with pytest.raises(P.PwfsError) as e:
        sh.forward(torch.zeros((3, 160, 160), device="cuda"))
    assert e.value.code == P.PWFS_ESTATE


# ------------------------------------------------- polychromatic sensor ----

def _compare_poly(D, n, M, r, ob, lam_ref, lams, ws, opd, label, frames=None):
    P = _P()
    F = opd.shape[0]
    print(f"[gpu] sh poly {label}: D={D} n={n} M={M} rebin={r} lambdas={lams} F={F}", flush=True)
    sh = P.SH(P.sh_desc(D, n, M, r, ob, lam_ref, lambdas_nm=lams, lambda_weights=ws), max_frames=F)
    x = torch.from_numpy(np.ascontiguousarray(opd, np.float32)).cuda()
    sl, pix = sh.forward(x, want_pixels=True)
    torch.cuda.synchronize()
    idx = list(range(F)) if frames is None else frames
    want_pix, want_sl = SH.forward_poly(opd[idx].astype(np.float32).astype(np.float64), D, n, M, r, ob, lam_ref,
                                        lams, ws)
    gp = pix.cpu().numpy()[idx]
    gs = sl.cpu().numpy()[idx]
    valid = SH.valid_subapertures(D, n, ob)
    assert (gp[:, ~valid] == 0).all()
    pe = np.abs(gp[:, valid] - want_pix[:, valid]).max() / np.abs(want_pix[:, valid]).max()
    se = np.abs(gs - want_sl).max()
    print(f"      pixels max rel {pe:.2e}, slopes max abs {se:.2e} px", flush=True)
    assert pe < 1e-5
    assert se < 1e-5
    return sl, pix


@pytest.mark.parametrize("D,n,M,r,ob", [
    (40, 5, 32, 4, 0.3),     # b = 8
    (28, 4, 60, 15, 0.1),    # b = 7, 15 x 15 samples per pixel
    (20, 4, 20, 4, 0.0),     # b = 5: run-time width
    (16, 2, 60, 5, 0.1),     # b = 8, four focal columns per register group and a ragged one
])
def test_polychromatic_small_sensors_match_oracle(D, n, M, r, ob):
    """Three wavelengths (600, 750, 900 nm; the grid fixed at 600 nm) against
    the oracle's weighted sum of scaled-frequency transforms."""
    opd = von_karman_opd(2, D, 2.0, 0.3, 25.0, seed=D + M)
    _compare_poly(D, n, M, r, ob, 600.0, [600.0, 750.0, 900.0], [0.25, 0.25, 0.5], opd, "small")


def test_polychromatic_every_wavelength_above_the_reference():
    """No sampled wavelength at the reference (every table scaled, s < 1),
    one of them with zero weight, and a run-time subaperture width (b = 5)."""
    opd = von_karman_opd(2, 30, 2.0, 0.3, 25.0, seed=77)
    _compare_poly(30, 6, 24, 3, 0.2, 500.0, [550.0, 700.0, 850.0, 1000.0], [0.4, 0.0, 0.35, 0.25], opd,
                  "all scaled")


def test_polychromatic_scao_shape_sampled_frames():
    """The SCAO SH shape over the 600-900 nm band (the heterogeneous pyramid
    batch's band) on sampled frames of a 200-frame launch."""
    w = workload("cfg2")
    opd = workload_opd(w, frames=range(200))
    _compare_poly(160, 20, 56, 7, 0.0, 600.0, [600.0, 750.0, 900.0], [1 / 3, 1 / 3, 1 / 3], opd, "SCAO band",
                  frames=[0, 199])


def test_polychromatic_split_reference_line_is_the_monochromatic_sensor():
    """Two halves of weight at the reference wavelength: each pass adds
    0.5 x (the monochromatic value), exactly, so pixels and slopes are the
    monochromatic sensor's bits."""
    P = _P()
    opd = von_karman_opd(2, 40, 2.0, 0.3, 25.0, seed=9)
    x = torch.from_numpy(np.ascontiguousarray(opd, np.float32)).cuda()
    mono = P.SH(P.sh_desc(40, 5, 32, 4, 0.3, 750.0), max_frames=2)
    poly = P.SH(P.sh_desc(40, 5, 32, 4, 0.3, 750.0, lambdas_nm=[750.0, 750.0], lambda_weights=[0.5, 0.5]),
                max_frames=2)
    s0, p0 = mono.forward(x, want_pixels=True)
    s1, p1 = poly.forward(x, want_pixels=True)
    torch.cuda.synchronize()
    assert torch.equal(p0, p1) and torch.equal(s0, s1)
