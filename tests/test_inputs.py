"""Statistical and bookkeeping checks of the seeded input generators."""

import math

import numpy as np

from workloads import jitter_opd, tilt_opd, von_karman_opd, workload, workload_opd


def test_screens_reproducible_and_addressable():
    a = von_karman_opd(range(4), 32, 8.0, 0.15, 25.0, seed=1)
    b = von_karman_opd([2, 3], 32, 8.0, 0.15, 25.0, seed=1)
    assert a.dtype == np.float32 and a.shape == (4, 32, 32)
    assert np.array_equal(a[2:], b)
    assert not np.allclose(a[0], a[1])


def test_kolmogorov_structure_function():
    """For L0 >> separation the phase structure function approaches the
    Kolmogorov law 6.88 (r / r0)^(5/3) (Fried 1965).  Checked at a few pixel
    separations with a very large outer scale on a 128 m grid, within 15 %
    (FFT screens without subharmonics run ~10 % low at these separations)."""
    D, Dtel, r0 = 64, 8.0, 0.3
    opd = von_karman_opd(40, D, Dtel, r0, 1e4, seed=9, grid=1024)
    phi = opd.astype(np.float64) * 2 * math.pi / 500.0
    dx = Dtel / D
    for sep in (2, 4, 8):
        d = phi[:, :, sep:] - phi[:, :, :-sep]
        sf = (d ** 2).mean()
        th = 6.88 * (sep * dx / r0) ** (5.0 / 3.0)
        assert abs(sf / th - 1.0) < 0.15, (sep, sf, th)


def test_jitter_rms_and_tilt_units():
    D, Dtel = 64, 8.0
    j = jitter_opd(400, D, Dtel, 5.0, seed=12).astype(np.float64)
    c = np.arange(D) - (D - 1) / 2
    # least-squares tip per frame from the x-gradient
    tx = (j * c[None, None, :]).sum(axis=(1, 2)) / (D * (c ** 2).sum()) / (Dtel / D) * 1e-9
    rms_mas = tx.std() * 206264.80624709636e3
    assert abs(rms_mas / 5.0 - 1.0) < 0.12
    # 1 lambda/D of tilt is one wave of OPD across the D-pixel pupil
    t = tilt_opd(D, 1.0, 0.0, 750.0)
    assert abs((t[0, -1] - t[0, 0]) - 750.0 * (D - 1) / D) < 1e-9


def test_workload_shapes():
    w = workload("cfg2")
    o = workload_opd(w, frames=[0, 999])
    assert o.shape == (2, 160, 160) and o.dtype == np.float32
    w4 = workload("cfg4")
    assert [s.n_fft for s in w4.sensors] == [256, 384, 512, 512, 768, 768]


def test_kl_modes_orthonormal_ordered_and_scaled():
    from workloads.modes import coefficient_sigmas, kl_modes
    Z, ev = kl_modes(64, 0.12, 8.0, 25.0, 60)
    pup = Z[0] != 0
    m = Z[:, pup]
    G = m @ m.T / m.shape[1]
    assert np.abs(G - np.eye(60)).max() < 1e-10          # unit RMS, orthogonal
    assert np.abs(m.mean(axis=1)).max() < 1e-10          # piston-free
    assert (np.diff(ev) <= 1e-12).all()                  # decreasing variance
    s = coefficient_sigmas(ev, 100.0, 750.0)
    assert abs((s ** 2).sum() - (2 * math.pi * 100 / 750) ** 2) < 1e-12
    # tip and tilt dominate a von Karman spectrum: the first two modes are
    # (nearly) linear ramps
    c = np.arange(64) - 31.5
    ramp = np.broadcast_to(c[None, :], (64, 64)).ravel()[pup]
    ramp = ramp / np.sqrt((ramp ** 2).mean())
    proj = (m[:2] @ ramp / m.shape[1])
    assert np.hypot(*proj) > 0.95


def test_init_params_he_scale_and_zero_output_layer():
    from workloads.modes import init_params
    sizes = [500, 1024, 64]
    a = init_params(sizes, 3)
    b = init_params(sizes, 3, zero_last=True)
    n0 = 500 * 1024
    W0 = a[:n0]
    assert abs(W0.std() - math.sqrt(2.0 / 500)) < 0.01 * math.sqrt(2.0 / 500)
    assert np.array_equal(a[:n0 + 1024], b[:n0 + 1024])            # hidden layer unchanged
    last = b[n0 + 1024:n0 + 1024 + 1024 * 64]
    assert not last.any() and a[n0 + 1024:n0 + 1024 + 1024 * 64].any()
    assert a.size == b.size == n0 + 1024 + 1024 * 64 + 64
