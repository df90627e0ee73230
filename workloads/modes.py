"""Seeded inputs of the learned-surrogate workload: a Karhunen-Loeve-like
modal basis, modal-coefficient draws and the network's initial weights.

Modal basis: eigenvectors of the von Karman phase covariance
    C(r) ~ x^(5/6) K_5/6(x),  x = 2 pi r / L0   (the r-dependence of the
    von Karman phase covariance; its prefactor cancels in the rescaling below)
between the pupil pixels of a 4x-decimated grid, with piston projected out,
sorted by decreasing eigenvalue; each is upsampled (bilinear) to the full
pupil, made piston-free and the set is re-orthonormalised in order by QR
over the full pupil's pixels, with unit RMS over the pupil.  Coefficient
variances follow the eigenvalues, scaled so that the total phase variance is
(2 pi * residual_nm / lambda)^2 -- a closed-loop residual of 100 nm RMS at
750 nm in the surrogate workload.

None of this is the sensor's arithmetic: it only produces OPD inputs.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.ndimage import zoom
from scipy.special import gamma, kv


def _pupil(n: int, obstruction: float) -> np.ndarray:
    c = np.arange(n) - (n - 1) / 2.0
    r2 = c[None, :] ** 2 + c[:, None] ** 2
    R = n / 2.0
    return (r2 <= R * R) & (r2 >= (obstruction * R) ** 2)


def von_karman_shape(r: np.ndarray, L0: float) -> np.ndarray:
    x = 2.0 * math.pi * np.asarray(r, np.float64) / L0
    out = np.empty_like(x)
    small = x < 1e-12
    out[small] = 2.0 ** (-1.0 / 6.0) * gamma(5.0 / 6.0)
    xs = x[~small]
    out[~small] = xs ** (5.0 / 6.0) * kv(5.0 / 6.0, xs)
    return out


def kl_modes(n_pupil: int, obstruction: float, diameter_m: float, L0_m: float, n_modes: int,
             decimate: int = 4):
    """(modes [n_modes][n_pupil^2] float64, zero outside the pupil and unit
    RMS over it; eigenvalues [n_modes], decreasing)."""
    nd = n_pupil // decimate
    pd = _pupil(nd, obstruction)
    c = (np.arange(nd) - (nd - 1) / 2.0) * (diameter_m / nd)
    yy, xx = np.meshgrid(c, c, indexing="ij")
    pts = np.stack([xx[pd], yy[pd]], 1)
    if pts.shape[0] <= n_modes:
        raise ValueError("decimated pupil has too few pixels for the number of modes")
    r = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1))
    C = von_karman_shape(r, L0_m)
    n = C.shape[0]
    Pm = np.eye(n) - np.full((n, n), 1.0 / n)
    w, V = np.linalg.eigh(Pm @ C @ Pm)
    order = np.argsort(w)[::-1][:n_modes]
    w = w[order]
    V = V[:, order]
    full = _pupil(n_pupil, obstruction)
    M = np.zeros((n_modes, full.sum()))
    img = np.zeros((nd, nd))
    for j in range(n_modes):
        img[:] = 0.0
        img[pd] = V[:, j]
        up = zoom(img, decimate, order=1, mode="nearest", grid_mode=True)
        v = up[full]
        M[j] = v - v.mean()
    Q, R = np.linalg.qr(M.T)
    Q *= np.sign(np.diag(R))[None, :]
    Q *= math.sqrt(full.sum())            # unit RMS over the pupil
    modes = np.zeros((n_modes, n_pupil * n_pupil))
    modes[:, full.ravel()] = Q.T
    return modes, w


def coefficient_sigmas(eigenvalues: np.ndarray, residual_nm: float, lambda_nm: float) -> np.ndarray:
    """Per-mode coefficient RMS (rad), proportional to sqrt(eigenvalue), with
    sum of variances = (2 pi residual / lambda)^2."""
    total = (2.0 * math.pi * residual_nm / lambda_nm) ** 2
    var = np.maximum(eigenvalues, 0.0)
    var = var * (total / var.sum())
    return np.sqrt(var)


def draws(n: int, n_modes: int, seed: int, chunk: int = 4096) -> np.ndarray:
    """Standard-normal draws [n][n_modes] float32; chunk i seeded by (seed, i)."""
    out = np.empty((n, n_modes), np.float32)
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        out[i0:i1] = np.random.default_rng([int(seed), i0 // chunk]).standard_normal((i1 - i0, n_modes))
    return out


def init_params(sizes, seed: int, zero_last: bool = False) -> np.ndarray:
    """He-normal weights (std sqrt(2/fan_in)), zero biases, packed per layer
    as W [out][in] then b [out] (float32).  With ``zero_last`` the output
    layer's weights start at zero (the draws are still taken, so the hidden
    layers are the same either way): a network that learns a correction then
    starts from no correction."""
    rng = np.random.default_rng(seed)
    parts = []
    n_layers = len(sizes) - 1
    for l, (i, o) in enumerate(zip(sizes[:-1], sizes[1:])):
        w = rng.standard_normal((o, i)) * math.sqrt(2.0 / i)
        if zero_last and l == n_layers - 1:
            w[:] = 0.0
        parts.append(w.ravel())
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)
