"""FP64 CPU oracle of the Shack-Hartmann wavefront sensor.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import or call
this module: only the tests do.  It shares no code with the HIP library.

The paper lists Shack-Hartmann sensors among its processing objects (Table 4:
``SH``, ``DistributedSH``) and sizes their FFT workload in Table 2 (e.g. the
SCAO SH: 160 px pupil, 20 x 20 subapertures, 314 of them valid, one 56 x 56
transform each).  It gives no equations; the textbook model, with the same
readings as the pyramid where they carry over, is:

  1. the pupil field A exp(i 2 pi OPD / lambda) is cut into n x n blocks of
     b x b pixels (b = D / n);
  2. each block is Fourier transformed onto an M x M focal grid at the
     half-integer frequencies (u - M/2 + 1/2) / M, so a flat wavefront puts
     the spot on the corner of the four central pixels (computed here as the
     FFT of the block zero-padded to M x M and tilted by half a pixel);
  3. the spot |F|^2 / (M^2 sum(A^2)) (all spots of a flat frame sum to 1) is
     binned rebin x rebin onto n_pix x n_pix detector pixels, M = n_pix rebin;
  4. slopes are the centre of gravity of each valid subaperture's pixels, in
     pixels from the subaperture centre (x: columns, y: rows); a subaperture
     is valid when at least half of its pupil pixels are illuminated.
"""

from __future__ import annotations

import numpy as np

from . import pwfs as O


def spots(opd_nm: np.ndarray, D: int, n: int, M: int, obstruction: float, lambda_nm: float) -> np.ndarray:
    """Focal-plane spots [F][n][n][M][M] (normalised) of OPD frames [F][D][D]."""
    opd = np.asarray(opd_nm, np.float64)
    if opd.ndim == 2:
        opd = opd[None]
    b = D // n
    A = O.pupil_amplitude(D, obstruction)
    sA2 = float((A * A).sum())
    s = -M / 2.0 + 0.5
    x = np.arange(b)
    tilt = np.exp(-2j * np.pi * s * (x[None, :] + x[:, None]) / M)
    out = np.zeros((opd.shape[0], n, n, M, M))
    for f in range(opd.shape[0]):
        E = A * np.exp(1j * 2.0 * np.pi * opd[f] / lambda_nm)
        for i in range(n):
            for j in range(n):
                pad = np.zeros((M, M), np.complex128)
                pad[:b, :b] = E[i * b:(i + 1) * b, j * b:(j + 1) * b] * tilt
                F = np.fft.fft2(pad)
                out[f, i, j] = (F.real ** 2 + F.imag ** 2) / (M * M * sA2)
    return out


def detector(sp: np.ndarray, rebin: int) -> np.ndarray:
    """Spots [..][M][M] binned to [..][M/rebin][M/rebin] pixels."""
    M = sp.shape[-1]
    k = M // rebin
    return sp.reshape(*sp.shape[:-2], k, rebin, k, rebin).sum(axis=(-3, -1))


def valid_subapertures(D: int, n: int, obstruction: float) -> np.ndarray:
    b = D // n
    A = O.pupil_amplitude(D, obstruction)
    return A.reshape(n, b, n, b).sum(axis=(1, 3)) / (b * b) >= 0.5


def centroids(pix: np.ndarray, valid: np.ndarray) -> np.ndarray:
    """Slopes [F][2][n][n]: centre of gravity of each subaperture's pixels in
    pixels from its centre (x along columns, y along rows); 0 where invalid
    or dark."""
    pix = np.asarray(pix, np.float64)
    k = pix.shape[-1]
    c = np.arange(k) - (k - 1) / 2.0
    tot = pix.sum(axis=(-2, -1))
    sx = (pix * c[None, :]).sum(axis=(-2, -1))
    sy = (pix * c[:, None]).sum(axis=(-2, -1))
    ok = valid[None] & (tot > 0)
    out = np.zeros((pix.shape[0], 2) + valid.shape)
    out[:, 0] = np.where(ok, sx / np.where(tot > 0, tot, 1.0), 0.0)
    out[:, 1] = np.where(ok, sy / np.where(tot > 0, tot, 1.0), 0.0)
    return out


def forward(opd_nm, D, n, M, rebin, obstruction, lambda_nm):
    """(detector pixels [F][n][n][M/rebin][M/rebin], slopes [F][2][n][n])."""
    pix = detector(spots(opd_nm, D, n, M, obstruction, lambda_nm), rebin)
    return pix, centroids(pix, valid_subapertures(D, n, obstruction))
