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


# ----------------------------------------------------------- polychromatic --
# The paper lists a polychromatic Shack-Hartmann sensor (Table 4,
# ``PolyChromSH``) without its equations.  Reading used here, the same as for
# the polychromatic pyramid (a weighted sum of monochromatic sensors over the
# sampled band):
#   * the focal samples are fixed in angle: n_fft of them span the field that
#     the pixelated pupil gives at the reference wavelength lambda_ref
#     (lambda_ref b / d), so at a wavelength lambda the block is transformed
#     at the frequencies (u - M/2 + 1/2) s / M cycles per pupil pixel,
#     s = lambda_ref / lambda (s = 1: the monochromatic sensor);
#   * lambda_ref may not exceed any sampled wavelength (s <= 1), so that the
#     grid never reaches past one period of the pixel-sampled spectrum;
#   * a sample stands for a fixed solid angle, so the intensity of wavelength
#     lambda carries the factor s^2: |F|^2 s^2 / (M^2 sum A^2) (a flat frame's
#     spots then hold the fraction of the light that falls on the grid);
#   * the spot image is sum_lambda w_lambda spot_lambda.
# A non-integer frequency scale has no FFT, so each block's transform is the
# two matrix products of the definition, F = W E W^T with
# W[u][x] = exp(-2 pi i (u - M/2 + 1/2)(x - (b-1)/2) s / M).

def dft_matrix(b: int, M: int, s: float) -> np.ndarray:
    """W [M][b] of the scaled half-integer-frequency transform."""
    f = (np.arange(M) - M / 2.0 + 0.5) * s / M
    c = np.arange(b) - (b - 1) / 2.0
    return np.exp(-2j * np.pi * f[:, None] * c[None, :])


def spots_poly(opd_nm: np.ndarray, D: int, n: int, M: int, obstruction: float, lambda_ref_nm: float,
               lambdas_nm, weights) -> np.ndarray:
    """Polychromatic spots [F][n][n][M][M] of OPD frames [F][D][D]."""
    opd = np.asarray(opd_nm, np.float64)
    if opd.ndim == 2:
        opd = opd[None]
    b = D // n
    A = O.pupil_amplitude(D, obstruction)
    sA2 = float((A * A).sum())
    out = np.zeros((opd.shape[0], n, n, M, M))
    for lam, w in zip(lambdas_nm, weights):
        s = lambda_ref_nm / lam
        W = dft_matrix(b, M, s)
        for f in range(opd.shape[0]):
            E = A * np.exp(1j * 2.0 * np.pi * opd[f] / lam)
            for i in range(n):
                for j in range(n):
                    F = W @ E[i * b:(i + 1) * b, j * b:(j + 1) * b] @ W.T
                    out[f, i, j] += w * (F.real ** 2 + F.imag ** 2) * (s * s) / (M * M * sA2)
    return out


def forward_poly(opd_nm, D, n, M, rebin, obstruction, lambda_ref_nm, lambdas_nm, weights):
    """(detector pixels, slopes) of the polychromatic sensor."""
    pix = detector(spots_poly(opd_nm, D, n, M, obstruction, lambda_ref_nm, lambdas_nm, weights), rebin)
    return pix, centroids(pix, valid_subapertures(D, n, obstruction))
