"""Seeded optical-path-difference inputs: von Karman screens, tip/tilt jitter.

Screens are drawn by FFT filtering of complex white Gaussian noise with the
von Karman phase spectrum

    Phi(f) = 0.0229 r0^(-5/3) (f^2 + L0^-2)^(-11/6)   [rad^2 m^2 at r0's wavelength]

on an M x M grid of pixel pitch D_tel / D_px, with the f = 0 term removed.
The real and the imaginary part of one filtered draw are two independent
screens, so frame 2p and 2p+1 come from the draw seeded by (seed, p); any
subset of frames is therefore reproducible on its own.  The central D_px^2
crop is converted to optical path in nm and stored as float32; that float32
array is the input both the oracle and the HIP path consume.

The paper's workloads are its own AO systems (Table 2); no public dataset is
involved, these synthetic screens stand in for its atmosphere objects.
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.fft

from .configs import Workload


def _grid_size(n_pupil: int, dx: float, L0_m: float) -> int:
    need = max(2 * n_pupil, int(math.ceil(L0_m / dx)))
    return 1 << (need - 1).bit_length()


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def von_karman_opd(frames, n_pupil: int, diameter_m: float, r0_m: float, L0_m: float,
                   seed: int, r0_lambda_nm: float = 500.0, grid: int | None = None) -> np.ndarray:
    """OPD screens in nm, float32 [len(frames)][n_pupil][n_pupil].

    ``frames`` is an int (0..n-1) or an iterable of frame indices.
    """
    if isinstance(frames, int):
        frames = range(frames)
    frames = list(frames)
    dx = diameter_m / n_pupil
    M = grid or _grid_size(n_pupil, dx, L0_m)
    f = np.fft.fftfreq(M, d=dx)
    f2 = f[None, :] ** 2 + f[:, None] ** 2
    psd = 0.0229 * r0_m ** (-5.0 / 3.0) * (f2 + L0_m ** -2) ** (-11.0 / 6.0)
    psd[0, 0] = 0.0
    amp = np.sqrt(psd) / (M * dx)            # sqrt(Phi) * df, df = 1 / (M dx)
    o = (M - n_pupil) // 2
    to_nm = r0_lambda_nm / (2.0 * math.pi)
    out = np.empty((len(frames), n_pupil, n_pupil), np.float32)

    def draw(pair):
        rng = np.random.default_rng([int(seed), pair])
        c = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
        scr = scipy.fft.ifft2(c * amp, workers=1) * (M * M)
        return scr[o:o + n_pupil, o:o + n_pupil].copy()

    pairs = sorted({int(fr) // 2 for fr in frames})
    with ThreadPoolExecutor(max_workers=_workers()) as ex:
        crops = dict(zip(pairs, ex.map(draw, pairs)))
    for i, fr in enumerate(frames):
        crop = crops[int(fr) // 2]
        out[i] = (crop.imag if int(fr) % 2 else crop.real) * to_nm
    return out


def periodic_layer(n: int, pixel_m: float, r0_m: float, L0_m: float, seed: int,
                   r0_lambda_nm: float = 500.0) -> np.ndarray:
    """One whole periodic von Karman OPD screen [n][n] in nm (float32): the
    real part of an n x n FFT screen with pixel size pixel_m (same spectrum
    and normalisation as von_karman_opd), for frozen-flow layers."""
    f = np.fft.fftfreq(n, d=pixel_m)
    f2 = f[None, :] ** 2 + f[:, None] ** 2
    psd = 0.0229 * r0_m ** (-5.0 / 3.0) * (f2 + L0_m ** -2) ** (-11.0 / 6.0)
    psd[0, 0] = 0.0
    amp = np.sqrt(psd) / (n * pixel_m)
    rng = np.random.default_rng([int(seed), 1 << 20])
    c = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    scr = scipy.fft.ifft2(c * amp, workers=_workers()) * (n * n)
    return (scr.real * (r0_lambda_nm / (2.0 * math.pi))).astype(np.float32)


def _centred(n_pupil: int) -> np.ndarray:
    return np.arange(n_pupil, dtype=np.float64) - (n_pupil - 1) / 2.0


def jitter_opd(frames, n_pupil: int, diameter_m: float, sigma_mas: float, seed: int) -> np.ndarray:
    """Per-frame Gaussian tip and tilt (sigma per axis, mas) as OPD in nm."""
    if isinstance(frames, int):
        frames = range(frames)
    frames = list(frames)
    sigma_rad = sigma_mas * 1e-3 / 206264.80624709636
    dx = diameter_m / n_pupil
    c = _centred(n_pupil) * dx                 # metres from the pupil centre
    out = np.empty((len(frames), n_pupil, n_pupil), np.float32)
    for i, fr in enumerate(frames):
        tx, ty = np.random.default_rng([int(seed), int(fr)]).standard_normal(2) * sigma_rad
        out[i] = (tx * c[None, :] + ty * c[:, None]) * 1e9
    return out


def tilt_opd(n_pupil: int, t_lod: float, theta: float = 0.0, lambda_nm: float = 750.0) -> np.ndarray:
    """A pure tilt of ``t_lod`` lambda/D (at ``lambda_nm``) along angle ``theta``.

    Column index is x, row index is y; the phase increases along
    (cos theta, sin theta).  Returns float64 [n_pupil][n_pupil] OPD in nm.
    """
    c = _centred(n_pupil)
    return lambda_nm * t_lod * (c[None, :] * math.cos(theta) + c[:, None] * math.sin(theta)) / n_pupil


def workload_opd(w: Workload, sensor: int = 0, frames=None) -> np.ndarray:
    """The OPD input of one sensor of a workload (screens plus jitter)."""
    s = w.sensors[sensor]
    if frames is None:
        frames = range(w.n_frames)
    frames = list(frames)
    opd = von_karman_opd(frames, s.n_pupil, s.diameter_m, w.r0_m, w.L0_m, w.seeds[sensor],
                         w.r0_lambda_nm)
    if w.jitter_mas > 0.0:
        opd += jitter_opd(frames, s.n_pupil, s.diameter_m, w.jitter_mas, w.jitter_seed)
    return opd
