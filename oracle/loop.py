"""FP64 CPU oracle of the closed adaptive-optics loop around the pyramid sensor.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import or call
this module: only the tests do.  It shares no code with the HIP library.

The loop is the chain of the SOUL configuration in the paper's Appendix B:
atmosphere (frozen-flow layers) -> propagation to the pupil, minus the
deformable mirror -> pyramid sensor -> slopes -> modal reconstructor
(``Modalrec``, a reconstruction matrix applied to the slopes) -> integrator
(``Integrator``: per-mode-group gains and forgetting factors, total delay of
two time steps) -> deformable mirror (``DM`` with modal influence functions),
closed through the delayed connection of Section 2.1.  The paper gives the
objects and their parameters, not their equations; the readings are:

  * layers: OPD(x, y, t) = sum_l w_l S_l(x + ox_l + vx_l t, y + oy_l + vy_l t),
    S_l periodic screens sampled bilinearly (pixel units, pupil pixel
    (x, y) at integer coordinates);
  * DM: OPD_dm = B c_applied, B the modal influence functions [pixels][modes];
  * reconstructor: m(t) = R s(t);
  * integrator: c(t) = ff * c(t-1) + g * m(t) (element-wise per mode);
  * delay: the mirror applies c(t - d) at step t (zero before the loop has
    produced it), d = 2 for the SOUL listing.
"""

from __future__ import annotations

import numpy as np

from . import pwfs as O


def bilinear_periodic(S: np.ndarray, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """S sampled at real pixel coordinates (X column, Y row), periodic."""
    n_r, n_c = S.shape
    x0 = np.floor(X)
    y0 = np.floor(Y)
    fx = X - x0
    fy = Y - y0
    i0 = np.mod(x0.astype(np.int64), n_c)
    j0 = np.mod(y0.astype(np.int64), n_r)
    i1 = np.mod(i0 + 1, n_c)
    j1 = np.mod(j0 + 1, n_r)
    S = np.asarray(S, np.float64)
    top = (1.0 - fx) * S[j0, i0] + fx * S[j0, i1]
    bot = (1.0 - fx) * S[j1, i0] + fx * S[j1, i1]
    return (1.0 - fy) * top + fy * bot


def layers_opd(screens: np.ndarray, weights, origins, velocities, t: int, D: int) -> np.ndarray:
    """OPD [D][D] at step t from layers: screens [L][n][n], weights [L],
    origins [L][2] (x, y) and velocities [L][2] (x, y) in pixels (per step)."""
    y, x = np.mgrid[0:D, 0:D].astype(np.float64)
    out = np.zeros((D, D))
    for S, w, o, v in zip(screens, weights, origins, velocities):
        out += float(w) * bilinear_periodic(S, x + o[0] + v[0] * t, y + o[1] + v[1] * t)
    return out


def integrator_step(c_prev: np.ndarray, m: np.ndarray, gain: np.ndarray, ff: np.ndarray) -> np.ndarray:
    return ff * c_prev + gain * m


def group_vector(values, sizes) -> np.ndarray:
    """Per-mode vector from per-group values and group sizes."""
    return np.concatenate([np.full(int(n), float(v)) for v, n in zip(values, sizes)])


def run(sensor, screens, weights, origins, velocities, B: np.ndarray, R: np.ndarray, gain, ff, delay: int,
        n_steps: int, t0: int = 0):
    """Closed loop for n_steps: returns per step the slopes [2][n][n], the
    reconstructed modes m, the integrator output c and the residual OPD RMS
    over the pupil.  B: [D*D][modes] nm per unit command, R: [modes][2 n n]."""
    D = sensor.n_pupil
    A = O.pupil_amplitude(D, sensor.obstruction) > 0
    n_modes = B.shape[1]
    hist = [np.zeros(n_modes) for _ in range(delay + 1)]      # c(t - delay .. t - 1) and the current slot
    out = {"slopes": [], "modes": [], "commands": [], "residual_rms": []}
    c_prev = np.zeros(n_modes)
    ref = O.reference_slopes(sensor) if sensor.flags & O.FLAG_REF_SLOPES else None
    for k in range(n_steps):
        t = t0 + k
        applied = hist[(t - delay) % (delay + 1)] if t >= delay else np.zeros(n_modes)
        opd = layers_opd(screens, weights, origins, velocities, t, D) - (B @ applied).reshape(D, D)
        res = opd[A]
        out["residual_rms"].append(float(np.sqrt(np.mean((res - res.mean()) ** 2))))
        I = O.forward(opd[None], sensor)
        s, _ = O.slopes(I, sensor, ref)
        m = R @ s[0].ravel()
        c = integrator_step(c_prev, m, gain, ff)
        hist[t % (delay + 1)] = c
        c_prev = c
        out["slopes"].append(s[0])
        out["modes"].append(m)
        out["commands"].append(c)
    return {k: np.array(v) for k, v in out.items()}
