"""Closed adaptive-optics loop around the pyramid sensor, on the library's kernels.

One timestep, as in the SOUL chain of the paper (Appendix B; the delayed
connection of Section 2.1):

    opd      = layers(t)                       pwfs_layers      (frozen flow)
    opd     -= B c_applied                     pwfs_gemv        (modal mirror)
    I        = sensor(opd); s = slopes(I)      pwfs_forward / pwfs_slopes
    m        = R s                             pwfs_gemv        (Modalrec)
    c(t)     = ff * c(t-1) + g * m             pwfs_integrator  (delay d)
    c_applied <- c(t + 1 - d); t <- t + 1

Every step runs in the library; the time index is device memory, so a
timestep captured in a HIP graph replays as the loop.  The interaction
matrix is measured by push-pull through the same sensor kernels; its
pseudo-inverse (the reconstructor, a calibration step done once) is taken on
the host in float64.
"""

from __future__ import annotations

import numpy as np

from . import pwfs as P


class ClosedLoop:
    def __init__(self, sensor, B: np.ndarray, screens: np.ndarray, layer_params, gain, ff, delay: int,
                 R: np.ndarray | None = None, device=None, precision: int = P.BF16X3):
        """sensor: SensorDesc; B [D*D][modes] mirror influence (nm per unit
        command); screens [L][rows][cols] nm; layer_params [(weight, origin_x,
        origin_y, vel_x, vel_y)] per layer (pixels, pixels per step); gain, ff
        per mode; R [modes][2 n n] reconstructor (measured by calibrate() if
        None)."""
        import torch
        self.torch = torch
        self.device = torch.device(device if device is not None else "cuda")
        self.sensor = sensor
        self.D = sensor.n_pupil
        self.n_modes = int(B.shape[1])
        self.delay = int(delay)
        self.precision = precision
        self.layer_params = [tuple(float(v) for v in p) for p in layer_params]
        dev = self.device
        self.B = torch.from_numpy(np.ascontiguousarray(B, np.float32)).to(dev)
        self.screens = torch.from_numpy(np.ascontiguousarray(screens, np.float32)).to(dev)
        self.gain = torch.from_numpy(np.asarray(gain, np.float32)).to(dev)
        self.ff = torch.from_numpy(np.asarray(ff, np.float32)).to(dev)
        self.plan = P.Plan([sensor], max_frames=1 if R is not None else 2 * self.n_modes, device=dev)
        self.n_slopes = 2 * sensor.n_subap ** 2
        self.step_t = torch.zeros(1, dtype=torch.int64, device=dev)
        self.hist = torch.zeros((self.delay + 1, self.n_modes), dtype=torch.float32, device=dev)
        self.applied = torch.zeros(self.n_modes, dtype=torch.float32, device=dev)
        self.opd = torch.empty((self.D, self.D), dtype=torch.float32, device=dev)
        self.I = self.plan.new_intensity(1)
        self.slopes = self.plan.new_slopes(1)
        self.flux = torch.zeros((1, 1), dtype=torch.float32, device=dev)
        self.modes = torch.empty(self.n_modes, dtype=torch.float32, device=dev)
        self.R = None if R is None else torch.from_numpy(np.ascontiguousarray(R, np.float32)).to(dev)
        self.IM = None
        self.graph = None

    # ------------------------------------------------------------ calibration --
    def calibrate(self, delta_nm: float = 10.0, rcond: float = 1e-3):
        """Push-pull interaction matrix [slopes][modes] through the sensor
        kernels, and R = pinv over the valid slopes (float64, host)."""
        torch = self.torch
        n = self.n_modes
        e = torch.zeros((2 * n, n), dtype=torch.float32, device=self.device)
        idx = torch.arange(n, device=self.device)
        e[idx, idx] = delta_nm
        e[n + idx, idx] = -delta_nm
        opd = P.gemm(e, self.B, precision=self.precision)                 # [2n][D*D]
        _, s, _ = self.plan.step(opd.view(2 * n, self.D, self.D))
        s = s.view(2 * n, -1).double()
        IM = ((s[:n] - s[n:]) / (2.0 * delta_nm)).t().cpu().numpy()        # [slopes][modes]
        valid = np.tile(self.plan.valid_map(0).reshape(-1), 2)
        R = np.zeros((n, self.n_slopes))
        R[:, valid] = np.linalg.pinv(IM[valid], rcond=rcond)
        self.IM = IM
        self.R = torch.from_numpy(R.astype(np.float32)).to(self.device)
        return IM, R

    # ------------------------------------------------------------------ loop --
    def reset(self, t0: int = 0):
        self.step_t.fill_(int(t0))
        self.hist.zero_()
        self.applied.zero_()

    def step(self, stream=None):
        if self.R is None:
            raise RuntimeError("no reconstructor: pass R or call calibrate()")
        D = self.D
        P.layers(self.screens, self.layer_params, D, self.step_t, out=self.opd, stream=stream)
        P.gemv(self.B, self.applied, out=self.opd.view(-1), alpha=-1.0, beta=1.0, stream=stream)
        self.plan.forward(self.opd.view(1, D, D), self.I, stream=stream)
        self.plan.slopes(self.I, self.slopes, self.flux, stream=stream)
        P.gemv(self.R, self.slopes.view(-1), out=self.modes, stream=stream)
        P.integrator(self.modes, self.gain, self.ff, self.delay, self.hist, self.applied, self.step_t,
                     stream=stream)

    def capture(self):
        """Record one timestep in a HIP graph (the loop's state stays in
        device buffers, so replays continue the loop)."""
        torch = self.torch
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        saved = (self.step_t.clone(), self.hist.clone(), self.applied.clone())
        with torch.cuda.stream(side):
            self.step(stream=side)              # warm-up outside the graph (allocator, first-use setup)
        side.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            self.step(stream=side)
        torch.cuda.synchronize(self.device)
        self.step_t.copy_(saved[0])
        self.hist.copy_(saved[1])
        self.applied.copy_(saved[2])
        self.graph = g
        return g

    def run(self, n_steps: int, use_graph: bool = True, record=None):
        """n_steps timesteps; ``record(loop)`` is called after each if given."""
        for _ in range(int(n_steps)):
            if use_graph and self.graph is not None:
                self.graph.replay()
            else:
                self.step()
            if record is not None:
                record(self)

    def residual_rms(self, pupil: np.ndarray) -> float:
        """Piston-removed RMS (nm) of the residual OPD of the last step over
        the pupil (telemetry; copies the plane to the host)."""
        r = self.opd.cpu().numpy()[pupil]
        return float(np.sqrt(np.mean((r - r.mean()) ** 2)))
