"""Learned-surrogate form of the pyramid sensor: modal coefficients -> slopes.

The surrogate is the linear push-pull interaction matrix (the method without
the network) plus a fully connected network (GELU, bf16 weights, fp32
accumulation) that learns what the linear model misses -- mostly the
sensor's loss of sensitivity (optical gain) and the cross-talk between modes
at a residual of this size:

    s(z) ~ IM z + r_rms * net(z).

The network is trained on the residual s - IM z of data the plain sensor
kernels generate, on the GPU by the library's own forward/backward/Adam
kernels; its output layer starts at zero, so training starts from the linear
model.  The plain sensor stays the reference for the surrogate's error and its
fallback for inputs outside the training distribution.  Every product and
every sensor step runs in the library (``pwfs.gemm``, ``pwfs.Plan``,
``pwfs.MLP``); torch only holds device memory.

Inputs of the network are the standard-normal draws z (coefficient / its
RMS); OPD = sum_j z_j sigma_j Z_j * lambda / (2 pi) with the KL-like basis
Z of ``workloads.modes``.  r_rms is the RMS of the training residual.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import pwfs as P


@dataclass
class TrainReport:
    epochs: int
    steps: int
    seconds: float
    losses: list


class SurrogatePipeline:
    def __init__(self, sensor, modes: np.ndarray, sigmas: np.ndarray, device=None, chunk: int = 1024):
        import torch
        self.torch = torch
        self.sensor = sensor
        self.device = torch.device(device if device is not None else "cuda")
        self.n_modes = modes.shape[0]
        self.chunk = int(chunk)
        lam = sensor.lambdas_nm[0] if len(sensor.lambdas_nm) == 1 else sensor.lambda_ref_nm
        basis = (modes * (sigmas * lam / (2.0 * math.pi))[:, None]).T       # [pixels][modes], nm per unit z
        self.basis = torch.from_numpy(np.ascontiguousarray(basis, np.float32)).to(self.device)
        self.plan = P.Plan([sensor], max_frames=self.chunk, device=self.device)
        self.n_out = 2 * sensor.n_subap ** 2
        self.valid = torch.from_numpy(self.plan.valid_map(0)).to(self.device)
        self._I = self.plan.new_intensity(self.chunk)
        self._opd = torch.empty((self.chunk, sensor.n_pupil * sensor.n_pupil), dtype=torch.float32,
                                device=self.device)
        self.mlp = None
        self.s_scale = 1.0
        self.im = None
        self._linear_set = False

    # ------------------------------------------------------------ plain path --
    def slopes_of(self, z, out=None):
        """Plain-sensor slopes [n][2 n_sub^2] of modal draws z [n][n_modes] (device)."""
        torch = self.torch
        n = int(z.shape[0])
        if out is None:
            out = torch.empty((n, self.n_out), dtype=torch.float32, device=self.device)
        D = self.sensor.n_pupil
        for i0 in range(0, n, self.chunk):
            i1 = min(n, i0 + self.chunk)
            c = i1 - i0
            opd = self._opd[:c]
            P.gemm(z[i0:i1], self.basis, out=opd, precision=P.BF16X3)
            I = self.plan.forward(opd.view(c, D, D), self._I[:c])
            self.plan.slopes(I, out=out[i0:i1])
        return out

    def generate(self, n: int, seed: int):
        """(z [n][n_modes], slopes [n][n_out]) on the device."""
        from workloads.modes import draws
        torch = self.torch
        z = torch.from_numpy(draws(n, self.n_modes, seed)).to(self.device)
        return z, self.slopes_of(z)

    # ------------------------------------------------ linear-IM baseline --
    def interaction_matrix(self, delta: float = 0.01):
        """Push-pull interaction matrix [n_out][n_modes] (slopes per unit z)."""
        torch = self.torch
        e = torch.zeros((2 * self.n_modes, self.n_modes), dtype=torch.float32, device=self.device)
        idx = torch.arange(self.n_modes, device=self.device)
        e[idx, idx] = delta
        e[self.n_modes + idx, idx] = -delta
        s = self.slopes_of(e)
        im = (s[:self.n_modes] - s[self.n_modes:]) / (2.0 * delta)   # [modes][n_out]
        self.im = im.t().contiguous()                                # [n_out][modes]
        return self.im

    def linear_predict(self, z):
        return P.gemm(z, self.im, precision=P.BF16X3)

    # ---------------------------------------------------------- surrogate --
    def residual(self, z, s):
        """s - IM z (device), the part of the slopes the linear model misses."""
        r = s.clone()
        P.gemm(z, self.im, out=r, alpha=-1.0, beta=1.0, precision=P.BF16X3)
        return r

    def train(self, z, s, hidden=(1024, 1024), epochs: int = 20, batch: int = 1024, lr: float = 1e-3,
              lr_final: float = 5e-5, seed: int = 5, precision: int = P.BF16,
              infer_batch: int = 32768) -> TrainReport:
        """Trains the network on the residual of (z, s) over the interaction
        matrix (built first if missing); cosine learning-rate decay from
        ``lr`` to ``lr_final``; one Adam step per batch.  The network holds
        activations for ``infer_batch`` rows, so that inference runs its
        products over that many rows at once (enough tiles to fill the chip)."""
        from workloads.modes import init_params
        torch = self.torch
        if self.im is None:
            self.interaction_matrix()
        n = int(z.shape[0]) // batch * batch
        sizes = [self.n_modes, *hidden, self.n_out]
        self.mlp = P.MLP(sizes, max_batch=max(batch, self.chunk, infer_batch), precision=precision,
                         device=self.device)
        self._linear_set = False
        self.mlp.set_params(torch.from_numpy(init_params(sizes, seed, zero_last=True)).to(self.device))
        r = self.residual(z[:n], s[:n])
        rms = P.row_rms(r)
        self.s_scale = float(torch.sqrt((rms.double() ** 2).mean()).item())
        ts = 1.0 / self.s_scale
        steps = epochs * (n // batch)
        losses = []
        t0 = time.perf_counter()
        k = 0
        for ep in range(epochs):
            for i0 in range(0, n, batch):
                frac = k / max(1, steps - 1)
                lr_k = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * frac))
                self.mlp.grad(z[i0:i0 + batch], r[i0:i0 + batch], ts)
                self.mlp.adam(lr_k)
                k += 1
            losses.append(float(self.mlp.loss_buf.item()))
        torch.cuda.synchronize(self.device)
        return TrainReport(epochs, steps, time.perf_counter() - t0, losses)

    def predict(self, z, out=None):
        """Surrogate slopes [n][n_out] (device): IM z + r_rms net(z), the
        interaction-matrix term folded into the network's output-layer
        product (bf16 like the network's weights), in chunks of max_batch."""
        torch = self.torch
        n = int(z.shape[0])
        if out is None:
            out = torch.empty((n, self.n_out), dtype=torch.float32, device=self.device)
        if not self._linear_set:
            self.mlp.set_linear(self.im)
            self._linear_set = True
        mb = self.mlp.max_batch
        for i0 in range(0, n, mb):
            i1 = min(n, i0 + mb)
            self.mlp.forward(z[i0:i1], out=out[i0:i1], out_scale=self.s_scale)
        return out

    def predict_with_fallback(self, z, rms_limit: float = 1.5):
        """Surrogate slopes, with the plain sensor for rows whose draw RMS
        exceeds ``rms_limit`` (outside the training distribution).  Returns
        (slopes, fallback row mask)."""
        out = self.predict(z)
        rms = P.row_rms(z)
        mask = (rms > rms_limit)
        rows = mask.nonzero().flatten()
        if rows.numel():
            out[rows] = self.slopes_of(z[rows].contiguous())
        return out, mask

    def rel_error(self, s, s_ref) -> float:
        """Pooled relative RMS error over valid subapertures."""
        torch = self.torch
        n = self.sensor.n_subap
        v = self.valid.reshape(-1)
        a = s.view(-1, 2, n * n)[:, :, v].double()
        b = s_ref.view(-1, 2, n * n)[:, :, v].double()
        return float(((a - b).norm() / b.norm()).item())
