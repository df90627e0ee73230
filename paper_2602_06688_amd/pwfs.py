"""Python binding of ``libpwfs.so`` (argument marshalling only).

Every step of the sensor path runs in the library's HIP kernels; this module
only turns torch tensors and streams into the plain pointers and sizes of the
C ABI in ``include/pwfs.h``.  There is no fallback: if the library is not
built, every call raises.
"""

from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpwfs.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pwfs.h")

PWFS_OK = 0
PWFS_EINVAL = -1
PWFS_EUNSUPPORTED = -2
PWFS_EWORKSPACE = -3
PWFS_EHIP = -4
PWFS_ESTATE = -5

F_REF_SLOPES = 1
F_FULL_PLANE = 2
F_LOCAL_NORM = 4
F_DOUBLE_ROOF = 8

FP32, BF16, BF16X3, FP16X3, FP16 = 0, 1, 2, 3, 4
MAX_LAMBDA = 16


class PwfsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pwfs error {code}: {msg}")
        self.code = code


class CSensorDesc(ctypes.Structure):
    _fields_ = [
        ("n_pupil", ctypes.c_int32), ("n_fft", ctypes.c_int32), ("n_subap", ctypes.c_int32),
        ("n_mod", ctypes.c_int32), ("n_lambda", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("src_rings", ctypes.c_int32),
        ("diameter_m", ctypes.c_double), ("obstruction", ctypes.c_double),
        ("pupil_sep_px", ctypes.c_double), ("mod_radius_lod", ctypes.c_double),
        ("lambda_ref_nm", ctypes.c_double),
        ("lambda_nm", ctypes.c_double * MAX_LAMBDA), ("lambda_weight", ctypes.c_double * MAX_LAMBDA),
        ("src_radius_lod", ctypes.c_double), ("fov_lod", ctypes.c_double),
    ]


class CSensorInfo(ctypes.Structure):
    _fields_ = [
        ("n_pupil", ctypes.c_int32), ("n_fft", ctypes.c_int32), ("n_subap", ctypes.c_int32),
        ("n_valid", ctypes.c_int32),
        ("opd_offset", ctypes.c_size_t), ("intensity_offset", ctypes.c_size_t),
        ("slope_offset", ctypes.c_size_t), ("opd_stride", ctypes.c_size_t),
        ("intensity_stride", ctypes.c_size_t), ("slope_stride", ctypes.c_size_t),
    ]


class CTuning(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("chunk", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("row_groups", ctypes.c_int32), ("max_chunk", ctypes.c_int32), ("spin_limit", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


MODE_LAUNCHES = 0
MODE_PERSISTENT = 1
MODE_FUSED = 2

CCD_PHOTON = 1
CCD_READOUT = 2
CCD_EXCESS = 4


class CCcdDesc(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int32), ("rebin", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("rebin_den", ctypes.c_int32), ("electrons", ctypes.c_double), ("readout_e", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class CShDesc(ctypes.Structure):
    _fields_ = [("n_pupil", ctypes.c_int32), ("n_subap", ctypes.c_int32), ("n_fft", ctypes.c_int32),
                ("rebin", ctypes.c_int32), ("n_lambda", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("obstruction", ctypes.c_double), ("lambda_nm", ctypes.c_double),
                ("lambdas_nm", ctypes.c_double * MAX_LAMBDA), ("lambda_weights", ctypes.c_double * MAX_LAMBDA)]


class CLayer(ctypes.Structure):
    _fields_ = [("weight", ctypes.c_double), ("origin_x", ctypes.c_double), ("origin_y", ctypes.c_double),
                ("vel_x", ctypes.c_double), ("vel_y", ctypes.c_double)]


def ccd_desc(n_det: int, rebin, electrons: float, flags: int = CCD_PHOTON, readout_e: float = 0.0,
             seed: int = 0) -> CCcdDesc:
    """A detector description (see pwfs_ccd_desc in include/pwfs.h); rebin is
    an integer or a fractions.Fraction (transform pixels per detector pixel)."""
    from fractions import Fraction
    r = Fraction(rebin)
    return CCcdDesc(int(n_det), int(r.numerator), int(flags), int(r.denominator) if r.denominator > 1 else 0,
                    float(electrons), float(readout_e), int(seed) & ((1 << 64) - 1))

_lib = None


def header_symbols() -> list:
    """Function names declared by include/pwfs.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pwfs_[a-z0-9_]+)\s*\(", text)))


def lib() -> ctypes.CDLL:
    """Loads the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2602_06688_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i32 = ctypes.c_int
    L.pwfs_validate.argtypes = [P(CSensorDesc), i32]
    L.pwfs_workspace_size.argtypes = [P(CSensorDesc), i32, i32, P(ctypes.c_size_t)]
    L.pwfs_plan.argtypes = [P(CSensorDesc), i32, i32, vp, ctypes.c_size_t, vp, P(vp)]
    L.pwfs_forward.argtypes = [vp, vp, i32, vp, vp]
    L.pwfs_slopes.argtypes = [vp, vp, i32, vp, vp, vp]
    L.pwfs_query.argtypes = [vp, i32, P(CSensorInfo)]
    L.pwfs_device_status.argtypes = [vp, vp]
    L.pwfs_valid_map.argtypes = [vp, i32, P(ctypes.c_uint8)]
    L.pwfs_last_error.restype = ctypes.c_char_p
    L.pwfs_last_error.argtypes = []
    L.pwfs_profile.argtypes = [vp, i32]
    L.pwfs_profile_read.argtypes = [vp, i32, P(ctypes.c_double), P(ctypes.c_int)]
    L.pwfs_destroy.argtypes = [vp]
    L.pwfs_destroy.restype = None
    L.pwfs_ccd.argtypes = [vp, i32, P(CCcdDesc), vp, i32, ctypes.c_longlong, vp, vp]
    L.pwfs_ccd_slopes.argtypes = [vp, i32, P(CCcdDesc), vp, i32, vp, vp, vp]
    L.pwfs_layers.argtypes = [vp, i32, i32, i32, P(CLayer), i32, vp, vp, vp]
    L.pwfs_integrator.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, vp]
    L.pwfs_gemv.argtypes = [vp, ctypes.c_longlong, vp, vp, i32, i32, ctypes.c_float, ctypes.c_float, vp]
    L.pwfs_sh_validate.argtypes = [P(CShDesc)]
    L.pwfs_sh_workspace_size.argtypes = [P(CShDesc), i32, P(ctypes.c_size_t)]
    L.pwfs_sh_plan.argtypes = [P(CShDesc), i32, vp, ctypes.c_size_t, vp, P(vp)]
    L.pwfs_sh_forward.argtypes = [vp, vp, i32, vp, vp, vp]
    L.pwfs_sh_query.argtypes = [vp, P(ctypes.c_int32), P(ctypes.c_int32)]
    L.pwfs_sh_destroy.argtypes = [vp]
    L.pwfs_sh_destroy.restype = None
    L.pwfs_get_tuning.argtypes = [vp, P(CTuning)]
    L.pwfs_set_tuning.argtypes = [vp, P(CTuning)]
    L.pwfs_set_row_tile.argtypes = [vp, i32, i32]
    L.pwfs_get_row_tile.argtypes = [vp, i32, P(ctypes.c_int32)]
    ll = ctypes.c_longlong
    L.pwfs_gemm_workspace_size.argtypes = [i32, i32, i32, i32, P(ctypes.c_size_t)]
    L.pwfs_gemm.argtypes = [vp, ll, vp, ll, vp, ll, i32, i32, i32, ctypes.c_float, ctypes.c_float, i32, vp,
                            ctypes.c_size_t, vp]
    L.pwfs_gemm_noalloc.argtypes = [vp, ll, vp, ll, vp, ll, i32, i32, i32, ctypes.c_float, ctypes.c_float, i32, vp]
    L.pwfs_row_rms.argtypes = [vp, ll, i32, i32, vp, vp]
    L.pwfs_mlp_workspace_size.argtypes = [i32, P(ctypes.c_int32), i32, i32, P(ctypes.c_size_t)]
    L.pwfs_mlp_create.argtypes = [i32, P(ctypes.c_int32), i32, i32, vp, ctypes.c_size_t, vp, P(vp)]
    L.pwfs_mlp_param_count.argtypes = [vp, P(ctypes.c_size_t)]
    L.pwfs_mlp_set_params.argtypes = [vp, vp, vp]
    L.pwfs_mlp_get_params.argtypes = [vp, vp, vp]
    L.pwfs_mlp_set_linear.argtypes = [vp, vp, vp]
    L.pwfs_mlp_get_state.argtypes = [vp, vp, P(ctypes.c_longlong), vp]
    L.pwfs_mlp_set_state.argtypes = [vp, vp, ctypes.c_longlong, vp]
    L.pwfs_mlp_forward.argtypes = [vp, vp, i32, vp, ctypes.c_float, vp]
    L.pwfs_mlp_grad.argtypes = [vp, vp, vp, i32, ctypes.c_float, vp, vp, vp]
    L.pwfs_mlp_adam.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]
    L.pwfs_mlp_destroy.argtypes = [vp]
    L.pwfs_mlp_destroy.restype = None
    for name in ("pwfs_validate", "pwfs_workspace_size", "pwfs_plan", "pwfs_forward", "pwfs_slopes",
                 "pwfs_query", "pwfs_device_status", "pwfs_set_row_tile", "pwfs_get_row_tile", "pwfs_valid_map", "pwfs_profile", "pwfs_profile_read",
                 "pwfs_gemm_workspace_size", "pwfs_gemm", "pwfs_gemm_noalloc", "pwfs_row_rms", "pwfs_mlp_workspace_size",
                 "pwfs_mlp_create", "pwfs_mlp_param_count", "pwfs_mlp_set_params", "pwfs_mlp_get_params",
                 "pwfs_mlp_get_state", "pwfs_mlp_set_state", "pwfs_mlp_set_linear",
                 "pwfs_mlp_forward", "pwfs_mlp_grad", "pwfs_mlp_adam", "pwfs_ccd", "pwfs_ccd_slopes", "pwfs_layers", "pwfs_integrator", "pwfs_gemv", "pwfs_sh_validate",
                 "pwfs_sh_workspace_size", "pwfs_sh_plan", "pwfs_sh_forward", "pwfs_sh_query"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != PWFS_OK:
        raise PwfsError(rc, lib().pwfs_last_error().decode())


def to_c(s) -> CSensorDesc:
    """A C description from any object with the SensorDesc attributes."""
    d = CSensorDesc()
    d.n_pupil = int(s.n_pupil)
    d.n_fft = int(s.n_fft)
    d.n_subap = int(s.n_subap)
    d.n_mod = int(s.n_mod)
    lams = tuple(s.lambdas_nm)
    ws = tuple(s.lambda_weights)
    d.n_lambda = len(lams)
    d.precision = int(getattr(s, "precision", FP32))
    d.flags = int(getattr(s, "flags", F_REF_SLOPES))
    d.src_rings = int(getattr(s, "src_rings", 0))
    d.src_radius_lod = float(getattr(s, "src_radius_lod", 0.0))
    d.fov_lod = float(getattr(s, "fov_lod", 0.0))
    d.diameter_m = float(getattr(s, "diameter_m", 8.0))
    d.obstruction = float(s.obstruction)
    d.pupil_sep_px = float(s.pupil_sep_px)
    d.mod_radius_lod = float(s.mod_radius_lod)
    d.lambda_ref_nm = float(s.lambda_ref_nm)
    for i in range(min(len(lams), MAX_LAMBDA)):
        d.lambda_nm[i] = float(lams[i])
        d.lambda_weight[i] = float(ws[i])
    return d


def _descs(sensors) -> ctypes.Array:
    sensors = list(sensors)
    arr = (CSensorDesc * len(sensors))()
    for i, s in enumerate(sensors):
        arr[i] = s if isinstance(s, CSensorDesc) else to_c(s)
    return arr


def validate(sensors) -> int:
    """Return code of pwfs_validate (host only)."""
    arr = _descs(sensors)
    return lib().pwfs_validate(arr, len(arr))


def workspace_size(sensors, max_frames: int) -> int:
    arr = _descs(sensors)
    n = ctypes.c_size_t()
    check(lib().pwfs_workspace_size(arr, len(arr), int(max_frames), ctypes.byref(n)))
    return n.value


def _stream_ptr(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _dev_ptr(t, name, dtype=None, min_numel=None):
    import torch
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {min_numel}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A plan over one or more sensors; owns its device workspace tensor."""

    def __init__(self, sensors: Sequence, max_frames: int, device=None, stream=None):
        import torch
        self.sensors = list(sensors)
        self._descs = _descs(self.sensors)
        self.max_frames = int(max_frames)
        self.device = torch.device(device if device is not None else "cuda")
        nbytes = workspace_size(self._descs, self.max_frames)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        h = ctypes.c_void_p()
        check(lib().pwfs_plan(self._descs, len(self._descs), self.max_frames, ctypes.c_void_p(self._ws_ptr),
                              nbytes, _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self.info = [self.query(i) for i in range(len(self.sensors))]
        i0 = self.info[0]
        self.opd_stride = i0.opd_stride
        self.intensity_stride = i0.intensity_stride
        self.slope_stride = i0.slope_stride

    def query(self, sensor: int) -> CSensorInfo:
        info = CSensorInfo()
        check(lib().pwfs_query(self._h, int(sensor), ctypes.byref(info)))
        return info

    def valid_map(self, sensor: int = 0):
        import numpy as np
        n = self.info[sensor].n_subap if hasattr(self, "info") else int(self.sensors[sensor].n_subap)
        buf = (ctypes.c_uint8 * (n * n))()
        check(lib().pwfs_valid_map(self._h, int(sensor), buf))
        return np.frombuffer(bytes(buf), dtype=np.uint8).reshape(n, n).astype(bool)

    # -- shapes of a single-sensor plan; multi-sensor plans use packed [F][stride]
    def _single(self) -> bool:
        return len(self.sensors) == 1

    def new_intensity(self, n_frames: int):
        import torch
        if self._single():
            N = self.info[0].n_fft
            planes = self.intensity_stride // (N * N)      # 2 for a double roof
            shape = (n_frames, N, N) if planes == 1 else (n_frames, planes, N, N)
            return torch.zeros(shape, dtype=torch.float32, device=self.device)
        return torch.zeros((n_frames, self.intensity_stride), dtype=torch.float32, device=self.device)

    def new_slopes(self, n_frames: int):
        import torch
        if self._single():
            n = self.info[0].n_subap
            return torch.zeros((n_frames, 2, n, n), dtype=torch.float32, device=self.device)
        return torch.zeros((n_frames, self.slope_stride), dtype=torch.float32, device=self.device)

    def forward(self, opd, out=None, stream=None):
        """OPD [F, D, D] (or packed [F, opd_stride]) float32 nm -> intensity."""
        import torch
        F = int(opd.shape[0])
        if out is None:
            out = self.new_intensity(F)
        po = _dev_ptr(opd, "opd", torch.float32, F * self.opd_stride)
        pi = _dev_ptr(out, "intensity", torch.float32, F * self.intensity_stride)
        check(lib().pwfs_forward(self._h, po, F, pi, _stream_ptr(stream)))
        return out

    def slopes(self, intensity, out=None, flux=None, stream=None):
        """intensity -> (slopes, flux [F, n_sensors])."""
        import torch
        F = int(intensity.shape[0])
        if out is None:
            out = self.new_slopes(F)
        if flux is None:
            flux = torch.zeros((F, len(self.sensors)), dtype=torch.float32, device=self.device)
        pi = _dev_ptr(intensity, "intensity", torch.float32, F * self.intensity_stride)
        ps = _dev_ptr(out, "slopes", torch.float32, F * self.slope_stride)
        pf = _dev_ptr(flux, "flux", torch.float32, F * len(self.sensors))
        check(lib().pwfs_slopes(self._h, pi, F, ps, pf, _stream_ptr(stream)))
        return out, flux

    def step(self, opd, intensity=None, slopes=None, flux=None, stream=None):
        """One pass of the whole path: forward then slopes."""
        I = self.forward(opd, intensity, stream)
        s, fl = self.slopes(I, slopes, flux, stream)
        return I, s, fl

    def ccd(self, intensity, ccd: CCcdDesc, frame0: int = 0, out=None, sensor: int = 0, stream=None):
        """Detector frames [F, n_det, n_det] (electrons) of one sensor's
        intensity, as written by ``forward``; frame f draws its noise as
        global frame frame0 + f."""
        import torch
        F = int(intensity.shape[0])
        n = int(ccd.n_det)
        if out is None:
            out = torch.empty((F, n, n), dtype=torch.float32, device=self.device)
        pi = _dev_ptr(intensity, "intensity", torch.float32, F * self.intensity_stride)
        po = _dev_ptr(out, "pixels", torch.float32, F * n * n)
        check(lib().pwfs_ccd(self._h, int(sensor), ctypes.byref(ccd), pi, F, int(frame0), po, _stream_ptr(stream)))
        return out

    def ccd_slopes(self, pixels, ccd: CCcdDesc, out=None, flux=None, sensor: int = 0, stream=None):
        """Slopes [F, 2, n, n] and flux [F] of detector frames."""
        import torch
        F = int(pixels.shape[0])
        n = int(self.info[sensor].n_subap)
        if out is None:
            out = torch.empty((F, 2, n, n), dtype=torch.float32, device=self.device)
        if flux is None:
            flux = torch.zeros(F, dtype=torch.float32, device=self.device)
        pp = _dev_ptr(pixels, "pixels", torch.float32, F * int(ccd.n_det) ** 2)
        ps = _dev_ptr(out, "slopes", torch.float32, F * 2 * n * n)
        pf = _dev_ptr(flux, "flux", torch.float32, F)
        check(lib().pwfs_ccd_slopes(self._h, int(sensor), ctypes.byref(ccd), pp, F, ps, pf, _stream_ptr(stream)))
        return out, flux

    KERNELS = {"rows": 0, "cols": 1, "slopes": 2, "mfma": 3, "field": 4, "hetero": 5, "ccd": 6, "fused": 7}

    def get_tuning(self) -> dict:
        t = CTuning()
        check(lib().pwfs_get_tuning(self._h, ctypes.byref(t)))
        return {"mode": t.mode, "chunk": t.chunk, "wg_per_cu": t.wg_per_cu, "row_groups": t.row_groups,
                "max_chunk": t.max_chunk, "spin_limit": t.spin_limit}

    def set_tuning(self, **kw) -> dict:
        cur = self.get_tuning()
        cur.update({k: v for k, v in kw.items() if v is not None})
        t = CTuning(int(cur["mode"]), int(cur["chunk"]), int(cur["wg_per_cu"]), int(cur["row_groups"]),
                    int(cur["max_chunk"]), int(cur["spin_limit"]))
        check(lib().pwfs_set_tuning(self._h, ctypes.byref(t)))
        return self.get_tuning()

    def row_tile(self, sensor: int) -> int:
        """Rows per row-pass workgroup that ``sensor`` runs with (pwfs_get_row_tile)."""
        r = ctypes.c_int32()
        check(lib().pwfs_get_row_tile(self._h, int(sensor), ctypes.byref(r)))
        return r.value

    def set_row_tile(self, sensor: int, rows: int) -> None:
        """Selects the row-pass tile of one FP32 sensor (0 = its default; pwfs_set_row_tile)."""
        check(lib().pwfs_set_row_tile(self._h, int(sensor), int(rows)))

    def status(self, stream=None) -> None:
        """Synchronises the stream and raises PwfsError (PWFS_EHIP) if a
        persistent pass's dependency wait gave up since the last check
        (pwfs_device_status); the flag is cleared."""
        check(lib().pwfs_device_status(self._h, _stream_ptr(stream)))

    def profile(self, max_launches: int) -> None:
        """Time the next ``max_launches`` kernel launches with HIP events (0 = off)."""
        check(lib().pwfs_profile(self._h, int(max_launches)))

    def profile_read(self, kernel: str):
        """(total ms, launches) of one kernel kind since ``profile`` was called."""
        t = ctypes.c_double()
        n = ctypes.c_int()
        check(lib().pwfs_profile_read(self._h, self.KERNELS[kernel], ctypes.byref(t), ctypes.byref(n)))
        return t.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().pwfs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ dense products --

def _aligned_workspace(nbytes: int, device):
    import torch
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    ptr = (buf.data_ptr() + 255) & ~255
    return buf, ptr


def _gemm_operands(A, B, out, beta):
    import torch
    M, K = (int(v) for v in A.shape)
    N, K2 = (int(v) for v in B.shape)
    if K2 != K:
        raise ValueError("inner dimensions differ")
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs an output to accumulate into")
        out = torch.empty((M, N), dtype=torch.float32, device=A.device)
    if tuple(out.shape) != (M, N):
        raise ValueError(f"out must have shape {(M, N)}, has {tuple(out.shape)}")
    for name, t in (("A", A), ("B", B), ("out", out)):
        if t.dtype != torch.float32 or not t.is_cuda or t.stride(1) != 1:
            raise ValueError(f"{name} must be a row-major float32 device matrix")
    return M, N, K, out


def gemm(A, B, out=None, alpha: float = 1.0, beta: float = 0.0, precision: int = BF16X3, stream=None):
    """out [M, N] = alpha * A [M, K] @ B [N, K]^T + beta * out on the matrix
    cores (with beta == 0 the old contents of ``out`` are not read)."""
    import torch
    M, N, K, out = _gemm_operands(A, B, out, beta)
    n = ctypes.c_size_t()
    check(lib().pwfs_gemm_workspace_size(M, N, K, precision, ctypes.byref(n)))
    ws, ptr = _aligned_workspace(n.value, A.device)
    st = stream if stream is not None else torch.cuda.current_stream(A.device)
    ws.record_stream(st)   # the kernels read it on `st` after this function returns
    check(lib().pwfs_gemm(ctypes.c_void_p(A.data_ptr()), A.stride(0), ctypes.c_void_p(B.data_ptr()), B.stride(0),
                          ctypes.c_void_p(out.data_ptr()), out.stride(0), M, N, K, float(alpha), float(beta),
                          precision, ctypes.c_void_p(ptr), n.value, _stream_ptr(st)))
    return out


def gemm_noalloc(A, B, out, alpha: float = 1.0, beta: float = 0.0, precision: int = BF16X3, stream=None):
    """``gemm`` into a caller-provided ``out`` with the operand planes in the
    library's static device scratch (pwfs_gemm_noalloc): nothing is allocated,
    so it can run where allocation is not allowed.  Calls that can overlap on
    one GPU share that scratch and must be serialised by the caller."""
    M, N, K, out = _gemm_operands(A, B, out, beta)
    check(lib().pwfs_gemm_noalloc(ctypes.c_void_p(A.data_ptr()), A.stride(0), ctypes.c_void_p(B.data_ptr()),
                                  B.stride(0), ctypes.c_void_p(out.data_ptr()), out.stride(0), M, N, K,
                                  float(alpha), float(beta), precision, _stream_ptr(stream)))
    return out


def layers(screens, params, D: int, step, out=None, stream=None):
    """Frozen-flow OPD [D, D] at t = step[0] (int64 device tensor) of screens
    [L, rows, cols]; params: sequence of (weight, origin_x, origin_y, vel_x,
    vel_y) per layer (see pwfs_layers)."""
    import torch
    Lr, rows, cols = (int(v) for v in screens.shape)
    arr = (CLayer * Lr)(*[CLayer(*[float(v) for v in p]) for p in params])
    if out is None:
        out = torch.empty((D, D), dtype=torch.float32, device=screens.device)
    check(lib().pwfs_layers(_dev_ptr(screens, "screens", torch.float32, Lr * rows * cols), Lr, rows, cols, arr, int(D),
                            _dev_ptr(step, "step", torch.int64, 1), _dev_ptr(out, "opd", torch.float32, D * D),
                            _stream_ptr(stream)))
    return out


def gemv(A, x, out=None, alpha: float = 1.0, beta: float = 0.0, stream=None):
    """out [M] = alpha * A [M, K] @ x [K] + beta * out, float32 (see pwfs_gemv)."""
    import torch
    M, K = (int(v) for v in A.shape)
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs an output to accumulate into")
        out = torch.empty(M, dtype=torch.float32, device=A.device)
    if A.stride(1) != 1:
        raise ValueError("A must be row-major")
    check(lib().pwfs_gemv(ctypes.c_void_p(A.data_ptr()), A.stride(0), _dev_ptr(x, "x", torch.float32, K),
                          _dev_ptr(out, "out", torch.float32, M), M, K, float(alpha), float(beta),
                          _stream_ptr(stream)))
    return out


def integrator(modes, gain, ff, delay: int, hist, applied, step, stream=None):
    """One integrator step (see pwfs_integrator); advances step[0]."""
    import torch
    n = int(modes.numel())
    check(lib().pwfs_integrator(_dev_ptr(modes, "modes", torch.float32, n), _dev_ptr(gain, "gain", torch.float32, n),
                                _dev_ptr(ff, "ff", torch.float32, n), n, int(delay),
                                _dev_ptr(hist, "hist", torch.float32, (int(delay) + 1) * n),
                                _dev_ptr(applied, "applied", torch.float32, n),
                                _dev_ptr(step, "step", torch.int64, 1), _stream_ptr(stream)))


def row_rms(x, out=None, stream=None):
    import torch
    rows, cols = x.shape
    if out is None:
        out = torch.empty(rows, dtype=torch.float32, device=x.device)
    check(lib().pwfs_row_rms(_dev_ptr(x, "x", torch.float32), x.stride(0), rows, cols,
                             _dev_ptr(out, "out", torch.float32), _stream_ptr(stream)))
    return out


def sh_desc(n_pupil: int, n_subap: int, n_fft: int, rebin: int, obstruction: float = 0.0,
            lambda_nm: float = 750.0, lambdas_nm=None, lambda_weights=None) -> CShDesc:
    """Monochromatic at lambda_nm, or polychromatic over lambdas_nm with
    lambda_nm the reference that fixes the angular sampling."""
    d = CShDesc(int(n_pupil), int(n_subap), int(n_fft), int(rebin), 0, 0, float(obstruction), float(lambda_nm))
    if lambdas_nm is not None:
        d.n_lambda = len(lambdas_nm)
        for i, (lam, w) in enumerate(list(zip(lambdas_nm, lambda_weights))[:MAX_LAMBDA]):   # the library checks the count
            d.lambdas_nm[i] = float(lam)
            d.lambda_weights[i] = float(w)
    return d


class SH:
    """A Shack-Hartmann sensor plan on the library's kernel (see pwfs_sh_* in
    include/pwfs.h)."""

    def __init__(self, desc: CShDesc, max_frames: int, device=None, stream=None):
        import torch
        self.desc = desc
        self.device = torch.device(device if device is not None else "cuda")
        self.max_frames = int(max_frames)
        n = ctypes.c_size_t()
        check(lib().pwfs_sh_workspace_size(ctypes.byref(desc), self.max_frames, ctypes.byref(n)))
        self.workspace, ptr = _aligned_workspace(n.value, self.device)
        h = ctypes.c_void_p()
        check(lib().pwfs_sh_plan(ctypes.byref(desc), self.max_frames, ctypes.c_void_p(ptr), n.value,
                                 _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        nv, npx = ctypes.c_int32(), ctypes.c_int32()
        check(lib().pwfs_sh_query(self._h, ctypes.byref(nv), ctypes.byref(npx)))
        self.n_valid, self.n_pix = nv.value, npx.value
        self.n = int(desc.n_subap)

    def forward(self, opd, slopes=None, pixels=None, want_pixels: bool = False, stream=None):
        """OPD [F, D, D] -> (slopes [F, 2, n, n], pixels [F, n, n, n_pix, n_pix] or None)."""
        import torch
        F = int(opd.shape[0])
        D = int(self.desc.n_pupil)
        if slopes is None:
            slopes = torch.empty((F, 2, self.n, self.n), dtype=torch.float32, device=self.device)
        if pixels is None and want_pixels:
            pixels = torch.empty((F, self.n, self.n, self.n_pix, self.n_pix), dtype=torch.float32, device=self.device)
        pp = ctypes.c_void_p(None) if pixels is None else \
            _dev_ptr(pixels, "pixels", torch.float32, F * self.n * self.n * self.n_pix ** 2)
        check(lib().pwfs_sh_forward(self._h, _dev_ptr(opd, "opd", torch.float32, F * D * D), F, pp,
                                    _dev_ptr(slopes, "slopes", torch.float32, F * 2 * self.n * self.n),
                                    _stream_ptr(stream)))
        return slopes, pixels

    def close(self):
        if getattr(self, "_h", None):
            lib().pwfs_sh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """The surrogate network on the library's kernels (see include/pwfs.h)."""

    def __init__(self, sizes, max_batch: int, precision: int = BF16, device=None, stream=None):
        import torch
        self.sizes = [int(v) for v in sizes]
        self.max_batch = int(max_batch)
        self.precision = int(precision)
        self.device = torch.device(device if device is not None else "cuda")
        arr = (ctypes.c_int32 * len(self.sizes))(*self.sizes)
        n = ctypes.c_size_t()
        L = len(self.sizes) - 1
        check(lib().pwfs_mlp_workspace_size(L, arr, self.max_batch, self.precision, ctypes.byref(n)))
        self.workspace, ptr = _aligned_workspace(n.value, self.device)
        h = ctypes.c_void_p()
        check(lib().pwfs_mlp_create(L, arr, self.max_batch, self.precision, ctypes.c_void_p(ptr), n.value,
                                    _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        c = ctypes.c_size_t()
        check(lib().pwfs_mlp_param_count(self._h, ctypes.byref(c)))
        self.n_params = c.value
        self.loss_buf = torch.zeros(1, dtype=torch.float32, device=self.device)

    def set_params(self, params, stream=None):
        import torch
        check(lib().pwfs_mlp_set_params(self._h, _dev_ptr(params, "params", torch.float32, self.n_params),
                                        _stream_ptr(stream)))

    def get_params(self, stream=None):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        check(lib().pwfs_mlp_get_params(self._h, _dev_ptr(out, "params", torch.float32), _stream_ptr(stream)))
        return out

    def set_linear(self, C, stream=None):
        """Fixed linear term C [sizes[-1], sizes[0]] added by forward (None removes it)."""
        import torch
        ptr = ctypes.c_void_p(None) if C is None else \
            _dev_ptr(C, "C", torch.float32, self.sizes[-1] * self.sizes[0])
        check(lib().pwfs_mlp_set_linear(self._h, ptr, _stream_ptr(stream)))

    def get_state(self, stream=None):
        """(Adam moments [2 * n_params] device tensor, step): m then v, each packed like the parameters."""
        import torch
        out = torch.empty(2 * self.n_params, dtype=torch.float32, device=self.device)
        step = ctypes.c_longlong()
        check(lib().pwfs_mlp_get_state(self._h, _dev_ptr(out, "moments", torch.float32), ctypes.byref(step),
                                       _stream_ptr(stream)))
        return out, step.value

    def set_state(self, moments, step: int, stream=None):
        """Restores the Adam state (after set_params, which clears it)."""
        import torch
        check(lib().pwfs_mlp_set_state(self._h, _dev_ptr(moments, "moments", torch.float32, 2 * self.n_params),
                                       int(step), _stream_ptr(stream)))

    def forward(self, x, out=None, out_scale: float = 1.0, stream=None):
        import torch
        B = int(x.shape[0])
        if out is None:
            out = torch.empty((B, self.sizes[-1]), dtype=torch.float32, device=self.device)
        check(lib().pwfs_mlp_forward(self._h, _dev_ptr(x, "x", torch.float32, B * self.sizes[0]), B,
                                     _dev_ptr(out, "y", torch.float32, B * self.sizes[-1]), float(out_scale),
                                     _stream_ptr(stream)))
        return out

    def grad(self, x, t, target_scale: float = 1.0, grads=None, stream=None):
        """Loss (device scalar tensor) and, if ``grads`` is given, packed gradients."""
        import torch
        B = int(x.shape[0])
        gp = ctypes.c_void_p(None) if grads is None else _dev_ptr(grads, "grads", torch.float32, self.n_params)
        check(lib().pwfs_mlp_grad(self._h, _dev_ptr(x, "x", torch.float32, B * self.sizes[0]),
                                  _dev_ptr(t, "t", torch.float32, B * self.sizes[-1]), B, float(target_scale),
                                  _dev_ptr(self.loss_buf, "loss", torch.float32), gp, _stream_ptr(stream)))
        return self.loss_buf

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
        check(lib().pwfs_mlp_adam(self._h, float(lr), float(beta1), float(beta2), float(eps), _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().pwfs_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
