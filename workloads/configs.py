"""Sensor descriptions and workload recipes.

Every number here is a parameter of a workload, not a step of the method.
The sensor parameters follow the pyramid block of the paper's SOUL
configuration listing (Appendix B: pupil diameter, pupil-centre separation,
modulation radius in lambda/D, wavelength) scaled to the five workloads the
build is measured on.  Readings of parameters the paper leaves open (pupil
separation of the 160 px sensor, the six heterogeneous instances, jitter per
axis) are listed in the design doc.
"""

from __future__ import annotations

import math

from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

# flags of the sensor description (mirrored by the C header)
FLAG_REF_SLOPES = 1   # subtract flat-wavefront reference slopes
FLAG_FULL_PLANE = 2   # compute and write every pixel of the N x N plane
FLAG_LOCAL_NORM = 4   # normalise slopes by per-subaperture flux
FLAG_DOUBLE_ROOF = 8  # two-arm double-roof sensor instead of the four-face pyramid

# precision of the forward transform (mirrored by the C header)
PREC_FP32 = 0
PREC_BF16 = 1
PREC_BF16X3 = 2
PREC_FP16X3 = 3
PREC_FP16 = 4


@dataclass(frozen=True)
class SensorDesc:
    """One pyramid sensor.  Lengths in pupil pixels unless stated."""
    n_pupil: int                 # D: pupil diameter in pixels
    n_fft: int                   # N: padded transform size
    n_subap: int                 # subapertures across the pupil
    n_mod: int                   # modulation points on the circle
    pupil_sep_px: float          # S: centre-to-centre pupil image separation
    mod_radius_lod: float        # modulation radius in lambda/D at lambda_ref
    obstruction: float = 0.0     # linear central-obstruction ratio
    diameter_m: float = 8.0      # telescope diameter (only used by input generation)
    lambda_ref_nm: float = 750.0
    lambdas_nm: Tuple[float, ...] = (750.0,)
    lambda_weights: Tuple[float, ...] = (1.0,)
    precision: int = PREC_FP32
    flags: int = FLAG_REF_SLOPES
    src_rings: int = 0           # extended source: rings sampling a uniform disk (0 = point source)
    src_radius_lod: float = 0.0  # extended-source radius in lambda/D at lambda_ref
    fov_lod: float = 0.0         # square field stop, side in lambda/D at lambda_ref (0 = none)

    @property
    def n_lambda(self) -> int:
        return len(self.lambdas_nm)

    def with_(self, **kw) -> "SensorDesc":
        return replace(self, **kw)


@dataclass(frozen=True)
class Workload:
    name: str
    sensors: Tuple[SensorDesc, ...]
    n_frames: int
    r0_m: float                  # Fried parameter at r0_lambda_nm
    L0_m: float                  # outer scale
    seeds: Tuple[int, ...]       # one screen seed per sensor
    r0_lambda_nm: float = 500.0
    jitter_mas: float = 0.0      # RMS tip and tilt per axis
    jitter_seed: Optional[int] = None
    extra: dict = field(default_factory=dict)


def _cfg1() -> Workload:
    s = SensorDesc(n_pupil=64, n_fft=128, n_subap=16, n_mod=16, pupil_sep_px=64.0,
                   mod_radius_lod=3.0, obstruction=0.0, diameter_m=8.0)
    return Workload("pwfs-64px-N128-16mod-16sub", (s,), n_frames=100,
                    r0_m=0.15, L0_m=25.0, seeds=(1,))


def _cfg2() -> Workload:
    s = SensorDesc(n_pupil=160, n_fft=512, n_subap=40, n_mod=48, pupil_sep_px=192.0,
                   mod_radius_lod=3.0, obstruction=0.12, diameter_m=8.0)
    return Workload("pwfs-160px-N512-48mod-40sub", (s,), n_frames=1000,
                    r0_m=0.12, L0_m=40.0, seeds=(2,), jitter_mas=5.0, jitter_seed=12)


def _cfg3() -> Workload:
    w = _cfg1()
    s = w.sensors[0].with_(precision=PREC_BF16X3)
    return replace(w, name="pwfs-64px-N128-16mod-16sub-mfma", sensors=(s,))


def _cfg4() -> Workload:
    pupils = (80, 120, 160, 160, 240, 240)
    ffts = (256, 384, 512, 512, 768, 768)
    mods = ((2.0, 16), (3.0, 32), (3.0, 48), (4.0, 64), (5.0, 80), (5.0, 96))
    sens = []
    for d, n, (r, k) in zip(pupils, ffts, mods):
        sens.append(SensorDesc(n_pupil=d, n_fft=n, n_subap=d // 4, n_mod=k,
                               pupil_sep_px=1.2 * d, mod_radius_lod=r, obstruction=0.28,
                               diameter_m=38.5, lambda_ref_nm=750.0,
                               lambdas_nm=(600.0, 750.0, 900.0),
                               lambda_weights=(1 / 3, 1 / 3, 1 / 3)))
    return Workload("pwfs-hetero6-poly3", tuple(sens), n_frames=500, r0_m=0.157,
                    L0_m=25.0, seeds=tuple(40 + i for i in range(6)))


def _cfg5() -> Workload:
    w = _cfg2()
    s = w.sensors[0]
    return Workload("pwfs-160px-surrogate-500modes", (s,), n_frames=200_000,
                    r0_m=0.12, L0_m=25.0, seeds=(5,),
                    extra=dict(n_modes=500, hidden=1024, n_test=20_000, test_seed=6,
                               residual_rms_nm=100.0))


# Detector of the 160 px sensor after the SOUL configuration (Appendix B):
# 120 x 120 pixels = the central 480 x 480 of the 512 plane in 4 x 4 blocks
# (one pixel per subaperture, the pupil images 40 px wide at 48 px spacing),
# a magnitude-8 source at 750 nm, 0.588 ms integration, 300 nm band,
# quantum efficiency x transmission 0.32, readout 0.4 e-.  The paper gives no
# photometric zero point; 5.0e7 photons / s / m^2 / nm at magnitude 0 near
# 750 nm (about Vega's flux there) is the reading used.
ZERO_POINT_PH = 5.0e7


def photo_electrons(magnitude: float, diameter_m: float, obstruction: float, band_nm: float, dt_s: float,
                    qe: float, zero_point: float = ZERO_POINT_PH) -> float:
    """Expected detected photo-electrons per frame from a source of the given
    magnitude on an annular pupil (obstruction as a diameter ratio)."""
    area = math.pi / 4.0 * diameter_m ** 2 * (1.0 - obstruction ** 2)
    return zero_point * 10.0 ** (-0.4 * magnitude) * area * band_nm * dt_s * qe


def soul_detector(s: SensorDesc) -> dict:
    """Detector parameters (pwfs_ccd_desc fields) for the 160 px sensor."""
    return dict(n_det=120, rebin=4, readout_e=0.4,
                electrons=photo_electrons(8.0, s.diameter_m, s.obstruction, 300.0, 0.000588, 0.32))


def soul_loop(s: SensorDesc) -> dict:
    """Closed loop of the SOUL configuration (Appendix B) around the 160 px
    sensor.  From the listing: 500 modes, integrator gains / forgetting
    factors per mode group of 30 / 70 / 100 / 300 modes, total delay 2,
    four layers with Cn2 fractions 0.70 / 0.06 / 0.14 / 0.10, L0 = 40 m,
    0.8 arcsec seeing on the line of sight (Fig. 9 caption), 0.588 ms steps,
    wind 2 / 4 / 6 / 25 m/s along 0 / 30 / -30 / 45 degrees.  Readings (not
    in the paper): the direction is that of the layer's motion, counted from
    +x towards +y; layers as 1024 x 1024 periodic screens at the pupil's
    pixel size (an on-axis source sees every layer unshifted by height)."""
    pixel_m = s.diameter_m / s.n_pupil
    r0 = 0.98 * 500e-9 / (0.8 / 206264.806)          # Fried parameter at 500 nm for 0.8"
    dt = 0.000588
    speeds = (2.0, 4.0, 6.0, 25.0)
    dirs = (0.0, 30.0, -30.0, 45.0)
    vel = [(v * dt / pixel_m * math.cos(math.radians(a)), v * dt / pixel_m * math.sin(math.radians(a)))
           for v, a in zip(speeds, dirs)]
    return dict(n_modes=500, groups=(30, 70, 100, 300), gains=(0.55, 0.45, 0.40, 0.35),
                ff=(1.0, 0.999996, 0.999365, 0.977895), delay=2, cn2=(0.70, 0.06, 0.14, 0.10),
                r0_m=r0, L0_m=40.0, screen_px=1024, pixel_m=pixel_m, velocities_px=vel,
                origins_px=[(37.0 * i, 111.0 * i) for i in range(4)], seeds=(50, 51, 52, 53), dt_s=dt)


WORKLOADS = {
    "cfg1": _cfg1, "cfg2": _cfg2, "cfg3": _cfg3, "cfg4": _cfg4, "cfg5": _cfg5,
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]()


def band_sampling(center_nm: float, width_nm: float, n: int):
    """n wavelengths sampling a flat band by the midpoint rule: centres of n
    equal sub-bands, equal weights (a polychromatic sensor, Table 4's
    PolyCromPyramid; the weighting of the band is a reading, the paper gives
    none)."""
    lams = tuple(center_nm - width_nm / 2.0 + (i + 0.5) * width_nm / n for i in range(n))
    return lams, tuple([1.0 / n] * n)


def tiny_sensor(**kw) -> SensorDesc:
    """A sensor small enough for brute-force checks: D=8, N=16, 4 points, 2x2."""
    base = dict(n_pupil=8, n_fft=16, n_subap=2, n_mod=4, pupil_sep_px=8.0,
                mod_radius_lod=1.0, obstruction=0.0, diameter_m=8.0)
    base.update(kw)
    return SensorDesc(**base)
