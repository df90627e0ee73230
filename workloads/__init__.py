"""Seeded synthetic inputs for the pyramid wavefront sensor workloads.

This package only *describes* sensors and *draws* inputs (phase screens,
tip/tilt jitter, modal coefficients).  It holds none of the sensor's own
arithmetic (pupil, modulation, pyramid mask, binning, slopes): that lives on
one side in the CPU oracle and on the other in the HIP library, which share
nothing but what is defined here.
"""

from .configs import (  # noqa: F401
    SensorDesc, Workload, WORKLOADS, workload, FLAG_REF_SLOPES, FLAG_FULL_PLANE,
    FLAG_LOCAL_NORM, FLAG_DOUBLE_ROOF, PREC_FP32, PREC_BF16, PREC_BF16X3, PREC_FP16X3, PREC_FP16, tiny_sensor, band_sampling,
)
from .screens import (  # noqa: F401
    von_karman_opd, jitter_opd, tilt_opd, workload_opd,
)
