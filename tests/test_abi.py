"""The C ABI library loads, exports every symbol its header declares, and
its host-only entry points (validation, workspace sizing) behave.  No compute
call is made here: these run without a GPU."""

import ctypes
import os

import pytest

from paper_2602_06688_amd import pwfs as P
from workloads import band_sampling, tiny_sensor, workload


def test_library_exports_header_symbols():
    L = P.lib()
    syms = P.header_symbols()
    assert len(syms) >= 9
    for s in syms:
        assert hasattr(L, s), s


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg4"])
def test_workload_sensors_validate(name):
    w = workload(name)
    assert P.validate(w.sensors) == P.PWFS_OK
    assert P.workspace_size(w.sensors, w.n_frames) > 0


def _bad(**kw):
    return workload("cfg1").sensors[0].with_(**kw)


@pytest.mark.parametrize("kw,code", [
    (dict(n_fft=60), P.PWFS_EINVAL),                   # N < D
    (dict(n_fft=129), P.PWFS_EINVAL),                  # N - D odd
    (dict(n_subap=65), P.PWFS_EINVAL),                 # n_subap > D
    (dict(pupil_sep_px=66.0, n_fft=128), P.PWFS_EINVAL),   # images outside the grid
    (dict(pupil_sep_px=62.0), P.PWFS_EINVAL),          # images overlap
    (dict(pupil_sep_px=64.5), P.PWFS_EINVAL),          # non-integer separation
    (dict(n_mod=0), P.PWFS_EINVAL),
    (dict(lambdas_nm=(0.0,)), P.PWFS_EINVAL),
    (dict(lambdas_nm=(600.0, 900.0), lambda_weights=(0.5, 0.6)), P.PWFS_EINVAL),
    (dict(lambdas_nm=band_sampling(750.0, 300.0, 17)[0],                    # > 16 wavelengths
          lambda_weights=band_sampling(750.0, 300.0, 17)[1]), P.PWFS_EINVAL),
    (dict(obstruction=1.0), P.PWFS_EINVAL),
    (dict(mod_radius_lod=-1.0), P.PWFS_EINVAL),
    (dict(n_fft=160, pupil_sep_px=64.0), P.PWFS_EUNSUPPORTED),   # no radix plan
    (dict(flags=64), P.PWFS_EINVAL),
    (dict(src_rings=9, src_radius_lod=1.0), P.PWFS_EINVAL),
    (dict(src_rings=-1), P.PWFS_EINVAL),
    (dict(src_rings=2, src_radius_lod=-0.5), P.PWFS_EINVAL),
    (dict(src_rings=8, src_radius_lod=1.0, n_mod=64), P.PWFS_EINVAL),         # > 8192 points
    (dict(src_rings=1, src_radius_lod=1.0, precision=2), P.PWFS_EUNSUPPORTED),  # matrix-core form
    (dict(flags=9, precision=2), P.PWFS_EUNSUPPORTED),                           # double roof: FP32 only
    (dict(fov_lod=20.0, precision=2), P.PWFS_EUNSUPPORTED),                      # field stop: FP32 only
    (dict(fov_lod=-1.0), P.PWFS_EINVAL),
    (dict(flags=16), P.PWFS_EINVAL),
])
def test_validate_rejects(kw, code):
    assert P.validate([_bad(**kw)]) == code
    assert P.lib().pwfs_last_error().decode() != ""


def test_validate_accepts_edge_sensors():
    ok = [tiny_sensor(n_pupil=32, n_fft=64, n_subap=4, pupil_sep_px=32.0),
          tiny_sensor(n_pupil=40, n_fft=128, n_subap=5, pupil_sep_px=48.0, n_mod=1, mod_radius_lod=0.0),
          tiny_sensor(n_pupil=64, n_fft=128, n_subap=16, pupil_sep_px=64.0, n_mod=5,
                      lambdas_nm=(600.0, 750.0, 900.0, 1000.0), lambda_weights=(0.1, 0.2, 0.3, 0.4)),
          tiny_sensor(n_pupil=64, n_fft=128, n_subap=16, pupil_sep_px=64.0, n_mod=5,
                      lambdas_nm=band_sampling(750.0, 300.0, 16)[0],
                      lambda_weights=band_sampling(750.0, 300.0, 16)[1]),
          tiny_sensor(n_pupil=64, n_fft=128, n_subap=16, pupil_sep_px=64.0, n_mod=8, flags=9)]
    for s in ok:
        assert P.validate([s]) == P.PWFS_OK, P.lib().pwfs_last_error()


def test_null_and_count_arguments():
    L = P.lib()
    assert L.pwfs_validate(None, 1) == P.PWFS_EINVAL
    arr = (P.CSensorDesc * 1)(P.to_c(workload("cfg1").sensors[0]))
    assert L.pwfs_validate(arr, 0) == P.PWFS_EINVAL
    assert L.pwfs_workspace_size(arr, 1, 0, ctypes.byref(ctypes.c_size_t())) == P.PWFS_EINVAL
    assert L.pwfs_workspace_size(arr, 1, 10, None) == P.PWFS_EINVAL
    h = ctypes.c_void_p()
    # no workspace: rejected before any device work
    assert L.pwfs_plan(arr, 1, 10, None, 0, None, ctypes.byref(h)) == P.PWFS_EWORKSPACE
    # misaligned workspace pointer: rejected before any device work
    assert L.pwfs_plan(arr, 1, 10, ctypes.c_void_p(0x1001), 1 << 40, None, ctypes.byref(h)) == P.PWFS_EWORKSPACE
    # too small: rejected before any device work
    assert L.pwfs_plan(arr, 1, 10, ctypes.c_void_p(0x10000), 16, None, ctypes.byref(h)) == P.PWFS_EWORKSPACE
    assert L.pwfs_forward(None, None, 1, None, None) == P.PWFS_EINVAL
    assert L.pwfs_slopes(None, None, 1, None, None, None) == P.PWFS_EINVAL
    L.pwfs_destroy(None)


def test_workspace_grows_with_frames_and_flags():
    s = workload("cfg1").sensors[0]
    a = P.workspace_size([s], 10)
    b = P.workspace_size([s], 100)
    c = P.workspace_size([s.with_(flags=P.F_REF_SLOPES | P.F_FULL_PLANE)], 100)
    assert a < b <= c


def test_ctypes_structs_match_header_layout(tmp_path):
    """sizeof / offsetof of every C struct of include/pwfs.h (compiled with the
    host C compiler) against the binding's ctypes mirrors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"pwfs_sensor_desc": P.CSensorDesc, "pwfs_sensor_info": P.CSensorInfo, "pwfs_tuning": P.CTuning,
               "pwfs_ccd_desc": P.CCcdDesc, "pwfs_layer": P.CLayer, "pwfs_sh_desc": P.CShDesc}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pwfs.h"', 'int main(void) {']
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)


@pytest.mark.parametrize("kw,code", [
    (dict(n_pupil=160, n_subap=21), P.PWFS_EINVAL),        # D % n
    (dict(n_fft=56, rebin=5), P.PWFS_EINVAL),             # rebin does not divide n_fft
    (dict(n_pupil=660, n_subap=20), P.PWFS_EUNSUPPORTED),  # b = 33 > 32
    (dict(n_fft=600), P.PWFS_EINVAL),
    (dict(obstruction=1.0), P.PWFS_EINVAL),
    (dict(lambda_nm=0.0), P.PWFS_EINVAL),
    (dict(n_pupil=512, n_subap=16, n_fft=512, rebin=8), P.PWFS_EUNSUPPORTED),   # tables beyond the LDS
    (dict(lambdas_nm=[700.0, 800.0], lambda_weights=[0.5, 0.5]), P.PWFS_EINVAL),  # below the 750 nm reference
    (dict(lambdas_nm=[750.0, 800.0], lambda_weights=[0.5, 0.6]), P.PWFS_EINVAL),  # weights sum to 1.1
    (dict(lambdas_nm=[750.0] * 17, lambda_weights=[1 / 17] * 17), P.PWFS_EINVAL),  # more than 16
])
def test_sh_validate_rejects(kw, code):
    base = dict(n_pupil=160, n_subap=20, n_fft=56, rebin=7, obstruction=0.0, lambda_nm=750.0)
    base.update(kw)
    assert P.lib().pwfs_sh_validate(ctypes.byref(P.sh_desc(**base))) == code
    assert P.lib().pwfs_sh_validate(ctypes.byref(P.sh_desc(160, 20, 56, 7))) == P.PWFS_OK
