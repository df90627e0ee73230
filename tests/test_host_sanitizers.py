"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Every source of the library is compiled for the host only (no device code)
with both sanitizers, and linked with tests/host_abi/hip_stub.cpp, a stand-in
for the HIP runtime that treats device memory as host memory and checks each
launch configuration.  tests/host_abi/abi_driver.cpp then drives every entry
point of include/pwfs.h: plans for the workload sensors and the edge sensors
of the GPU tests (their float64 tables are written into host workspaces of
exactly the size pwfs_workspace_size reports, so a table that overran its
region would be an ASan report), every tuning, the detector, the
Shack-Hartmann sensor, the dense products, the network, the loop kernels,
and the error paths.  Runs on the CPU; needs hipcc only to compile.
"""

import ctypes
import os
import shutil
import struct
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "paper_2602_06688_amd", "csrc")
HOST = os.path.join(HERE, "host_abi")
BUILD = os.path.join(HOST, "_build")
SOURCES = ["pwfs_lib.hip", "pwfs_mfma.hip", "pwfs_mlp.hip", "pwfs_ccd.hip", "pwfs_loop.hip", "pwfs_sh.hip"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all"]


def _tool(name):
    for c in (os.path.join("/opt/rocm/bin", name), os.path.join("/opt/rocm/llvm/bin", name), shutil.which(name)):
        if c and os.path.exists(c):
            return c
    return None


def _build():
    hipcc, clang = _tool("hipcc"), _tool("clang++")
    if not hipcc or not clang:
        pytest.skip("hipcc / clang++ not available")
    os.makedirs(BUILD, exist_ok=True)
    cmds = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([hipcc, "-x", "hip", "--cuda-host-only", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                     *SAN, "-I", os.path.join(ROOT, "include"), "-I", SRC, "-c", os.path.join(SRC, src), "-o", obj])
    for src in ("hip_stub.cpp", "abi_driver.cpp"):
        obj = os.path.join(BUILD, src.replace(".cpp", ".o"))
        objs.append(obj)
        cmds.append([clang, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
                     "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
                     "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-c", os.path.join(HOST, src),
                     "-o", obj])
    procs = [subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT) for c in cmds]
    for c, p in zip(cmds, procs):
        out = p.communicate()[0].decode(errors="replace")
        assert p.returncode == 0, f"{' '.join(c)}\n{out}"
    # the host objects name each translation unit's (absent) device code object
    syms = set()
    for o in objs:
        r = subprocess.run(["nm", "-u", o], capture_output=True, text=True, check=True)
        syms |= {ln.split()[-1] for ln in r.stdout.splitlines() if "__hip_fatbin" in ln}
    fat = os.path.join(BUILD, "fatbin_names.c")
    with open(fat, "w") as f:
        for s in sorted(syms):
            f.write(f"const char {s}[16] = {{0}};\n")
    fobj = fat.replace(".c", ".o")
    subprocess.run([clang, "-x", "c", "-c", fat, "-o", fobj], check=True)
    exe = os.path.join(BUILD, "abi_driver")
    subprocess.run([clang, "-fsanitize=address,undefined", *objs, fobj, "-o", exe], check=True)
    return exe


def _descriptions(path):
    """Groups (sensors, frames) that abi_driver plans: the workloads' sensors in
    every precision, the six-sensor heterogeneous plan, and the GPU tests'
    edge sensors."""
    sys.path.insert(0, ROOT)
    from paper_2602_06688_amd import pwfs as P
    from workloads import (FLAG_DOUBLE_ROOF, FLAG_FULL_PLANE, FLAG_REF_SLOPES, band_sampling, tiny_sensor,
                           workload)
    c1 = workload("cfg1").sensors[0]
    c2 = workload("cfg2").sensors[0]
    groups = []
    for prec in (0, 1, 2, 3):
        groups.append(([c1.with_(precision=prec)], 5))
        groups.append(([c2.with_(precision=prec)], 3))
    groups.append((list(workload("cfg4").sensors), 2))
    groups.append(([c2.with_(flags=FLAG_DOUBLE_ROOF | FLAG_REF_SLOPES)], 2))
    lams, ws = band_sampling(750.0, 300.0, 16)
    groups.append(([c2.with_(lambdas_nm=lams, lambda_weights=ws)], 2))
    soul = tiny_sensor(n_pupil=220, n_fft=768, n_subap=40, pupil_sep_px=264.0, n_mod=24, mod_radius_lod=3.0,
                       diameter_m=8.222, fov_lod=2.0 / (750e-9 / 8.222 * 206264.806), flags=FLAG_REF_SLOPES)
    groups.append(([soul], 2))
    sys.path.insert(0, HERE)
    from test_gpu_pwfs import EDGE
    for s in EDGE.values():
        groups.append(([s], 3))
        groups.append(([s.with_(flags=s.flags | FLAG_FULL_PLANE)], 1))
    groups.append(([EDGE["N256"], EDGE["ragged_odd_mod"]], 2))
    with open(path, "wb") as f:
        f.write(struct.pack("<i", len(groups)))
        for sensors, frames in groups:
            f.write(struct.pack("<ii", len(sensors), frames))
            for s in sensors:
                f.write(bytes(P.to_c(s)))
    return len(groups)


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = _build()
    n = _descriptions(str(tmp_path / "descs.bin"))
    env = dict(os.environ)
    # verify_asan_link_order=0: the process may have preloaded libraries of its own
    env["ASAN_OPTIONS"] = ("detect_leaks=1:abort_on_error=0:halt_on_error=1:detect_stack_use_after_return=1:"
                           "verify_asan_link_order=0")
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe, str(tmp_path / "descs.bin")], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    print(out[-4000:])
    if "LeakSanitizer has encountered a fatal error" in out:
        # leak checking needs ptrace, which some containers deny: run again without it
        env["ASAN_OPTIONS"] = env["ASAN_OPTIONS"].replace("detect_leaks=1", "detect_leaks=0")
        r = subprocess.run([exe, str(tmp_path / "descs.bin")], capture_output=True, text=True, env=env, timeout=600)
        out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "ALL OK" in out
    assert "runtime error" not in out and "AddressSanitizer" not in out
    assert out.count(": ok") >= n
