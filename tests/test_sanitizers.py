"""The C oracle and the library's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer (ROCm's clang, host only) and run on the CPU.

* oracle: the small elastic tube (LV inlet, Windkessel outlet, exterior,
  membrane with the shell terms, normal-neighbour extrapolation) and the
  rigid branched duct (two outlets with their own Windkessels), a few steps
  each through every entry point, then the standalone helpers; the leak
  checker is on.
* host code (csrc/lbm_api.cpp with its device launchers stubbed out): the
  geometry checks and buffer sizes of the elastic tube in every precision
  and extrapolation variant, a batch of two, and the rejections of bad
  inputs.  Nothing reaches the GPU.
Any sanitizer report fails the run.
"""
import os
import struct
import subprocess

import numpy as np
import pytest

import lbm_inputs as L

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CLANG = "/opt/rocm/llvm/bin/clang"
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")

pytestmark = pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists(CLANGXX)),
                                reason="ROCm clang not found")


def _oracle_input(path, c, steps, shell=0):
    nz, ny, nx = c["flags"].shape
    out = [struct.pack("3i", nx, ny, nz), np.ascontiguousarray(c["flags"], np.uint8).tobytes(),
           struct.pack("d", c["tau"]), struct.pack("i", c.get("nee_variant", 0))]
    bcs = [(0,) + tuple(c["inlet"])]
    if "outlet" in c:
        bcs.append((1,) + tuple(c["outlet"]))
    for k, ob in enumerate(c.get("outlets", [])):
        bcs.append((1 if k == 0 else 2 + k,) + tuple(ob))
    if "exterior" in c:
        bcs.append((2,) + tuple(c["exterior"]))
    out.append(struct.pack("i", len(bcs)))
    for b in bcs:
        boundary, kind, par = b[0], b[1], list(b[2])
        st = list(b[3]) if len(b) > 3 else ([c["outlet_state"][0]] if boundary == 1 and "outlet_state" in c else [])
        out.append(struct.pack("4i", boundary, kind, len(par), len(st)))
        out.append(struct.pack(f"{len(par)}d", *par) + struct.pack(f"{len(st)}d", *st))
    out.append(struct.pack("d", c.get("p_init", 0.0)))
    if "mesh" in c:
        m = c["mesh"]
        out.append(struct.pack("3i", 1, m["n_theta"], m["n_z"]))
        out.append(np.ascontiguousarray(m["X0"], np.float64).tobytes())
        out.append(struct.pack("8d", m["ds_theta"], m["ds_z"], m["area"], c["k"], c["ei"], c["mass"],
                               c["alpha"], c["beta"]))
        out.append(struct.pack("2id", c.get("kernel", 0), shell, 0.3))
    else:
        out.append(struct.pack("i", 0))
    out.append(struct.pack("i", steps))
    with open(path, "wb") as f:
        f.write(b"".join(out))


def _run(cmd, cwd):
    # the OpenMP runtime keeps one allocation of its thread pool to the end
    sup = os.path.join(cwd, "lsan.supp")
    with open(sup, "w") as f:
        f.write("leak:libomp.so\n")
    env = dict(ENV, LSAN_OPTIONS=f"suppressions={sup}:print_suppressions=0")
    r = subprocess.run(cmd, cwd=cwd, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-6000:])
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-6000:]
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.run([CLANG] + SAN + ["-fopenmp", "-std=c11", "-o", exe,
                                    os.path.join(HERE, "sanitize", "oracle_driver.c"),
                                    os.path.join(ROOT, "oracle", "lbm_oracle.c"), "-lm"],
                   check=True, capture_output=True, timeout=600)
    fsi = L.small_fsi()
    fsi["nee_variant"] = 1
    _oracle_input(str(tmp_path / "fsi.bin"), fsi, 12, shell=1)
    duct = L.branched_duct()
    _oracle_input(str(tmp_path / "duct.bin"), duct, 12)
    for name in ("fsi.bin", "duct.bin"):
        assert "oracle driver: ok" in _run([exe, str(tmp_path / name)], str(tmp_path))


def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2112_05258_amd", "csrc"),
           "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
    r = subprocess.run([CLANGXX] + SAN + ["-std=c++17"] + inc +
                       ["-o", exe, os.path.join(HERE, "sanitize", "host_driver.cpp"),
                        os.path.join(ROOT, "paper_2112_05258_amd", "csrc", "lbm_api.cpp"),
                        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    c = L.small_fsi()
    nz, ny, nx = c["flags"].shape
    with open(tmp_path / "flags.bin", "wb") as f:
        f.write(struct.pack("3i", nx, ny, nz) + np.ascontiguousarray(c["flags"], np.uint8).tobytes())
    assert "0 failure(s)" in _run([exe, str(tmp_path / "flags.bin")], str(tmp_path))
