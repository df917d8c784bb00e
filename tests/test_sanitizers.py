"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (plain C), built with gcc -fsanitize=address,undefined, runs its
  operators, decomposition, solver (both linesearch norms, fixed step), adjoint and
  least-squares paths on small, ragged and degenerate gathers, and must give the
  same numbers as the normal build.
* The library's host code, built with hipcc with the sanitizers on the host side
  only (the GPU code is compiled as usual), runs the ABI contract tests: parameter
  and descriptor validation, error strings, the exported symbols.

Each runs in a child process with the sanitizer runtime preloaded; the first report
aborts the child, which fails the test.
"""
import glob
import json
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}

# the oracle calls the child makes; the parent makes the same calls on the normal build
CASES = r"""
import json, sys
import numpy as np
import oracle as O
from synth import config1_pairs, random_small_pair

out = {}
for (nr, nt, seed) in [(7, 13, 1), (1, 40, 2), (25, 1, 3), (1, 1, 4), (16, 33, 5)]:
    g = random_small_pair(nr, nt, seed)
    for mode in (O.MASS_BALANCE, O.MASS_UNIT, O.MASS_NONE):
        s, f, gg, mass = O.decompose(g.pcal, g.pobs, g.dx, g.dt, mass_mode=mode)
        out[f"mass {nr}x{nt} {mode}"] = mass.tolist()
    s, f, gg, mass = O.decompose(g.pcal, g.pobs, g.dx, g.dt)
    for ls in (O.LS_L2, O.LS_L1, O.LS_FIXED):
        r = O.solve(s, g.dx, g.dt, O.Params(tol_res=1e-6, max_iter=3000, ls_mode=ls), trace=True)
        out[f"solve {nr}x{nt} {ls}"] = [r.status, r.iters, r.ls_trials, r.emd, r.transport,
                                         float(np.abs(r.phi).sum()), float(r.alpha_trace.sum())]
    out[f"adjoint {nr}x{nt}"] = O.adjoint(r.phi, g.pcal, g.pobs, mass, g.dx, g.dt).tolist()
    out[f"lsd {nr}x{nt}"] = O.lsd(g.pcal, g.pobs, g.dx, g.dt)[0]
    gx, gt = O.grad(r.phi, g.dx, g.dt)
    out[f"grad {nr}x{nt}"] = [float(gx.sum()), float(gt.sum())]
    out[f"div {nr}x{nt}"] = float(np.abs(O.div(r.ux, r.ut, g.dx, g.dt)).sum())
z = np.zeros((4, 6))
out["zero"] = O.solve(z, 0.1, 0.1).status
bad = np.ones((4, 6)); bad[1, 2] = np.nan
out["nan"] = O.solve(bad, 0.1, 0.1).status
g = config1_pairs([40], nt=120, dt=1.0 / 119)[0]
s, _, _, _ = O.decompose(g.pcal, g.pobs, g.dx, g.dt)
out["1d"] = O.solve(s, g.dx, g.dt, O.Params(tol_res=1e-6, max_iter=50000)).emd
json.dump(out, sys.stdout)
"""


def _mapped(pid_maps: str, name: str) -> bool:
    return any(name in line for line in pid_maps.splitlines())


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call([gcc, "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-Wall",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-o", lib,
                           os.path.join(ROOT, "oracle", "emd_oracle.c"), "-lm"])
    check = CASES + "\nsys.stderr.write(open('/proc/self/maps').read())\n"
    env = dict(os.environ, EMD_ORACLE_LIB=lib, LD_PRELOAD=asan, PYTHONPATH=ROOT, **SAN_ENV)
    r = subprocess.run([sys.executable, "-c", check], capture_output=True, text=True, env=env,
                       cwd=ROOT, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert _mapped(r.stderr, "liboracle_san.so") and _mapped(r.stderr, "libasan")
    got = json.loads(r.stdout)
    # the same calls on the normal build, in a child without sanitizers
    r2 = subprocess.run([sys.executable, "-c", CASES], capture_output=True, text=True,
                        env=dict(os.environ, PYTHONPATH=ROOT), cwd=ROOT, timeout=600)
    assert r2.returncode == 0, r2.stderr[-4000:]
    ref = json.loads(r2.stdout)
    assert got.keys() == ref.keys()
    for k in ref:
        np.testing.assert_allclose(np.asarray(got[k], float), np.asarray(ref[k], float),
                                   rtol=1e-13, atol=0, err_msg=k)


def test_library_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not os.path.exists(hipcc) or not rts:
        pytest.skip("hipcc or clang's AddressSanitizer runtime is not installed")
    sys.path.insert(0, ROOT)
    from paper_1808_07284_amd import build as B
    flags = [f for f in B.HIPCC_FLAGS if f != "-O3"] + [
        "-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
        "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libasan"]
    procs, objs = [], []
    for src in B.SOURCES:
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([hipcc, *flags, "-c", os.path.join(B.CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err[-4000:]
    lib = str(tmp_path / "libemd_mi355x_san.so")
    subprocess.check_call([hipcc, "-shared", "-fPIC", f"--offload-arch={B.ARCH}", "-shared-libasan",
                           "-fsanitize=address,undefined", *objs, "-o", lib,
                           f"-L{B.ROCM_LIB}", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{B.ROCM_LIB}"])
    child = (
        "import os, sys, pytest\n"
        "code = pytest.main(['-x', '-q', '-p', 'no:cacheprovider', "
        f"{os.path.join(ROOT, 'tests', 'test_abi_contract.py')!r}])\n"
        "from paper_1808_07284_amd import _lib as L\n"
        "assert L.LIB_PATH == os.environ['EMD_MI355X_LIB'] and L._lib is not None\n"
        "sys.stderr.write(open('/proc/self/maps').read())\n"
        "sys.exit(int(code))\n")
    env = dict(os.environ, EMD_MI355X_LIB=lib, LD_PRELOAD=rts[-1], PYTHONPATH=ROOT, **SAN_ENV)
    r = subprocess.run([sys.executable, "-c", child], capture_output=True, text=True, env=env,
                       cwd=ROOT, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout
    assert _mapped(r.stderr, "libemd_mi355x_san.so") and _mapped(r.stderr, "libclang_rt.asan")


def test_tile_bookkeeping_under_sanitizers(tmp_path):
    # the host-only part of the solve's bookkeeping (csrc/emd_tiling.h: padded layout,
    # tile tables over the XCDs, chains, narrowing rule) on 300 random batches, built
    # with g++ and both sanitizers; every rule the sweep relies on is checked
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_tiling_check")
    subprocess.check_call([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-I", os.path.join(ROOT, "paper_1808_07284_amd", "csrc"),
                           os.path.join(ROOT, "tests", "host_tiling_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, env={**os.environ, **SAN_ENV}, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok: 300 batches")
