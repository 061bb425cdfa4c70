"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the plan's parameter code (csrc/nr_params.cpp) with a driver over its whole
domain, the plan code (csrc/nr_plan.cpp, host parts only, up to its first
device allocation) planning the 1 h workload, and the C oracle exercised
through its Python binding's calls."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _need_gcc():
    if not shutil.which("g++") or not shutil.which("gcc"):
        pytest.skip("no host compiler")


def test_params_code_is_clean_under_asan_ubsan(tmp_path):
    _need_gcc()
    exe = tmp_path / "params_driver"
    csrc = os.path.join(ROOT, "paper_2609_12476_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", *SAN, "-I", csrc, os.path.join(ROOT, "tests", "host", "params_driver.cpp"),
                    os.path.join(csrc, "nr_params.cpp"), "-o", str(exe)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


ORACLE_SCRIPT = r"""
import numpy as np, sys
sys.path.insert(0, {root!r})
import oracle, synth
oracle._LIB = {lib!r}
w = synth.semicoherent(hours=0.02, n_mc=2, n_sub=2, seed=3)
X, off, ok = oracle.spectra(w)
S, soff, used = oracle.semicoherent(w)
X1, v = oracle.spectrum(np.random.default_rng(1).standard_normal(37), 64.0, 0.0, 1e-2, 50.0, 40.0, 0.5, 9)
d = oracle.dtau(1e-2, 50.0, 0.0, 256.0, 100)
assert np.all(np.isfinite(X)) and np.all(np.isfinite(S)) and np.all(np.isfinite(d))
print("oracle ok", X.size, S.size)
"""


def test_oracle_is_clean_under_asan_ubsan(tmp_path):
    _need_gcc()
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", *SAN, os.path.join(ROOT, "oracle", "nr_oracle.c"),
                    "-o", str(lib), "-lquadmath", "-lm"], check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("libasan not found")
    env = dict(os.environ, LD_PRELOAD=" ".join(p for p in (asan, ubsan) if os.path.isabs(p)),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", ORACLE_SCRIPT.format(root=ROOT, lib=str(lib))], capture_output=True,
                       text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "oracle ok" in r.stdout
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr


def test_plan_host_code_is_clean_under_asan_ubsan(tmp_path):
    """nr_plan.cpp built by hipcc with the sanitizers on the host side only
    (device code is never instrumented), linked with the library's other
    objects as built by build()."""
    _need_gcc()
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/lib/llvm/bin/clang++"
    objs = [os.path.join(ROOT, "paper_2609_12476_amd", "_build", f) for f in ("nr_kernels.hip.o", "nr_static.hip.o")]
    if not (os.path.exists(hipcc) and os.path.exists(clang) and all(os.path.exists(o) for o in objs)):
        pytest.skip("hipcc or the library's objects are missing")
    csrc = os.path.join(ROOT, "paper_2609_12476_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    for src in ("nr_plan.cpp", "nr_params.cpp"):
        subprocess.run([hipcc, "-x", "hip", "-c", os.path.join(csrc, src), "-o", str(tmp_path / (src + ".o")), "-O1",
                        "-g", "-fPIC", "-std=c++17", "--offload-arch=gfx950", *host_san, "-I", inc], check=True,
                       capture_output=True)
    subprocess.run(["g++", "-std=c++17", *SAN, "-I", inc, "-c", os.path.join(ROOT, "tests", "host", "plan_driver.cpp"),
                    "-o", str(tmp_path / "drv.o")], check=True)
    exe = tmp_path / "plan_driver"
    subprocess.run([clang, "--hip-link", "--offload-arch=gfx950", str(tmp_path / "drv.o"),
                    str(tmp_path / "nr_plan.cpp.o"), str(tmp_path / "nr_params.cpp.o"), *objs,
                    "-fsanitize=address,undefined", "-L/opt/rocm/lib", "-lamdhip64", "-o", str(exe)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "0 unexpected statuses" in r.stdout
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
