"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

1. The oracle (``oracle/kco.c``) is rebuilt with both sanitizers and every
   oracle pin test runs against that build: any out-of-bounds access, use
   after free, signed overflow, bad shift or misaligned load in the oracle
   aborts the run.
2. The HIP library is rebuilt with both sanitizers on its host code only
   (device code is untouched), and the ABI tests, which drive the host-side
   checks without a device (range validation, default window, reachability,
   argument checks of every entry point that has them), run against it.

Each build goes to a temporary directory; the real builds are untouched.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_TESTS = ["tests/test_oracle_xxh64.py", "tests/test_oracle_snapshot.py", "tests/test_oracle_compare.py",
             "tests/test_oracle_graph.py", "tests/test_oracle_region.py", "tests/test_oracle_ragged.py",
             "tests/test_oracle_units.py", "tests/test_golden.py"]
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:protect_shadow_gap=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _runtime_gcc():
    if shutil.which("gcc") is None:
        return None
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _runtime_clang():
    hipcc = "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        return None
    res = subprocess.run([clang, "-print-resource-dir"], capture_output=True, text=True).stdout.strip()
    p = os.path.join(res, "lib", "linux", "libclang_rt.asan-x86_64.so")
    return p if os.path.exists(p) else None


def _run(cmd, preload, extra_env=None, timeout=900):
    env = dict(os.environ, LD_PRELOAD=preload, **SAN_ENV, **(extra_env or {}))
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-6000:]
    return out


def test_oracle_pins_under_sanitizers(tmp_path):
    rt = _runtime_gcc()
    if rt is None:
        pytest.skip("gcc with libasan is not available")
    lib = str(tmp_path / "libkco_san.so")
    san_flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fPIC", "-shared", "-ffp-contract=off", *san_flags,
                    "-o", lib, os.path.join(ROOT, "oracle", "kco.c"), "-lm"], check=True)
    out = _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *PIN_TESTS], rt,
               {"KCO_LIB": lib})
    assert " passed" in out


def test_library_host_code_under_sanitizers(tmp_path):
    rt = _runtime_clang()
    if rt is None:
        pytest.skip("hipcc / the clang sanitizer runtime is not available")
    sys.path.insert(0, ROOT)
    from paper_2605_03208_amd import build as B
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all"]
    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g"] + host_san
    objs = []
    procs = []
    for src in B.SOURCES:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([B.hipcc(), *flags, "-c", os.path.join(B.CSRC, src), "-o", obj],
                                      stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
    for p in procs:
        _, err = p.communicate(timeout=600)
        assert p.returncode == 0, err.decode()[-4000:]
    lib = str(tmp_path / "libkc_san.so")
    subprocess.run([B.hipcc(), f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *host_san, "-o", lib, *objs],
                   check=True, capture_output=True)
    code = ("import sys; sys.path.insert(0, '.'); import paper_2605_03208_amd.kc as K; "
            f"K.LIB_PATH = {lib!r}; import pytest; "
            "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', 'tests/test_abi.py']))")
    out = _run([sys.executable, "-c", code], rt)
    assert " passed" in out
