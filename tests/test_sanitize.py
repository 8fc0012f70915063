"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the oracle's C routines, libpd's host set-up routines, and the host paths of
libpd's C ABI (argument checks, workspace sizes, switches), each built into a
small executable with the sanitizers on the host code and run on small
inputs.  The device code is built as usual (no GPU work is done here)."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="verify_asan_link_order=0:detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")


def _run(exe, *args, timeout=300):
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=ENV, timeout=timeout)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), (r.returncode, r.stdout[-2000:], r.stderr[-4000:])


@pytest.fixture(scope="module")
def outdir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("sanitize"))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(outdir):
    exe = os.path.join(outdir, "oracle_driver")
    subprocess.check_call(["gcc", "-std=c11", "-fopenmp", *SAN, "-o", exe,
                           os.path.join(HERE, "sanitize", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    h = O.symmlet(6)
    kt, R = O.op1_profiles(16, 1.5)
    fh, fk = os.path.join(outdir, "h.txt"), os.path.join(outdir, "kt.txt")
    with open(fh, "w") as f:
        f.write(f"{len(h)} " + " ".join(repr(float(v)) for v in h) + "\n")
    with open(fk, "w") as f:
        f.write(f"{R} " + " ".join(repr(float(v)) for v in np.asarray(kt).ravel()) + "\n")
    _run(exe, fh, fk)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_setup_routines_under_sanitizers(outdir):
    exe = os.path.join(outdir, "setup_driver")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-o", exe,
                           os.path.join(HERE, "sanitize", "setup_driver.cpp"),
                           os.path.join(ROOT, "paper_2005_09870_amd", "csrc", "pd_setup.cpp")])
    _run(exe)


def test_abi_host_paths_under_sanitizers(outdir):
    from paper_2005_09870_amd import build as B
    if not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    # sanitizers on the host side only ("-Xarch_host" before each option)
    host_san = []
    for opt in SAN:
        host_san += ["-Xarch_host", opt]
    hosted = [s for s in B.SOURCES if s.endswith(".cpp")]
    devobjs = [os.path.join(B.OBJDIR, s + ".o") for s in B.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in devobjs):
        B.build(verbose=False)

    def one(src):
        obj = os.path.join(outdir, src + ".san.o")
        subprocess.check_call([B.HIPCC, *B.COMMON, *B.DEVICE_FLAGS, *host_san, "-x", "hip", "-c",
                               os.path.join(B.CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(len(hosted)) as ex:
        objs = list(ex.map(one, hosted))
    drv = os.path.join(outdir, "abi_driver.o")
    subprocess.check_call([B.HIPCC, "-std=c++17", *host_san, "-I", B.INCLUDE, "-c",
                           os.path.join(HERE, "sanitize", "abi_driver.cpp"), "-o", drv])
    exe = os.path.join(outdir, "abi_driver")
    subprocess.check_call([B.HIPCC, f"--offload-arch={B.ARCH}", "-fsanitize=address,undefined",
                           "-fno-gpu-sanitize", "-o", exe, drv, *objs, *devobjs])
    _run(exe)
