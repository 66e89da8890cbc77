"""The host code of the C ABI under AddressSanitizer (CPU only).

The driver source is compiled with its host pass instrumented (hipcc's
-Xarch_host), linked with the other objects of the normal build into a
separate library, and exercised by tests/asan_driver.cpp: argument and option
validation, NULL contexts and dmpt_init's failure path, all of which return
before any device work.  Any ASan report (out-of-bounds access, use after
free, leak in the library's own code) fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1503_07037_amd", "csrc")
INC = os.path.join(ROOT, "include")


def _tools():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("hipcc / ROCm clang++ not available")
    return hipcc, clang


@pytest.mark.timeout(600)
def test_abi_host_paths_under_asan(tmp_path):
    hipcc, clang = _tools()
    from paper_1503_07037_amd import build as B
    objs = [os.path.join(B.BUILD_DIR, s.replace(".hip", ".o")) for s in B.SOURCES if s != "dmpt_api.hip"]
    if not all(os.path.exists(o) for o in objs):
        B.build()
    api = str(tmp_path / "dmpt_api_asan.o")
    lib = str(tmp_path / "libdmpt_asan.so")
    exe = str(tmp_path / "asan_driver")
    flags = [f for f in B.FLAGS if f not in ("-O3",)]
    subprocess.run([hipcc, *flags, "-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                    "-fno-omit-frame-pointer", "-c", os.path.join(CSRC, "dmpt_api.hip"), "-o", api],
                   check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    subprocess.run([hipcc, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", api, *objs, "-Xarch_host",
                    "-fsanitize=address", *B.LINK, "-o", lib],
                   check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    subprocess.run([clang, "-g", "-fsanitize=address", "-I", INC, os.path.join(ROOT, "tests", "asan_driver.cpp"),
                    "-L", str(tmp_path), "-ldmpt_asan", "-Wl,-rpath," + str(tmp_path), "-o", exe],
                   check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    nm = shutil.which("nm")
    if nm:  # the library's host code really is instrumented
        syms = subprocess.run([nm, "-D", lib], stdout=subprocess.PIPE, text=True).stdout
        assert "__asan_report" in syms
    supp = tmp_path / "lsan.supp"
    # allocations the HIP / HSA runtimes keep until exit are theirs, not the library's
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libhsakmt\nleak:librocprofiler\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               LSAN_OPTIONS=f"suppressions={supp}")
    p = subprocess.run([exe], env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    print(p.stdout[-4000:])
    assert "ERROR: AddressSanitizer" not in p.stdout and "ERROR: LeakSanitizer" not in p.stdout
    assert p.returncode == 0 and "asan driver: ok" in p.stdout
