"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

Builds every HIP source with the sanitizers on the host pass only (the
device code is compiled as usual and never runs here), links
tests/host_checks.cpp against the objects and runs it: sizes, option and
camera validation, the argument errors of every entry point, the schedule
and densification defaults -- the host checks of test_library.py, in a
program the sanitizers watch.  The build is cached in the package's _build
folder and redone when a source is newer than the program.
"""
import os
import shutil
import subprocess

import pytest

from paper_2406_02720_amd import build as BLD

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(BLD.BUILD, "sanitized")
EXE = os.path.join(OUT, "host_checks")
DRIVER = os.path.join(HERE, "host_checks.cpp")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
CLANG = "/opt/rocm/llvm/bin/clang++"


def _host_only(flags):
    """Sanitizer flags for the host pass of hipcc only."""
    out = []
    for f in flags:
        out += ["-Xarch_host", f]
    return out


def _stale(sources):
    if not os.path.exists(EXE):
        return True
    t = os.path.getmtime(EXE)
    return any(os.path.getmtime(s) > t for s in sources)


def _build():
    csrc = [os.path.join(BLD.CSRC, s) for s in BLD.SOURCES]
    headers = [os.path.join(BLD.CSRC, f) for f in os.listdir(BLD.CSRC) if f.endswith(".h")]
    headers.append(os.path.join(BLD.ROOT, "include", "hgs.h"))
    if not _stale(csrc + headers + [DRIVER]):
        return
    os.makedirs(OUT, exist_ok=True)
    cc = BLD.hipcc()
    objs, procs = [], []
    for src in csrc:
        obj = os.path.join(OUT, os.path.basename(src).replace(".hip", ".o"))
        objs.append(obj)
        cmd = [cc, *BLD.FLAGS, "-O1", *_host_only(SAN), "-c", src, "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out
    drv = os.path.join(OUT, "host_checks.o")
    subprocess.run([CLANG, "-std=c++17", "-O1", "-g", *SAN, "-D__HIP_PLATFORM_AMD__", "-I",
                    os.path.join(BLD.ROOT, "include"), "-I", "/opt/rocm/include", "-c", DRIVER, "-o", drv],
                   check=True)
    subprocess.run([CLANG, *SAN, "-o", EXE, drv, *objs, "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib"], check=True)


@pytest.mark.skipif(not (os.path.exists(CLANG) and shutil.which(BLD.hipcc())), reason="ROCm compilers missing")
def test_host_code_under_address_and_undefined_behaviour_sanitizers():
    _build()
    env = dict(os.environ)
    # leaks inside the HIP runtime's own start-up are not the library's
    supp = os.path.join(OUT, "lsan.supp")
    with open(supp, "w") as f:
        f.write("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libamd_comgr\n")
    env["ASAN_OPTIONS"] = "abort_on_error=0:halt_on_error=1:detect_leaks=1"
    env["LSAN_OPTIONS"] = f"suppressions={supp}"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([EXE], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks passed" in r.stdout
    assert "runtime error" not in r.stderr, r.stderr
