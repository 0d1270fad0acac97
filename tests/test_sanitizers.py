"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU code:
the oracle (every function on a small box) and the library's host code
(validation, creation without a device, the tile cache, the no-allocation
entry point's checks).  Device code is built without sanitizers: only the
host pass of hipcc gets them (-Xarch_host)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", *SAN, os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "rbe_oracle.c"), "-o", exe, "-lm"])
    r = _run([exe], env=ENV)
    assert "oracle driver: ok" in r.stdout


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_host_library_under_sanitizers(tmp_path):
    from paper_2010_01559_amd import build as B
    hipcc = B.hipcc()
    host_san = [a for flag in SAN for a in ("-Xarch_host", flag)]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", B.CSRC]
    objs = []
    for src in B.SOURCES:
        obj = str(tmp_path / (src + ".o"))
        # the host code with sanitizers, device code as in the library
        _run([hipcc, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", *host_san, *inc, "-x", "hip", "-c", os.path.join(B.CSRC, src), "-o",
              obj])
        objs.append(obj)
    drv = str(tmp_path / "host_driver.o")
    _run([hipcc, "-O1", "-g", *host_san, *inc, "-x", "c", "-c", os.path.join(HERE, "host_driver.c"), "-o", drv])
    exe = str(tmp_path / "host_driver")
    _run([hipcc, "--offload-arch=gfx950", *host_san, drv, *objs, "-o", exe])
    env = dict(ENV, RBE_TUNE_CACHE=str(tmp_path / "no_cache.txt"))
    r = _run([exe], env=env)
    assert "host driver: ok" in r.stdout
