"""Host C++ of the library under AddressSanitizer and UndefinedBehaviorSanitizer
(no device work): the library's host sources are rebuilt with both
sanitizers on their host code and linked into a driver that builds trees,
runs the multi-threaded traversal and host plans on several handles from
several threads at once, exports structures, builds BIE and curved-element
handles, drives the server's host half and the argument checks
(tests/sanitize/host_driver.cpp).  Any sanitizer report fails the test."""
import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1803_09948_amd import build as B  # noqa: E402

pytestmark = pytest.mark.slow

# sanitizers apply to host code only (each flag behind -Xarch_host)
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-3000:] + r.stderr[-3000:]


def test_host_code_under_asan_ubsan():
    hip = os.path.exists(B.HIPCC)
    if not hip:
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        csrc = B.CSRC
        hips = sorted(glob.glob(os.path.join(csrc, "*.hip")))
        cpps = sorted(glob.glob(os.path.join(csrc, "*.cpp")))

        def one(src):
            obj = os.path.join(d, os.path.basename(src) + ".o")
            if src.endswith(".hip"):   # device code unchanged, host part sanitized
                cmd = [B.HIPCC, *B.COMMON, *B.DEVICE, *SAN, "-O1", "-x", "hip", "-c", src, "-o", obj]
            else:
                cmd = [B.HIPCC, *B.COMMON, *SAN, "-O1", "-D__HIP_PLATFORM_AMD__", "-c", src, "-o", obj]
            _run(cmd)
            return obj

        with ThreadPoolExecutor(8) as ex:
            objs = list(ex.map(one, hips + cpps + [os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp")]))
        exe = os.path.join(d, "host_driver")
        _run([B.HIPCC, f"--offload-arch={B.ARCH}", *SAN, "-o", exe, *objs, "-lamdhip64", "-lpthread"])
        # inputs: points on an ellipsoid, a flat icosphere, a curved icosphere
        x = synth.scale_axes(synth.sphere_points(60000, 9), (1.0, 0.7, 1.3)).astype(np.float32)
        V, T = synth.icosphere(3)
        N6, T6 = synth.curved_icosphere(2)
        files = []
        for name, arr in (("p.f32", x), ("v.f64", np.asarray(V, np.float64)), ("t.i32", np.asarray(T, np.int32)),
                          ("n6.f64", np.asarray(N6, np.float64)), ("t6.i32", np.asarray(T6, np.int32))):
            path = os.path.join(d, name)
            np.ascontiguousarray(arr).tofile(path)
            files.append(path)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
        r = subprocess.run([exe, *files], capture_output=True, text=True, env=env, timeout=600)
        out = r.stdout + r.stderr
        print(out[-4000:])
        assert "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out
        assert r.returncode == 0 and "host driver: ok" in out
