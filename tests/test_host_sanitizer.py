"""The host side of the library (tree builder, table planning, leaf layout, the C ABI's
argument handling) built with AddressSanitizer (host code only; leak detection on) and
driven through randomised trees by tests/native/tree_fuzz.cpp.  No GPU is used."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
KOBJ = os.path.join(ROOT, "paper_1901_11370_amd", "_build", "mg_kernels.hip.o")


@pytest.mark.skipif(not os.path.exists(HIPCC) or not os.path.exists(KOBJ),
                    reason="needs hipcc and the built kernel object (run the build first)")
def test_host_code_under_address_sanitizer():
    csrc = os.path.join(ROOT, "paper_1901_11370_amd", "csrc")
    flags = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-Xarch_host", "-fsanitize=address"]
    tmp = tempfile.mkdtemp(prefix="mg_asan_")
    try:
        objs = []
        for src in (os.path.join(csrc, "tree.cpp"), os.path.join(csrc, "mg_api.cpp"),
                    os.path.join(ROOT, "tests", "native", "tree_fuzz.cpp")):
            o = os.path.join(tmp, os.path.basename(src) + ".o")
            subprocess.check_call(flags + ["-c", src, "-o", o])
            objs.append(o)
        exe = os.path.join(tmp, "tree_fuzz")
        subprocess.check_call(flags + objs + [KOBJ, "-o", exe])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
        r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
        print(r.stdout, r.stderr[-2000:])
        assert r.returncode == 0 and "ERROR: AddressSanitizer" not in r.stderr
        assert "rejected 0 " in r.stdout
        n, s = [int(x) for x in r.stdout.split()[1::2][:1] + r.stdout.split()[-1:]]
        assert n + s == 300 and n >= 200
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
