"""The C ABI's host code under AddressSanitizer (no GPU needed): the API
source is rebuilt with the sanitizer on its host pass only, linked with the
library's other objects and a driver that calls every entry point on
exactly-sized heap buffers; the driver must report no status mismatch and
the sanitizer no memory error."""
import os
import shutil
import subprocess

import pytest

from paper_2505_03269_amd import build as libbuild

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2505_03269_amd", "csrc")

pytestmark = pytest.mark.skipif(not os.path.exists(libbuild.HIPCC) and shutil.which("hipcc") is None,
                                reason="no hipcc")


def test_host_abi_under_address_sanitizer(tmp_path):
    objs = [os.path.join(libbuild.BUILD, f) for f in sorted(os.listdir(libbuild.BUILD))
            if f.endswith(".hip.o") and f != "tcbf_api.hip.o"] if os.path.isdir(libbuild.BUILD) else []
    if len(objs) < 5:
        libbuild.build()
        objs = [os.path.join(libbuild.BUILD, f) for f in sorted(os.listdir(libbuild.BUILD))
                if f.endswith(".hip.o") and f != "tcbf_api.hip.o"]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    api = str(tmp_path / "tcbf_api_asan.o")
    drv = str(tmp_path / "driver.o")
    exe = str(tmp_path / "host_abi_asan")
    steps = [
        [libbuild.HIPCC] + libbuild.FLAGS + san + ["-c", os.path.join(CSRC, "tcbf_api.hip"), "-o", api],
        [libbuild.HIPCC, "-std=c++17", "-O1", "-I" + libbuild.INCLUDE] + san +
        ["-c", os.path.join(HERE, "host_asan_driver.cpp"), "-o", drv],
        [libbuild.HIPCC, "--offload-arch=gfx950"] + san + [api, drv] + objs + ["-o", exe],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=99")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0 and "0 mismatches" in r.stdout, out[-4000:]
