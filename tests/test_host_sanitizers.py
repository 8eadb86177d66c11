"""The library's host planning code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only, no GPU): ``tests/host/planner_sanitize.cpp``
is linked with the host parts of api.hip, batch.hip and se8.hip, built with
the sanitizers on the host side only, and drives geometry, stage and launch
planning, batch planning and the argument checks over extreme sizes, widths
and depths.  A report from either sanitizer fails the test."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1803_04880_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_planners_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    flags = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fno-gpu-sanitize",
             "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    srcs = [os.path.join(CSRC, f) for f in ("api.hip", "batch.hip", "se8.hip")]
    srcs.append(os.path.join(ROOT, "tests", "host", "planner_sanitize.cpp"))
    objs, procs = [], []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        procs.append(subprocess.Popen([HIPCC] + flags + lang + ["-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    for p in procs:
        out = p.communicate()[0].decode(errors="replace")
        assert p.returncode == 0, out
    exe = str(tmp_path / "planner_sanitize")
    link = subprocess.run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                           "-fsanitize=undefined", "-o", exe] + objs,
                          capture_output=True, text=True)
    assert link.returncode == 0, link.stdout + link.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               HIP_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, run.stdout[-4000:] + run.stderr[-4000:]
    assert "failures" in run.stdout and "ERROR: AddressSanitizer" not in run.stderr
    assert "runtime error" not in run.stderr
