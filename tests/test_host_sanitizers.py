"""The library's host code under AddressSanitizer (with leak detection) and
UndefinedBehaviorSanitizer, without a GPU: every source is built with the
sanitizers on its host side only (each -fsanitize after -Xarch_host; device
code is compiled as usual and never launched here), linked with
tests/host_sanitize.cpp, and run.  The harness packs plans of many shapes in
both precisions, sizes arenas and workspaces for every launch configuration,
round-trips factors and walks the argument errors; any sanitizer report or
wrong result fails the test."""
import concurrent.futures
import glob
import os
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
BUILD = ROOT / "_build" / "host_sanitize"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
CFLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", *SAN,
          "-Xarch_host", "-fno-omit-frame-pointer", "-Wno-unused-result", "-Wno-unused-value",
          "-I", str(ROOT / "include")]


def _compile(src: str) -> str:
    obj = BUILD / (os.path.basename(src) + ".o")
    deps = [src, *glob.glob(str(ROOT / "include" / "*.h")),
            *glob.glob(str(ROOT / "paper_2103_06393_amd" / "csrc" / "*.h"))]
    if obj.exists() and obj.stat().st_mtime > max(os.path.getmtime(d) for d in deps):
        return str(obj)
    r = subprocess.run([HIPCC, *CFLAGS, "-c", src, "-o", str(obj)], capture_output=True,
                       text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    return str(obj)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_code_under_address_and_ub_sanitizers():
    BUILD.mkdir(parents=True, exist_ok=True)
    srcs = sorted(glob.glob(str(ROOT / "paper_2103_06393_amd" / "csrc" / "*.hip")) +
                  glob.glob(str(ROOT / "paper_2103_06393_amd" / "csrc" / "*.cpp")))
    srcs.append(str(ROOT / "tests" / "host_sanitize.cpp"))
    jobs = max(1, min(8, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    exe = BUILD / "host_sanitize"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", *SAN, "-o", str(exe), *objs],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "0 failures" in out
    assert "runtime error" not in out and "ERROR: AddressSanitizer" not in out
