"""Address and undefined-behaviour sanitizers on the host code (CPU only).

1. The plain C parts, the oracle and the power-law sampler, built with gcc
   -fsanitize=address,undefined into tests/sanitize/host_c_paths.c, which runs
   the oracle's solver in every check mode and shift policy, its metrics and
   the sampler on small tall, wide and square inputs.
2. The library's host-only paths, the driver built with the sanitizers on its
   host half (-Xarch_host: device code is untouched): argument checks, the
   measuring pass that lays out the arena of a solve and of a batch (the
   layout the real run then takes buffer by buffer), status strings and the
   failure of dashsvd_create without a device
   (tests/sanitize/host_driver_paths.cpp).

Any out-of-bounds access, use after free or undefined operation aborts the
harness with the sanitizer's report, and the test fails with it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2404_09276_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr[-4000:]}"
    return r.stdout


def test_oracle_and_sampler_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_c_paths")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-fno-sanitize-recover=all", "-o", exe, os.path.join(SAN, "host_c_paths.c"),
          os.path.join(ROOT, "oracle", "dashsvd_oracle.c"), os.path.join(ROOT, "synth", "zipf_gen.c"), "-lm"])
    out = _run([exe], env=ENV, timeout=300)
    assert out.count("case ") == 4


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_driver_host_paths_under_asan_ubsan(tmp_path):
    from paper_2404_09276_amd import build as hip_build
    flags = ["--offload-arch=gfx950", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Wno-unused-result"]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
           "-fno-omit-frame-pointer"]
    procs, objs = [], []
    for src in hip_build.SOURCES:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        objs.append(obj)
        extra = ["-O1", "-g"] + san if src == "driver.hip" else ["-O1"]
        procs.append(subprocess.Popen([HIPCC, *flags, *extra, "-c", os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    main_obj = str(tmp_path / "main.o")
    objs.append(main_obj)
    procs.append(subprocess.Popen([HIPCC, "-std=c++17", "-O1", "-g", *san, "-I", os.path.join(ROOT, "include"),
                                   "-c", os.path.join(SAN, "host_driver_paths.cpp"), "-o", main_obj],
                                  stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out[-4000:]
    exe = str(tmp_path / "host_driver")
    _run([HIPCC, "--offload-arch=gfx950", *san[:4], "-o", exe, *objs])
    out = _run([exe], env=ENV, timeout=300)
    assert "host driver paths: ok" in out
    shutil.rmtree(str(tmp_path), ignore_errors=True)
