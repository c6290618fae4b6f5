"""The CPU debug preset: host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

* tests/host/geometry_check.cpp with topology.cpp: the decomposition and tile-layout invariants
  (every upper-triangle entry of a block stored once, lines aligned, symmetric neighbour tables,
  owners), built with -fsanitize=address,undefined and no recovery, so any report fails the run.
* tests/host/xcd_check.cpp: the XCD-contiguous work-group numbering (xcd.h) is a bijection whose
  per-XCD shares are contiguous ranges, for every grid size up to 20,000 work-groups.
* the debug build of libsfm.so (SFM_DEBUG launch checks, host code sanitized, build_lib
  debug=True) loads and runs the configuration checks of sfm_create with the sanitizer runtime
  preloaded.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1406_6923_amd", "csrc")


def _compiler():
    for cxx in ("g++", "/opt/rocm/llvm/bin/clang++"):
        if shutil.which(cxx):
            return cxx
    pytest.skip("no host C++ compiler")


def test_geometry_under_sanitizers(tmp_path):
    exe = tmp_path / "geometry_check"
    cmd = [_compiler(), "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           os.path.join(ROOT, "tests", "host", "geometry_check.cpp"), "-x", "c++", os.path.join(CSRC, "topology.cpp"),
           "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "geometry checks passed" in res.stdout


def test_xcd_numbering_under_sanitizers(tmp_path):
    """The work-group renumbering of the build stencil and the FDTD comparator: a bijection for
    every grid size, each XCD's round-robin share mapped to one contiguous range."""
    exe = tmp_path / "xcd_check"
    cmd = [_compiler(), "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", os.path.join(ROOT, "tests", "host", "xcd_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-2000:]
    assert "xcd numbering checks passed" in res.stdout


def _asan_runtime():
    res = subprocess.run(["/opt/rocm/llvm/bin/clang++", "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = res.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_debug_library_config_checks_under_sanitizers():
    from paper_1406_6923_amd import build_lib
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime for the HIP compiler")
    lib = build_lib.build(debug=True)
    script = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1406_6923_amd import sfm\n"
        "sfm.load_library(%r)\n"
        "bad = [dict(ncell=(32, 32, 30)), dict(m=0), dict(k=1), dict(h=0.0), dict(m=25, ncell=(8, 8, 8), sub=(4, 4, 4)),\n"
        "       dict(m=4, k=300), dict(precision=7), dict(sub=((12, 16), 16, 16))]\n"
        "for kw in bad:\n"
        "    a = dict(ncell=(32, 32, 32), sub=(16, 16, 16), h=10.0, m=4, k=8, precision=0); a.update(kw)\n"
        "    try:\n"
        "        sfm.sfm_create(a['ncell'], a['sub'], a['h'], a['m'], a['k'], a['precision'])\n"
        "    except sfm.SfmError as e:\n"
        "        assert e.status == sfm.SFM_EINVAL, (kw, e)\n"
        "    else:\n"
        "        raise AssertionError(kw)\n"
        "print('debug library checks passed')\n" % (ROOT, lib))
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1", HIP_VISIBLE_DEVICES="")
    res = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "debug library checks passed" in res.stdout
