"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code:
the oracle's C loops (gcc, a standalone driver on a refined octahedron) and
the library's host runtime behind the C-ABI (hipcc with the sanitizers on
the host side only, a C++ driver that runs option validation, null
contexts and pbmp_create's quadrature set-up up to its first HIP call; on a
machine with a GPU the same driver also runs a small solve and backward).
CPU only: each build must run clean (exit 0, no sanitizer report)."""

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]


def _run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, **kw)
    return p.returncode, p.stdout + p.stderr


def test_oracle_c_loops_under_sanitizers(tmp_path):
    exe = str(tmp_path / "orc_san")
    rc, out = _run(["gcc", "-O1", "-g"] + SAN + ["-o", exe,
                    os.path.join(ROOT, "oracle", "sanitize_driver.c"),
                    os.path.join(ROOT, "oracle", "bie_c.c"), "-lm"])
    assert rc == 0, out
    rc, out = _run([exe], timeout=300)
    print(out)
    assert rc == 0 and "ERROR" not in out and "runtime error" not in out, out


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    # the sanitizers act on the host code only (each one after -Xarch_host)
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-fno-omit-frame-pointer"]
    flags = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + host_san
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_1810_03698_amd", "csrc", "*.cpp")) +
                  glob.glob(os.path.join(ROOT, "paper_1810_03698_amd", "csrc", "*.hip")))
    srcs.append(os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp"))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        rc, out = _run([hipcc] + flags + ["-c", src, "-o", obj])
        assert rc == 0, out
        return obj

    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "abi_san")
    rc, out = _run([hipcc, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-o", exe] + objs)
    assert rc == 0, out
    rc, out = _run([exe], timeout=600)
    print(out)
    assert rc == 0 and "ERROR" not in out and "runtime error" not in out, out
    assert "OK" in out
