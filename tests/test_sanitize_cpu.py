"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU side,
run on the CPU (no GPU needed): the C oracle under a driver that checks it
against a dense brute force on small shapes (empty rows, a full row, empty
operands), and the library's host code (its device code built as usual)
under a driver that exercises every entry point that touches host memory
only: status strings, descriptor checks, the batched plan, model
create/get/save/load with good and bad inputs, and the size queries."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1303_1651_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# every sanitizer flag applies to host code only
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, cwd, **kw):
    out = subprocess.run(cmd, cwd=cwd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, **kw)
    return out.returncode, out.stdout.decode(errors="replace")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    rc, log = _run(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", exe,
                    os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "spgemm_ref.c")], str(tmp_path))
    assert rc == 0, log
    rc, log = _run([exe], str(tmp_path), env=ENV)
    assert rc == 0 and "oracle driver: ok" in log, log


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc missing")
def test_host_abi_under_address_and_undefined_sanitizers(tmp_path):
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"] + SAN_HOST
    procs, objs = [], []
    for src in ("spgemm_kernels", "spgemm_host", "mlp", "batched", "transpose"):
        obj = str(tmp_path / (src + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, *flags, "-c", os.path.join(CSRC, src + ".hip"), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out.decode(errors="replace")
    drv = str(tmp_path / "host_driver.o")
    rc, log = _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", *SAN_HOST, "-x", "c++", "-c",
                    os.path.join(HERE, "host_driver.c"), "-o", drv], str(tmp_path))
    assert rc == 0, log
    exe = str(tmp_path / "host_driver")
    rc, log = _run([HIPCC, "--offload-arch=gfx950", *SAN_HOST, "-o", exe, drv, *objs], str(tmp_path))
    assert rc == 0, log
    rc, log = _run([exe, str(tmp_path)], str(tmp_path), env=ENV)
    assert rc == 0 and "host driver: ok" in log, log
