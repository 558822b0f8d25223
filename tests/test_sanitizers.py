"""The library's host-only code (host.cpp: validation, packing, launch planning,
threshold rows) and the oracle, built with AddressSanitizer and
UndefinedBehaviorSanitizer by the host compiler and run on the CPU.  Any
out-of-bounds access, leak, overflow of a signed integer or other undefined
behaviour aborts the run."""
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_1004_0024_amd", "csrc")
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe, **env):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=dict(ENV, **env))
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    return r.stdout


def test_host_planning_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_check")
    subprocess.run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", CSRC,
                    os.path.join(CSRC, "host.cpp"), os.path.join(NATIVE, "host_check.cpp"), "-o", exe],
                   check=True, capture_output=True, text=True)
    out = _run(exe)
    assert "host_check OK" in out
    lim = {m.group(1): int(m.group(2)) for m in re.finditer(r"^(\w+) systems .* sweep_limit (\d+)", out, re.M)}
    # 2^32 - 1 flips of one 32,768-spin walker: 131,071 sweeps per launch
    assert lim["B"] == (2 ** 32 - 1) // 32768
    # 4,096 spins in 32 slices, one column per thread: a lane's |2 sum d| grows by at
    # most 2 * 63 * 32 per sweep, which binds before the flips do
    assert lim["C"] == min((2 ** 32 - 1) // 4096, (2 ** 31 - 1) // (2 * 63 * 32))
    assert all(v >= 1 for v in lim.values())
    assert out.count("reject ") == 10
    # ISING_LAUNCH_SWEEPS_MAX lowers both limits (a value below 1 is ignored)
    out = _run(exe, ISING_LAUNCH_SWEEPS_MAX="3")
    pairs = {m.group(1): (int(m.group(2)), int(m.group(3)))
             for m in re.finditer(r"^(\w+) systems .* sweep_limit (\d+) pairs_limit (\d+)", out, re.M)}
    assert pairs.keys() == lim.keys() and all(v == (3, 3) for v in pairs.values())
    out = _run(exe, ISING_LAUNCH_SWEEPS_MAX="0")
    assert {m.group(1): int(m.group(2)) for m in re.finditer(r"^(\w+) systems .* sweep_limit (\d+)", out, re.M)} == lim


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    subprocess.run(["gcc", "-std=c11", *SAN, "-ffp-contract=off", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "oracle", "orc.c"), os.path.join(NATIVE, "oracle_check.c"), "-o", exe,
                    "-lm", "-lpthread"], check=True, capture_output=True, text=True)
    assert "oracle_check OK" in _run(exe)

