"""CPU sanitizer tier: the library's host code and the oracle built with
AddressSanitizer + UndefinedBehaviorSanitizer, the serving runtime with
ThreadSanitizer, each run in a subprocess on this machine (no GPU).

- The host code (C ABI argument checks, tuning table, batch preparation,
  host co-rank, the serving runtime) is linked with tests/sanitize/hip_stub.cpp
  (the HIP runtime calls it makes, completing at once on host memory) and
  tests/sanitize/launch_stub.cpp (kernel launches that do nothing), and
  driven by tests/sanitize/host_driver.cpp; under ThreadSanitizer several
  client threads submit, poll and release while the scheduler thread runs.
- The oracle (oracle/oracle.c) is driven by tests/sanitize/oracle_driver.c.
- The serving arena's ring allocator is run through random sequences by the
  driver of tests/test_ring_alloc.py.

Every run must exit 0 with no sanitizer report.  Built with the ROCm LLVM
clang (its ThreadSanitizer runtime intercepts the timed condition-variable
waits the scheduler uses); nothing here touches a GPU."""
import os
import random
import subprocess
import concurrent.futures

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1303_4312_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang"
CLANGXX = "/opt/rocm/llvm/bin/clang++"
ROCM_INCLUDE = "/opt/rocm/include"

pytestmark = pytest.mark.skipif(not (os.path.exists(CLANGXX) and os.path.isdir(ROCM_INCLUDE)),
                                reason="needs the ROCm LLVM clang and HIP headers")

ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
TSAN = ["-fsanitize=thread"]
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer",
           "ERROR: LeakSanitizer")


def host_sources():
    return [os.path.join(CSRC, f) for f in ("api.cpp", "host_co_rank.cpp", "server.cpp")] + [
        os.path.join(SAN, f) for f in ("hip_stub.cpp", "launch_stub.cpp", "host_driver.cpp")]


def host_command(flags, exe):
    return [CLANGXX, "-std=c++17", "-O1", "-g", *flags, "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE,
            "-I", os.path.join(ROOT, "include"), "-I", CSRC, '-DCM_BUILD_ID="sanitize"',
            *host_sources(), "-pthread", "-o", exe]


@pytest.fixture(scope="module")
def programs(tmp_path_factory):
    d = tmp_path_factory.mktemp("sanitize")
    from tests.test_ring_alloc import DRIVER
    ring_src = d / "ring.cpp"
    ring_src.write_text(DRIVER.replace("#include <stdio.h>", "#include <stdio.h>\n#include <stdlib.h>"))
    exes = {name: str(d / name) for name in ("host_asan", "host_tsan", "oracle_asan", "ring_asan")}
    cmds = {
        "host_asan": host_command(ASAN, exes["host_asan"]),
        "host_tsan": host_command(TSAN, exes["host_tsan"]),
        "oracle_asan": [CLANG, "-O1", "-g", *ASAN, os.path.join(ROOT, "oracle", "oracle.c"),
                        os.path.join(SAN, "oracle_driver.c"), "-o", exes["oracle_asan"]],
        "ring_asan": [CLANGXX, "-std=c++17", "-O1", "-g", *ASAN, "-I", CSRC, str(ring_src), "-o",
                      exes["ring_asan"]],
    }
    with concurrent.futures.ThreadPoolExecutor(4) as pool:
        runs = dict(zip(cmds, pool.map(
            lambda c: subprocess.run(c, capture_output=True, text=True, timeout=600), cmds.values())))
    for name, r in runs.items():
        assert r.returncode == 0, f"building {name} failed:\n{r.stderr[-4000:]}"
    return exes


def run_clean(cmd, stdin=None, timeout=300):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", TSAN_OPTIONS="halt_on_error=0")
    r = subprocess.run(cmd, input=stdin, capture_output=True, text=True, timeout=timeout, env=env)
    text = r.stdout + r.stderr
    assert not any(k in text for k in REPORTS), text[-6000:]
    assert r.returncode == 0, text[-6000:]
    return r.stdout


def test_host_code_under_asan_ubsan(programs):
    out = run_clean([programs["host_asan"]])
    assert "host driver: 0 failed checks" in out
    assert "reported once each" in out


def test_server_scheduler_under_tsan(programs):
    out = run_clean([programs["host_tsan"], "threads"])
    assert "900 requests from 6 client threads reported once each" in out


def test_oracle_under_asan_ubsan(programs):
    assert "0 failures" in run_clean([programs["oracle_asan"]])


def test_ring_allocator_under_asan_ubsan(programs):
    rng = random.Random(5)
    size = 256 * 64
    ops, live, nxt = [], [], 0
    for _ in range(4000):
        if live and rng.random() < 0.45:
            ops.append(f"r {live.pop(rng.randrange(len(live)))}")
        else:
            ops.append(f"a {nxt} {rng.randrange(0, 256 * 20)}")
            live.append(nxt)
            nxt += 1
    out = run_clean([programs["ring_asan"], str(size)], stdin="\n".join(ops) + "\n")
    assert len(out.splitlines()) == len(ops)
