"""The serving runtime's host logic (admission, budget, eviction, the dispatcher's state
machine, ticket lifetime) built on the CPU against stand-ins of the library phases, of its
batches and of the few HIP host calls it makes, under ThreadSanitizer and AddressSanitizer:
200 requests of six geometries from a submitting thread, groups of up to four of one
geometry, a budget that forces queueing and evictions.  The stand-in chunks complete after a delay, so a read before completion,
two chunks in flight on one handle or a use after destroy fails the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "server_host")


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_server_logic_under_sanitizer(tmp_path, san):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    server = tmp_path / "server.cpp"
    shutil.copy(os.path.join(ROOT, "paper_1411_6206_amd", "csrc", "pls_server.hip"), server)
    exe = tmp_path / "drv"
    cmd = ["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={san}", "-DPLS_SERVER_MAX_IN_FLIGHT=4",
           "-I", SRC,
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1411_6206_amd", "csrc"),
           str(server), os.path.join(SRC, "fake_lib.cpp"), os.path.join(SRC, "driver.cpp"),
           "-o", str(exe), "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "completed 200 failed 0" in r.stdout and "bad 0" in r.stdout
    assert " evicted 0 " not in r.stdout            # the budget did force evictions


RT = os.path.join(HERE, "runtime_host")


@pytest.mark.parametrize("san,mode", [("thread", ""), ("address,undefined", ""),
                                      ("address,undefined", "full")],
                         ids=["thread", "address", "address_full_size"])
def test_runtime_and_server_host_code_under_sanitizer(tmp_path, san, mode):
    """The library's own runtime (pls_runtime.hip) and server, host code as built for the GPU,
    against a HIP stand-in whose streams run asynchronously on threads and kernel stand-ins
    that touch their arrays at full extent: sequences of five geometries, up to four of one
    geometry in flight as a batched group, evictions and sample-store growth, then the
    synchronous API from four threads and batches.  "full": the serving volume classes at
    their real sizes, four 192x192x32 x 30 frames x 8 coils sequences in flight."""
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    csrc = os.path.join(ROOT, "paper_1411_6206_amd", "csrc")
    exe = tmp_path / "rt"
    cmd = ["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={san}", "-DPLS_SERVER_MAX_IN_FLIGHT=4",
           "-I", RT, "-I", os.path.join(ROOT, "include"), "-I", csrc,
           "-x", "c++", os.path.join(csrc, "pls_runtime.hip"), os.path.join(csrc, "pls_server.hip"),
           "-x", "none", os.path.join(RT, "kernels_stub.cpp"), os.path.join(RT, "driver.cpp"),
           "-o", str(exe), "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1",
               ASAN_OPTIONS="halt_on_error=1:detect_leaks=0")
    r = subprocess.run([str(exe)] + ([mode] if mode else []), capture_output=True, text=True,
                       timeout=600, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "failed 0" in r.stdout and "done: bad 0 sync_bad 0" in r.stdout
    # sequences of one geometry ran together as a batched group
    import re
    assert int(re.search(r"peak_active (\d+)", r.stdout).group(1)) >= 2


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_autotuner_sequence_host_code_under_sanitizer(tmp_path, san):
    """The autotuner's host code (prior_ls_tune: a reload, a captured chunk and two replays per
    candidate, graphs destroyed between candidates) in the GPU tuner test's exact sequence,
    five times: tune, step, destroy; a fresh handle with the choice set by hand solves; a
    third loads, steps and is destroyed."""
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    csrc = os.path.join(ROOT, "paper_1411_6206_amd", "csrc")
    exe = tmp_path / "rt"
    cmd = ["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={san}", "-DPLS_SERVER_MAX_IN_FLIGHT=4",
           "-I", RT, "-I", os.path.join(ROOT, "include"), "-I", csrc,
           "-x", "c++", os.path.join(csrc, "pls_runtime.hip"), os.path.join(csrc, "pls_server.hip"),
           "-x", "none", os.path.join(RT, "kernels_stub.cpp"), os.path.join(RT, "driver.cpp"),
           "-o", str(exe), "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1",
               ASAN_OPTIONS="halt_on_error=1:detect_leaks=0:detect_stack_use_after_return=1",
               UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe), "tune"], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
    assert "tune done: bad 0" in r.stdout and r.stdout.count("tune round") == 5
