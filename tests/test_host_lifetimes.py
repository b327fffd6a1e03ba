"""Host-side memory safety and API lifetimes of the library.

Every source of libidp_dg is compiled for the host only (kernel launches
become runtime calls), with AddressSanitizer and UndefinedBehaviorSanitizer
(fatal) on the host code, and linked
against a stand-in for the HIP runtime (tests/hostmock/hip_mock.cpp) that
keeps queued work pending until the host synchronises and aborts on
misuse: a graph exec destroyed with a launch pending, double frees, pinned
memory freed or changed while a copy from it is pending, destroyed handles
used.  tests/hostmock/lifetimes.cpp drives a serving loop with nested
sub-steps (batch membership changing between unsynchronised steps) and the
plain path's graph re-capture.  No GPU is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2004_08503_amd", "csrc")
MOCK = os.path.join(ROOT, "tests", "hostmock")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    assert r.returncode == 0, "%s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr[-4000:])


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm toolchain not found")
    d = str(tmp_path_factory.mktemp("hostmock"))
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    host_only = ["--offload-host-only", "-O1", "-g", "-std=c++17", "-fPIC", "-Xarch_host", "-fsanitize=address",
                 "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
                 "-Wno-unused-result", "-I", CSRC, "-I", os.path.join(ROOT, "include")]
    procs = [subprocess.Popen([HIPCC] + host_only + ["-c", os.path.join(CSRC, f), "-o", f + ".o"], cwd=d,
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE) for f in srcs]
    for p, f in zip(procs, srcs):
        out, err = p.communicate()
        assert p.returncode == 0, "%s: %s" % (f, err.decode()[-3000:])
    objs = [f + ".o" for f in srcs]
    # the host-only objects still name the device code blobs: give them storage
    syms = subprocess.run(["nm", "-u"] + objs, cwd=d, capture_output=True, text=True).stdout.split()
    blobs = sorted({s for s in syms if s.startswith("__hip_fatbin")})
    with open(os.path.join(d, "blobs.cpp"), "w") as f:
        for s in blobs:
            f.write('extern "C" { char %s[16]; }\n' % s)
    asan = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-O1",
            "-g", "-std=c++17"]
    _run([CLANG] + asan + ["-c", os.path.join(MOCK, "hip_mock.cpp"), "-o", "hip_mock.o"], d)
    _run([CLANG] + asan + ["-c", "blobs.cpp", "-o", "blobs.o"], d)
    _run([CLANG] + asan + ["-I", os.path.join(ROOT, "include"), "-c", os.path.join(MOCK, "lifetimes.cpp"),
                           "-o", "lifetimes.o"], d)
    _run([CLANG, "-fsanitize=address,undefined", "-o", "lifetimes", "lifetimes.o", "hip_mock.o", "blobs.o"] + objs, d)
    yield os.path.join(d, "lifetimes")
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("seed", [5, 6])
def test_serving_and_plain_lifetimes(driver, seed):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([driver, "60", "16", str(seed)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-6000:]
    assert "served 60 requests" in r.stdout and "plain path done" in r.stdout
    assert "curved path done" in r.stdout
    assert "live device allocations 0, pinned 0, graph execs 0" in r.stderr
