"""Sanitizer builds of the library's host code (CPU only, no device): the
units that hold the host logic (planning, validation, the batched template
and schedule replay, the serving scheduler, the tile model) are compiled
with the sanitizer on the host side only, linked with the library's other
objects as built (the tile units) and a native driver from tests/native,
and run.
  * ThreadSanitizer: the serving scheduler under concurrent clients, injected
    launch failures, stalls and deadlines (server_stress.cpp);
  * AddressSanitizer + UndefinedBehaviorSanitizer: configuration checks,
    workspace sizes, the tuning loader, the batched template and schedule
    replay, the fake scheduler with faults (host_checks.cpp).
A report from either sanitizer fails the test."""
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2607_22484_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))
CLANG = "/opt/rocm/llvm/bin/clang++"

pytestmark = pytest.mark.skipif(not (os.path.exists(build.HIPCC) and os.path.exists(CLANG)),
                                reason="ROCm compilers not installed")


HOST_UNITS = ["api.hip", "server.hip", "batched.hip", "batch.hip", "noalloc.hip", "trace.hip", "kernels.hip"]


def _build(tmp, san, driver):
    flags = [f for f in build.FLAGS if f != "-Wall"] + ["-O1", "-g", "-fno-omit-frame-pointer", "-w"]
    for s in san:  # host side only
        flags += ["-Xarch_host", "-fsanitize=" + s]
    objs = []
    todo = []
    for src in build.SOURCES:
        if src in HOST_UNITS:
            obj = os.path.join(tmp, src + ".o")
            todo.append((os.path.join(build.CSRC, src), obj))
        else:  # the library's own object (device code built as usual)
            obj = os.path.join(build.OBJ_DIR, src.replace(".hip", ".o"))
            if not os.path.exists(obj):
                pytest.skip("library objects not built (python -m paper_2607_22484_amd.build)")
        objs.append(obj)

    def one(pair):
        src, obj = pair
        subprocess.run([build.HIPCC] + flags + ["-c", src, "-o", obj], check=True, capture_output=True)
    with ThreadPoolExecutor(8) as ex:
        list(ex.map(one, todo))
    exe = os.path.join(tmp, os.path.splitext(os.path.basename(driver))[0])
    link = [CLANG, "-g"] + ["-fsanitize=" + s for s in san] + \
           ["-I", os.path.join(build.ROOT, "include"), driver] + objs + \
           ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-lpthread", "-o", exe]
    subprocess.run(link, check=True, capture_output=True)
    return exe


def _run(exe, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    return p.returncode, p.stdout + p.stderr


@pytest.fixture(scope="module")
def tmpdir_native():
    d = tempfile.mkdtemp(prefix="psvt_san_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def test_thread_sanitizer_serving_scheduler(tmpdir_native):
    d = os.path.join(tmpdir_native, "tsan")
    os.makedirs(d, exist_ok=True)
    exe = _build(d, ["thread"], os.path.join(HERE, "native", "server_stress.cpp"))
    supp = os.path.join(tmpdir_native, "tsan.supp")
    with open(supp, "w") as f:  # the HIP runtime is not instrumented
        f.write("called_from_lib:libamdhip64.so\ncalled_from_lib:libhsa-runtime64.so\n")
    rc, out = _run(exe, {"TSAN_OPTIONS": "halt_on_error=1 second_deadlock_stack=1 suppressions=" + supp})
    assert "ThreadSanitizer" not in out, out[-4000:]
    assert rc == 0, out[-4000:]


def test_address_and_ub_sanitizer_host_paths(tmpdir_native):
    d = os.path.join(tmpdir_native, "asan")
    os.makedirs(d, exist_ok=True)
    exe = _build(d, ["address", "undefined"], os.path.join(HERE, "native", "host_checks.cpp"))
    supp = os.path.join(tmpdir_native, "lsan.supp")
    with open(supp, "w") as f:  # allocations the HIP runtime keeps for the process
        f.write("leak:libamdhip64.so\nleak:libhsa-runtime64.so\nleak:libamd_comgr.so\n")
    rc, out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1 abort_on_error=0",
                         "LSAN_OPTIONS": "suppressions=" + supp,
                         "UBSAN_OPTIONS": "print_stacktrace=1 halt_on_error=1"})
    assert "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert rc == 0, out[-4000:]
