"""Host-side audit of the library on a mock HIP runtime (CPU only).

The engine's host code (serving threads and the cooperative server,
device-memory pool, deferred releases, staging, batch calls) is built with AddressSanitizer or
ThreadSanitizer and linked against tests/host_audit/mock_hip.cpp, a stand-in
runtime whose streams run their queues asynchronously on threads and whose
kernels only check what they would read.  The mock reports device blocks that
return to the pool (or are freed) while queued work still uses them, and
descriptor fields of running kernels that point outside live blocks; the
sanitizers report host memory errors and data races.  Requests come from two
threads at once, a batch call runs beside them, and some requests are left
for the context teardown.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_audit")
KOBJ = os.path.join(ROOT, "paper_1309_5050_amd", "_build", "kernels.o")


def _have_tools():
    return (os.path.exists("/opt/rocm/bin/hipcc") and os.path.exists("/opt/rocm/llvm/bin/clang++"))


def _build(tmp, san):
    if not os.path.exists(KOBJ):
        import __graft_entry__ as g   # the kernels object of the regular build is linked
        g.build()
    out = os.path.join(tmp, san)
    res = subprocess.run(["bash", os.path.join(HERE, "build.sh"), out, san], capture_output=True, text=True,
                         timeout=600)
    if res.returncode != 0:
        pytest.fail("audit build failed:\n" + res.stdout + res.stderr)
    return os.path.join(out, "audit")


def _run(exe, nreq, env_extra, timeout=300):
    env = dict(os.environ)
    env.update(env_extra)
    env.setdefault("MOCK_OP_US", "20")
    res = subprocess.run([exe, str(nreq)], capture_output=True, text=True, timeout=timeout, env=env)
    out = res.stdout + res.stderr
    return res.returncode, out


pytestmark = pytest.mark.skipif(not _have_tools(), reason="hipcc / clang++ not installed")


@pytest.fixture(scope="module")
def tmpdir_mod(tmp_path_factory):
    d = tmp_path_factory.mktemp("host_audit")
    yield str(d)
    shutil.rmtree(str(d), ignore_errors=True)


def test_serving_and_pool_under_address_sanitizer(tmpdir_mod):
    exe = _build(tmpdir_mod, "address")
    rc, out = _run(exe, 24, {"ASAN_OPTIONS": "detect_leaks=1"})
    assert rc == 0, out[-4000:]
    assert "0 unexpected statuses" in out and "0 audit reports" in out, out[-2000:]
    # a device memory cap: allocation failures take the pool's release-and-retry
    # path, which must free no block that queued work still uses
    rc, out = _run(exe, 24, {"MOCK_DEVICE_BYTES": "50000000", "ASAN_OPTIONS": "detect_leaks=1"})
    assert rc == 0, out[-4000:]
    assert "0 audit reports" in out, out[-2000:]


def test_cooperative_serving_under_address_sanitizer(tmpdir_mod):
    """The cooperative server (no worker threads: the clients' waits drive
    admissions and restart cycles on the context's stream), with and
    without a device memory cap."""
    exe = _build(tmpdir_mod, "address")
    rc, out = _run(exe, 24, {"AUDIT_COOP": "1", "ASAN_OPTIONS": "detect_leaks=1"})
    assert rc == 0, out[-4000:]
    assert "0 unexpected statuses" in out and "0 audit reports" in out, out[-2000:]
    rc, out = _run(exe, 24, {"AUDIT_COOP": "1", "MOCK_DEVICE_BYTES": "50000000", "ASAN_OPTIONS": "detect_leaks=1"})
    assert rc == 0, out[-4000:]
    assert "0 audit reports" in out, out[-2000:]


def test_serving_and_pool_under_thread_sanitizer(tmpdir_mod):
    exe = _build(tmpdir_mod, "thread")
    rc, out = _run(exe, 16, {"TSAN_OPTIONS": "halt_on_error=1"}, timeout=600)
    assert rc == 0, out[-4000:]
    assert "WARNING: ThreadSanitizer" not in out, out[-4000:]
    assert "0 unexpected statuses" in out and "0 audit reports" in out, out[-2000:]
    # with the length tuner and a tune cache file (tuning runs and cache
    # writes beside the other threads' calls on the same context)
    cache = os.path.join(tmpdir_mod, "tune.txt")
    rc, out = _run(exe, 12, {"TSAN_OPTIONS": "halt_on_error=1", "AUDIT_TUNE_CACHE": cache}, timeout=600)
    assert rc == 0, out[-4000:]
    assert "WARNING: ThreadSanitizer" not in out, out[-4000:]
    assert "0 unexpected statuses" in out and "0 audit reports" in out, out[-2000:]
    assert os.path.exists(cache)
    # the cooperative server: two clients' waits drive it in turn
    rc, out = _run(exe, 16, {"TSAN_OPTIONS": "halt_on_error=1", "AUDIT_COOP": "1"}, timeout=600)
    assert rc == 0, out[-4000:]
    assert "WARNING: ThreadSanitizer" not in out, out[-4000:]
    assert "0 unexpected statuses" in out and "0 audit reports" in out, out[-2000:]
