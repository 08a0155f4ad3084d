"""Host-side race check of the batch adjoint's worker pool: the library's C ABI
and kernels compiled for the CPU (tests/emu) with ThreadSanitizer, driven by
tests/emu/tsan_batch_adjoint.cpp.  The emulator keeps all of its grid state
per host thread and takes no lock around launches, so the library's host
code runs exactly as concurrently as its worker pool makes it; the sanitizer
sees every fiber switch.  A planted race in the driver (not in the library)
shows that the instrumentation is live."""
import os
import subprocess

import pytest


@pytest.fixture(scope="module")
def driver():
    from emu import build_emu

    return build_emu.build_tsan_driver()


def _run(exe, *args, timeout=900):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=0 exitcode=66")
    return subprocess.run([exe, *args], capture_output=True, text=True, timeout=timeout, env=env)


def test_sanitizer_reports_a_planted_race(driver):
    r = _run(driver, "--planted-race", timeout=120)
    assert r.returncode == 66, (r.returncode, r.stderr[-2000:])
    assert "ThreadSanitizer: data race" in r.stderr


def test_batch_adjoint_worker_pool_is_race_free(driver):
    r = _run(driver)
    print(r.stdout)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr[-2000:])
    assert "bitwise equal" in r.stdout
