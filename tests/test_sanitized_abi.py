"""The C ABI under host-side AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer.

tests/abi_driver.cpp is linked against a copy of libnuasm whose host code is
instrumented (build --sanitized; the kernels are compiled as usual).  On the
CPU it exercises argument validation, status strings and the no-device paths;
on a GPU it also runs every operator's life cycle with each device or pinned
allocation in turn failing (nuasm_debug_fail_alloc), checking that the call
that allocated reports NUASM_ERR_ALLOC, that every plan and batch still
destroys cleanly and that the memory the library holds returns to where it
started (its own count of live allocations).  Any
sanitizer report ends the driver with a non-zero status.
"""
import os
import subprocess

import pytest

from paper_1308_6644_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = ":".join([
        "detect_leaks=1", "halt_on_error=1", "abort_on_error=0", "exitcode=23",
        # the ROCm runtime maps device apertures at fixed low addresses
        "protect_shadow_gap=0", "verify_asan_link_order=0",
    ])
    env["LSAN_OPTIONS"] = f"suppressions={os.path.join(HERE, 'lsan_hip.supp')}:print_suppressions=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=24"
    return env


def _run(mode, timeout):
    r = subprocess.run([B.SAN_DRIVER, mode], capture_output=True, text=True, timeout=timeout, env=_env())
    out = r.stdout + r.stderr
    print(out[-4000:])
    assert r.returncode == 0, f"abi_driver {mode} exited with {r.returncode}:\n{out[-4000:]}"
    assert "ABI_DRIVER_OK" in r.stdout
    return r.stdout


def test_sanitized_driver_cpu_paths():
    if B.sanitized_stale():
        B.build_sanitized()
    out = _run("cpu", timeout=300)
    assert "cpu checks done" in out


@pytest.mark.gpu
def test_sanitized_driver_allocation_failures_on_gpu():
    if B.sanitized_stale():
        pytest.skip("the sanitized build is missing or was made from other sources: "
                    "python -m paper_1308_6644_amd.build --sanitized")
    out = _run("gpu", timeout=240)
    print([l for l in out.splitlines() if l.startswith("gpu:")])
    assert "injected allocation failures" in out
