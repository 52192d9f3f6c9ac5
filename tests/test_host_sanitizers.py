"""The C-ABI's host layer under AddressSanitizer and UndefinedBehavior-
Sanitizer (no GPU needed).

tests/host_abi_check.c drives every host-side decision of libgs3 (size
queries up to the documented limits, argument checks, status-block decoding
and the refusals that follow it) against a copy of the library whose host
code is built with both sanitizers (paper_2410_11419_amd.build.
build_host_check). A memory error, a leak or undefined behaviour in that
code ends the program with the sanitizer's report and a non-zero status."""
import os
import subprocess

from paper_2410_11419_amd import build as B


def test_host_layer_under_asan_and_ubsan():
    if not (os.path.exists(B.HOST_CHECK) and os.path.exists(B.LIB_SAN)):
        B.build_host_check(verbose=False)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([B.HOST_CHECK], capture_output=True, text=True, env=env, timeout=300)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report
    assert "host ABI checks passed" in r.stdout, report
    assert "Sanitizer" not in report, report
