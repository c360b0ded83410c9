"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

oracle/sanitize_driver.c calls every oracle entry point on seeded small maps and edge-case
rays; built with -fsanitize=address,undefined and -fno-sanitize-recover, any out-of-bounds
access, use of uninitialised heap memory through a bad index, signed overflow or invalid shift
ends the run with a report and a non-zero status."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", f"-I{ORACLE}",
           os.path.join(ORACLE, "nbt_oracle.c"), os.path.join(ORACLE, "sanitize_driver.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ)
    # another preloaded library may come first in the link order; ASan only needs to be loaded
    env["ASAN_OPTIONS"] = "verify_asan_link_order=0:detect_leaks=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, f"exit {r.returncode}\n{r.stdout}\n{r.stderr[-4000:]}"
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "oracle sanitize driver ok" in r.stdout
