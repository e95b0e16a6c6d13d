"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer passes its own CPU pins
(every oracle test except the two long reflection sweeps): no out-of-bounds access, use after free,
signed overflow, misaligned or otherwise undefined operation on any path those tests exercise."""
import shutil

import pytest


@pytest.mark.slow
def test_oracle_suite_under_asan_and_ubsan():
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    from oracle import sanitize
    try:
        sanitize.runtime()
    except Exception as e:  # noqa: BLE001
        pytest.skip(f"no sanitizer runtime: {e}")
    rc, out = sanitize.run_suite()
    tail = out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, tail
    assert rc == 0, tail
    assert " passed" in out, tail
