"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a C driver
(tests/oracle_sanitize_driver.c, one translation unit with the oracle source)
calls every routine on small inputs -- energies, tail terms, acceptance, the
chain, cell grid and neighbour sets (paper's and pruned microcell grids),
gradients and virial of a mixture -- and must exit cleanly with no sanitizer
report.  Built with gcc into a temporary directory; CPU only."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_clean_under_sanitizers():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "driver")
        flags = ["-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-omit-frame-pointer",
                 "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
        r = subprocess.run([gcc, *flags, os.path.join(HERE, "oracle_sanitize_driver.c"), "-lm", "-o", exe],
                           capture_output=True, text=True)
        if r.returncode != 0 and "asan" in r.stderr.lower():
            pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
        assert r.returncode == 0, r.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
        assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
        assert r.stdout.startswith("n="), r.stdout
