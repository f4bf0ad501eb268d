"""The oracle under AddressSanitizer + UndefinedBehaviorSanitizer and under
ThreadSanitizer (CPU only): oracle/sanitize_check.c runs every oracle
function on small seeded graphs (Algorithm 2 threaded and not, against the
plain definition; estimates and both union estimators; SKIM to the full
permutation; IC-model sketches and unions) in a sanitized build."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sanitize_check.c")


@pytest.mark.parametrize("flags", [["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                                   ["-fsanitize=thread"]], ids=["asan_ubsan", "tsan"])
def test_oracle_under_sanitizers(tmp_path, flags):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "sanitize_check")
    r = subprocess.run([gcc, "-O1", "-g", *flags, "-pthread", SRC, "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0 and "cannot find" in r.stderr:
        pytest.skip("sanitizer runtime not installed: " + r.stderr.strip()[:200])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all oracle checks passed" in out.stdout
