"""The oracle's pins again, with the oracle built under AddressSanitizer and
UndefinedBehaviorSanitizer (host code; gcc).  An out-of-bounds access, a
use after free or undefined arithmetic anywhere the pins reach aborts the
run.  The sanitized library is loaded in a child process that preloads the
ASan runtime."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_lattice.py", "tests/test_oracle_ibm.py", "tests/test_oracle_membrane_energy.py",
        "tests/test_oracle_contact.py", "tests/test_oracle_rbc.py", "tests/test_oracle_magnetic.py"]

CHECK = """
import ctypes, oracle
assert oracle._SO.endswith("liboracle_san.so"), oracle._SO
L = oracle.lib()
# instrumented code calls into the ASan and UBSan runtimes
for sym in ("__asan_report_load8", "__ubsan_handle_add_overflow"):
    assert hasattr(L, sym), sym
print("sanitized oracle loaded")
"""


def _env():
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                             check=True).stdout.strip()
    env = dict(os.environ)
    env.update(ORACLE_SANITIZE="1", LD_PRELOAD=libasan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS=env.get("OMP_NUM_THREADS", "4"))
    return env


def test_oracle_pins_under_asan_and_ubsan():
    env = _env()
    subprocess.run([sys.executable, "-c", "import oracle; oracle.build(force=True)"], cwd=ROOT, env=env,
                   check=True)
    r = subprocess.run([sys.executable, "-c", CHECK], cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode == 0 and "sanitized oracle loaded" in r.stdout, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *PINS], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
