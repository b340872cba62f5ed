"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The C-ABI library: its host code (argument checks, planning, error paths,
  the loader) is rebuilt with the sanitizers on the host pass only
  (`python -m paper_2602_20376_amd.build --sanitize`, device code unchanged),
  and the ABI tests run against it with clang's ASan runtime preloaded.
* The C oracle: built with gcc's -fsanitize=address,undefined, and the pin
  tests that call it run against it with gcc's runtime preloaded.

Each check runs in a child process, because an ASan runtime has to be the
first library loaded.  Any sanitizer report aborts the child (UBSan does not
recover), so a clean exit is the pass condition.  Leak checking is off: the
interpreter's own allocations at exit are not this project's.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2602_20376_amd import build as B  # noqa: E402

ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _stale(target, sources):
    return not os.path.exists(target) or os.path.getmtime(target) < max(os.path.getmtime(s) for s in sources)


def _child(cmd, extra_env, timeout=900):
    env = dict(os.environ, **ENV, **extra_env)
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, (r.returncode, r.stdout[-3000:], r.stderr[-3000:])
    return r.stdout


def test_host_library_under_asan_and_ubsan():
    sources = glob.glob(os.path.join(B.CSRC, "*")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    if _stale(B.LIB_SAN, sources):
        B.build(sanitize=True)
    env = {"LD_PRELOAD": B.asan_runtime(), "LRQO_LIBRARY": B.LIB_SAN}
    # the child really runs the instrumented library
    probe = ("from paper_2602_20376_amd import lrqo; lrqo.load(); "
             "maps = open('/proc/self/maps').read(); "
             "assert lrqo.LIB_PATH.endswith('_build_san/liblrqo.so'), lrqo.LIB_PATH; "
             "assert '_build_san/liblrqo.so' in maps and 'libclang_rt.asan' in maps; print('instrumented')")
    assert "instrumented" in _child([sys.executable, "-c", probe], env)
    out = _child([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_abi_cpu.py"], env)
    assert " passed" in out


def test_oracle_under_asan_and_ubsan():
    import oracle

    so = oracle.build(sanitize=True)
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    assert os.path.exists(libasan), libasan
    env = {"LD_PRELOAD": libasan, "LRQO_ORACLE_LIBRARY": so}
    out = _child([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                  "tests/test_oracle_pins.py", "tests/test_oracle_pins_more.py", "tests/test_spectral_pins.py"], env)
    assert " passed" in out
