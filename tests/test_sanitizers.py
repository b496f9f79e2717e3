"""The oracle's pin battery under AddressSanitizer and UndefinedBehaviorSanitizer.

The C oracle is rebuilt with -fsanitize=address,undefined (host code only:
the oracle has no GPU code) and the whole pin battery of the mutant test
runs against it in a child process with the ASan runtime preloaded, so an
out-of-bounds access, a use after free or undefined arithmetic anywhere in
the oracle aborts the run.  A copy with a planted heap overflow shows that
the harness does catch one.  (The host logic of the library, the served
form's allocator and the bounded wait, runs under the same sanitizers in
test_host_logic.py.)"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hp_oracle.c")
BATTERY = os.path.join(ROOT, "tests", "_mutant_battery.py")
FLAGS = ["-O1", "-g", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-fno-fast-math", "-ffp-contract=off"]


def _asan_runtime():
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _build(tmp_path, name, text):
    c = tmp_path / f"{name}.c"
    c.write_text(text)
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", *FLAGS, f"-I{os.path.dirname(SRC)}", str(c), "-o", str(so)], check=True,
                   capture_output=True, text=True)
    return str(so)


def _run(so):
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    return subprocess.run([sys.executable, BATTERY, so], capture_output=True, text=True, timeout=600, env=env)


@pytest.fixture(scope="module")
def runtime():
    if _asan_runtime() is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")


def test_oracle_battery_clean_under_sanitizers(tmp_path, runtime):
    r = _run(_build(tmp_path, "oracle_asan", open(SRC).read()))
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def test_sanitizers_catch_planted_overflow(tmp_path, runtime):
    text = open(SRC).read()
    old = "for (int64_t j = 0; j < nJ; j++) list[fillp[J[j]]++] = (int32_t)j;"
    assert old in text
    bad = text.replace(old, old + "\n    list[nJ] = 0;   /* one past the end */", 1)
    r = _run(_build(tmp_path, "oracle_overflow", bad))
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]
