"""The oracle under the compilers' sanitizers (CPU): a driver calling every exported
entry point -- both schemes, a rate, several threads and path ranges, the error paths --
built with AddressSanitizer + UndefinedBehaviorSanitizer, and with ThreadSanitizer for
the worker threads that share the chunk queue.  Each build must run clean and give the
plain build's checksum."""
import os
import shutil
import subprocess

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "sanitize", "oracle_driver.c")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


def _build_and_run(tmp_path, name, flags, threads=4):
    exe = str(tmp_path / name)
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer"] + flags + [DRIVER, oracle.SOURCE, "-o", exe,
                                                                                  "-lm", "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # the environment's own preloaded libraries may come before the sanitizer runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, str(threads)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, f"{name}: exit {r.returncode}\n{r.stderr[-3000:]}"
    assert r.stdout.strip().endswith("ok"), r.stdout
    assert "runtime error" not in r.stderr and "ERROR:" not in r.stderr, r.stderr[-3000:]
    return r.stdout.split()[1]


def test_oracle_clean_under_sanitizers(tmp_path):
    plain = _build_and_run(tmp_path, "plain", [])
    asan = _build_and_run(tmp_path, "asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    tsan = _build_and_run(tmp_path, "tsan", ["-fsanitize=thread"], threads=8)
    assert asan == plain and tsan == plain


def _build_planted(tmp_path, name, flags, driver_edit=None, oracle_edit=None):
    drv, src = open(DRIVER).read(), open(oracle.SOURCE).read()
    if driver_edit:
        assert drv.count(driver_edit[0]) == 1
        drv = drv.replace(*driver_edit)
    if oracle_edit:
        assert src.count(oracle_edit[0]) == 1
        src = src.replace(*oracle_edit)
    d, o = tmp_path / f"{name}_driver.c", tmp_path / f"{name}_oracle.c"
    d.write_text(drv)
    o.write_text(src)
    exe = str(tmp_path / name)
    subprocess.run(["gcc", "-O1", "-g", "-std=c11"] + flags + [str(d), str(o), "-o", exe, "-lm", "-lpthread"],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1", TSAN_OPTIONS="halt_on_error=1")
    return subprocess.run([exe, "8"], capture_output=True, text=True, env=env, timeout=300)


def test_sanitizers_catch_planted_mistakes(tmp_path):
    """The builds above would see a mistake: a read one past a path's state array, and a
    counter the worker threads update without the queue's lock (both planted in copies)."""
    r = _build_planted(tmp_path, "oob", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                       driver_edit=("check += y[N] + lam[0] * 1e-3;", "check += y[N + 1] + lam[0] * 1e-3;"))
    assert r.returncode != 0 and ("out of bounds" in r.stderr or "ERROR: AddressSanitizer" in r.stderr), r.stderr[-2000:]
    r = _build_planted(tmp_path, "race", ["-fsanitize=thread"],
                       oracle_edit=("static void *lvo_worker(void *arg)\n{",
                                    "static int lvo_race;\nstatic void *lvo_worker(void *arg)\n{\n    lvo_race++;"))
    assert r.returncode != 0 and "ThreadSanitizer: data race" in r.stderr, r.stderr[-2000:]
