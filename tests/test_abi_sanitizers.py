"""The library's host code under AddressSanitizer + UndefinedBehaviorSanitizer (CPU):
a driver over the host-only entry points -- request validation with one mutation per
rule, state-buffer sizes, the autotuner's candidate shapes, the option order -- linked
with the host runtime built plain and built sanitized (the kernels' objects as built).
Both must give the expected status of every validation case and the same digest of
all results, the sanitized one with no report; a write past a vector planted in a copy
of the runtime is caught."""
import os
import shutil
import subprocess

import pytest

from paper_2002_02481_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "sanitize", "abi_driver.c")
KERNEL_OBJECTS = [os.path.join(B.BUILD, stem + ".o") for _, device, _, stem in B.SOURCES if device]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
HOST_SAN = [f for flag in SAN for f in ("-Xarch_host", flag)]   # host code only

pytestmark = [
    pytest.mark.skipif(shutil.which("hipcc") is None or shutil.which("gcc") is None, reason="needs hipcc and gcc"),
    pytest.mark.skipif(not all(os.path.exists(o) for o in KERNEL_OBJECTS),
                       reason="the kernels' objects are not built (run the package build first)"),
]

# lv_check's status for each mutation of the driver's valid request (lvmc.h's codes:
# 1 argument, 2 grid, 3 step, 6 unsupported), in the driver's case order
EXPECTED = [1, 1, 2, 2, 1, 1, 3, 1, 1, 2, 2, 2, 2, 1, 1, 1, 1, 1, 6, 1, 1, 1, 1, 1, 6, 6, 0, 1, 0, 0, 0, 0]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _runtime(tmp_path, name, flags):
    obj = str(tmp_path / f"api_{name}.o")
    subprocess.run(["hipcc", "-O1", "-g", "-std=c++17", "-fPIC", f"-I{B.INCLUDE}", f"-I{B.CSRC}"] + flags +
                   ["-c", os.path.join(B.CSRC, "lv_api.cpp"), "-o", obj], check=True, capture_output=True, text=True)
    return obj


def _program(tmp_path, name, api_obj, driver, cflags, lflags):
    drv = str(tmp_path / f"drv_{name}.o")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", f"-I{B.INCLUDE}"] + cflags + ["-c", driver, "-o", drv],
                   check=True, capture_output=True, text=True)
    exe = str(tmp_path / name)
    subprocess.run(["hipcc", f"--offload-arch={B.ARCH}"] + lflags + [drv, api_obj] + KERNEL_OBJECTS + ["-o", exe],
                   check=True, capture_output=True, text=True)
    return subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)


def _parse(r, name):
    assert r.returncode == 0, f"{name}: exit {r.returncode}\n{r.stderr[-3000:]}"
    assert "runtime error" not in r.stderr and "ERROR:" not in r.stderr, r.stderr[-3000:]
    lines = r.stdout.split("\n")
    status = [int(l.split()[3]) for l in lines if l.startswith("case ")]
    tail = [l for l in lines if l.startswith("abi ")]
    assert len(tail) == 1 and tail[0].endswith(" ok"), r.stdout[-500:]
    return status, tail[0]


def test_host_runtime_clean_under_sanitizers(tmp_path):
    plain = _parse(_program(tmp_path, "plain", _runtime(tmp_path, "plain", []), DRIVER, [], []), "plain")
    san_api = _runtime(tmp_path, "san", HOST_SAN)
    san = _parse(_program(tmp_path, "san", san_api, DRIVER, SAN, HOST_SAN), "sanitized")
    assert plain[0] == EXPECTED
    assert san == plain
    # the sanitized runtime sees a mistake planted in a copy of it: the option order's
    # step table written one past its end
    src = open(os.path.join(B.CSRC, "lv_api.cpp")).read()
    line = "for (int k = 0; k < book->n_opt; ++k) steps[k] = "
    assert src.count(line) == 1
    bad = tmp_path / "lv_api_planted.cpp"
    bad.write_text(src.replace(line, "for (int k = 0; k <= book->n_opt; ++k) steps[k] = "))
    obj = str(tmp_path / "api_planted.o")
    subprocess.run(["hipcc", "-O1", "-g", "-std=c++17", "-fPIC", f"-I{B.INCLUDE}", f"-I{B.CSRC}"] + HOST_SAN +
                   ["-c", str(bad), "-o", obj], check=True, capture_output=True, text=True)
    r = _program(tmp_path, "planted", obj, DRIVER, SAN, HOST_SAN)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]
