"""The host side of the library under the address, undefined-behaviour and
thread sanitizers (CPU only).

tests/host_check.cpp drives the C-ABI without a GPU: argument validation,
tile queries, and the serving loop on its host-only fake executor with four
concurrent submitters, unstable requests retired early, oversized and
malformed requests refused.  The runtime, the server and the host side of the
kernel sources are compiled for the host only (no device code), once with
ASan + UBSan and once with TSan, and the driver must finish cleanly with no
sanitizer report.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2504_10539_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-I", CSRC, "-I",
          os.path.join(ROOT, "include")]
# each sanitizer flag applies to the host compilation only
SANITIZERS = {
    "asan": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"],
    "tsan": ["-Xarch_host", "-fsanitize=thread"],
}
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer",
           "ERROR: LeakSanitizer")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


def _build(kind, out):
    san = SANITIZERS[kind]
    jobs = []
    for src in ("sc_kernels.hip", "sc_noalloc.hip", "sc_pinn.hip"):
        jobs.append([HIPCC, "-x", "hip", "--offload-new-driver", "--cuda-host-only", *COMMON, *san,
                     "-c", os.path.join(CSRC, src), "-o", os.path.join(out, src + ".o")])
    for src in ("sc_runtime.cpp", "sc_server.cpp"):
        jobs.append([HIPCC, *COMMON, *san, "-c", os.path.join(CSRC, src), "-o",
                     os.path.join(out, src + ".o")])
    # host_check calls the host side of the kernel headers' launch accounting
    jobs.append([HIPCC, "-x", "hip", "--offload-new-driver", "--cuda-host-only", *COMMON, *san,
                 "-c", os.path.join(ROOT, "tests", "host_check.cpp"),
                 "-o", os.path.join(out, "host_check.o")])
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(_run, jobs))
    objs = [j[-1] for j in jobs]
    exe = os.path.join(out, "host_check_" + kind)
    _run([HIPCC, *COMMON, *san, *objs, "-o", exe, "-lpthread"])
    return exe


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="no hipcc")
@pytest.mark.parametrize("kind", ["asan", "tsan"])
def test_host_side_is_clean_under_sanitizers(kind, tmp_path):
    exe = _build(kind, str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "host_check: ok" in r.stdout
    for rep in REPORTS:
        assert rep not in out, out[-4000:]
