"""libdi's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): a build of every library source with the sanitizers on its
host pass runs the link-list validation of di_graph_create and the argument
checks of the solve entry points in a child process. The validation runs on
the host before any device work, so without a GPU every call ends either in
its documented error status or in DI_E_DEVICE. A second child hands the
library a link count one larger than its arrays: the read past their end
must abort it (the sanitizer is live)."""

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1204_6255_amd import build as pb  # noqa: E402

ASAN_RT = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))

CHILD = r'''
import numpy as np
from paper_1204_6255_amd import di
rng = np.random.default_rng(0)
def create(n, s, t):
    return di.di_graph_create(n, np.asarray(s, np.int32), np.asarray(t, np.int32))[0]
assert create(3, [0, 1, 1], [1, 0, 0]) == di.DI_E_DUP
assert create(3, [0, 1, 0], [1, 0, 2]) == di.DI_E_UNSORTED
assert create(3, [0, 1], [1, 3]) == di.DI_E_RANGE
assert create(3, [-1, 1], [1, 2]) == di.DI_E_RANGE
assert create(0, [], []) == di.DI_E_INVAL
assert create(5, [], []) in (di.DI_OK, di.DI_E_DEVICE)
# a large valid list and the same list with one link out of order / repeated
n = 20000
key = np.unique(rng.integers(0, n, 200000) * n + rng.integers(0, n, 200000))
s, t = (key // n).astype(np.int32), (key % n).astype(np.int32)
assert create(n, s, t) in (di.DI_OK, di.DI_E_DEVICE)
s2, t2 = s.copy(), t.copy(); s2[-1], t2[-1] = s2[0], t2[0]
assert create(n, s2, t2) == di.DI_E_UNSORTED
s3, t3 = s.copy(), t.copy(); t3[-1] = t3[-2]; s3[-1] = s3[-2]
assert create(n, s3, t3) == di.DI_E_DUP
st, h = di.di_graph_create(3, np.array([0], np.int32), np.array([1], np.int32), flags=4)
assert st == di.DI_E_INVAL and not h
# solve entry points reject a missing graph before any device work
X = np.empty(3)
assert di.di_solve(None, None, 0.85, 1e-9, None, X)[0] == di.DI_E_INVAL
assert di.di_last_error()
print("host checks passed")
'''


def _build(out_dir):
    """Host-only objects of every library source with the sanitizers (each
    -fsanitize right after -Xarch_host), linked into out_dir/libdi.so."""
    src_dir = os.path.join(out_dir, "src")
    os.makedirs(src_dir, exist_ok=True)
    for name in os.listdir(pb.CSRC):
        with open(os.path.join(pb.CSRC, name)) as f:
            text = f.read()
        with open(os.path.join(src_dir, name), "w") as f:
            f.write(text)
    flags = ["--offload-arch=gfx950", "-O1", "-Xarch_host", "-g", "-std=c++20", "-fPIC",
             "-munsafe-fp-atomics",
             "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             f"-I{pb.INCLUDE}", f"-I{src_dir}"]

    def one(name):
        obj = os.path.join(out_dir, name + ".o")
        subprocess.run([pb.hipcc(), *flags, "-c", "-x", "hip", os.path.join(src_dir, name), "-o", obj],
                       check=True, capture_output=True)
        return obj

    with ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(one, pb.HIP_SOURCES))
    lib = os.path.join(out_dir, "libdi.so")
    subprocess.run([pb.hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-shared-libsan", "-o", lib, *objs], check=True, capture_output=True)
    return lib


PLANTED = r'''
import ctypes
import numpy as np
from paper_1204_6255_amd import di
src = np.arange(0, 1000, dtype=np.int32)
dst = np.arange(1, 1001, dtype=np.int32) % 1000
dst = np.ascontiguousarray(dst)
h = ctypes.c_void_p()
# one link more than the arrays hold: the validation reads past their end
di.lib().di_graph_create(1000, 1001, src.ctypes.data, dst.ctypes.data, 0, ctypes.byref(h))
print("no report")
'''


def _run_child(lib, code=CHILD):
    env = dict(os.environ)
    env.update({
        "DI_LIB": lib,
        "LD_PRELOAD": ASAN_RT[-1],
        # the interpreter is not instrumented: no leak report at exit
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "PYTHONPATH": ROOT,
        "HIP_VISIBLE_DEVICES": "",
    })
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                          text=True, timeout=600)


@pytest.mark.skipif(not ASAN_RT, reason="clang's ASan runtime is not installed")
def test_libdi_host_code_under_sanitizers(tmp_path):
    lib = _build(str(tmp_path / "asan"))
    r = _run_child(lib)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "host checks passed" in r.stdout
    r = _run_child(lib, PLANTED)
    assert r.returncode != 0 and "no report" not in r.stdout
    assert "AddressSanitizer" in r.stderr, r.stderr[-3000:]
