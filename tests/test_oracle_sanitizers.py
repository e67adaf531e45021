"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): a tiny 1D and 2D assembly (all pair classes, the boundary term, the
row-subset mode, the symmetry weights), the CG solve and the band-pair
listing run in a child process that preloads the ASan runtime; it must exit
cleanly, with no sanitizer report, and give the same numbers as the
ordinary build."""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_CHILD = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import oracle as O
from oracle import surrogate as S
from paper_1708_03912_amd import meshgen as M
out = {}
m1 = M.interval(16)
out["A1"], _, _ = O.assemble(m1, 0.75, O.Orders())
m2 = M.disk_for_cells(60, seed=2)
for s in (0.25, 0.75):
    A, dofs, cnt = O.assemble(m2, s, O.Orders(k_touch=4, k_touch_bnd=4))
    out["A2_%g" % s] = A
    out["cnt_%g" % s] = cnt
    b = O.load_vector_one(m2, dofs)
    out["u_%g" % s] = O.pcg(A, b, rtol=1e-12)[0]
rows = np.array([3, 10, 17])
out["R"], _ = O.assemble_full(m2, 0.6, O.Orders(), rows=rows, compact=True)
w = np.zeros(len(m2["cells"])); w[: len(w) // 2] = 1.0
out["W"], _ = O.assemble_full(m2, 0.4, O.Orders(), cell_w=w)
out["band"] = np.asarray(S.band_pairs(m2, [1.5, 3.0, 6.0], 2), dtype=np.float64)
np.savez(sys.argv[2], **out)
print("child done", flush=True)
"""


def _run_child(tmp_path, sanitized):
    env = dict(os.environ)
    env["OMP_NUM_THREADS"] = "2"
    if sanitized:
        env["FL_ORACLE_SANITIZED"] = "1"
        env["LD_PRELOAD"] = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
        env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=23"
        env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    else:
        env.pop("FL_ORACLE_SANITIZED", None)
    out = tmp_path / ("san.npz" if sanitized else "plain.npz")
    p = subprocess.run([sys.executable, "-c", _CHILD, ROOT, str(out)], env=env, capture_output=True, text=True,
                       timeout=600)
    return p, out


def test_oracle_clean_under_asan_ubsan(tmp_path):
    O.build(sanitize=True)
    O.build()
    p, out = _run_child(tmp_path, sanitized=True)
    report = p.stdout + p.stderr
    assert p.returncode == 0, report[-4000:]
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert "child done" in p.stdout
    q, ref = _run_child(tmp_path, sanitized=False)
    assert q.returncode == 0, (q.stdout + q.stderr)[-4000:]
    a, b = np.load(out), np.load(ref)
    assert sorted(a.files) == sorted(b.files)
    for k in a.files:
        x, y = a[k], b[k]
        assert x.shape == y.shape, k
        # entries that are never formed (boundary rows for s >= 1/2) are NaN
        # in both; the rest agree to rounding (same source, other flags)
        assert np.array_equal(np.isnan(x), np.isnan(y)), k
        fin = ~np.isnan(y)
        if fin.any():
            assert np.abs(x[fin] - y[fin]).max() <= 1e-13 * max(np.abs(y[fin]).max(), 1e-300), k
