"""Write the golden ground-state energies of tests/golden/e0_*.txt from the oracle alone.

Every number written here comes from ``oracle/`` (the float64 Lanczos iteration of Alg. 1 and the
lowest eigenvalue of T, Sec. 2.2; SciPy's ARPACK on the oracle's H.v as a second algorithm) applied to
the seeded inputs of ``synth/``.  Nothing of the device library is imported.

Cases (one file each, so they can run in parallel processes):

* ``torus4x4_5x5``: 4x4 periodic Hubbard, 5 + 5, U = 4, start seed 2; Alg. 1 for 200 steps (E0 after
  each tenth step) and ARPACK's lowest eigenvalue of the same operator.
* ``torus4x4_8x8``: 4x4 periodic Hubbard at half filling, 8 + 8, U = 4, start seed 5; Alg. 1 for 200
  steps (E0 after each tenth step).  ``torus4x4_8x8_seed55`` repeats it from another start vector: an
  independent trajectory that must reach the same E0.
* ``batch34``: every instance of the 64-instance batch draw (4x4 torus, U ~ U[0, 8], seed 1000) with
  3 or 4 particles per species: Alg. 1 from the instance's start seed until E0 changes by less than
  1e-13 between consecutive steps (at most 400 steps).

Usage: python tests/golden/make_energies.py CASE [CASE ...]   (several hours of CPU in total for 8 + 8)
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.hamiltonian import Model  # noqa: E402
from oracle.lanczos import lanczos, ritz_lowest  # noqa: E402
from synth import batch_instances, start_vector, torus_bonds, workload  # noqa: E402


def _log(msg):
    print("[%s] %s" % (time.strftime("%H:%M:%S"), msg), file=sys.stderr, flush=True)


def _write(name, header, rows):
    path = os.path.join(HERE, "e0_%s.txt" % name)
    with open(path, "w") as fh:
        for line in header:
            fh.write("# %s\n" % line)
        for row in rows:
            fh.write(" ".join(str(v) for v in row) + "\n")
    _log("wrote %s" % path)


def lanczos_case(wname, seed, steps, arpack=False, name=None):
    w = workload(wname)
    m = Model(w.n_sites, w.bonds, w.n_up, w.n_dn, w.t, w.U)
    x = start_vector(seed, m.dim)
    _log("%s: dim %d, %d oracle Lanczos steps from seed %d" % (wname, m.dim, steps, seed))
    t0 = time.time()
    r = lanczos(m.hv, x, steps)
    ritz = ritz_lowest(r["a"], r["b"])
    _log("%s: Lanczos done in %.0f s, E0(%d) = %r" % (wname, time.time() - t0, len(r["a"]), ritz[-1]))
    rows = [("lanczos", seed, j, repr(float(ritz[j - 1]))) for j in range(10, len(ritz) + 1, 10)]
    header = ["%s: %s" % (wname, w.note), "U = %r, t = %r, start = synth.start_vector(%d, dim)" % (w.U, w.t, seed),
              "columns: method, start seed, steps j, E0 (lowest eigenvalue of T_j; for arpack, of H)",
              "written by tests/golden/make_energies.py from oracle/ only"]
    if arpack:
        import scipy.sparse.linalg as sla
        op = sla.LinearOperator((m.dim, m.dim), matvec=m.hv, dtype=np.float64)
        t0 = time.time()
        ev = sla.eigsh(op, k=1, which="SA", tol=1e-14, v0=x, ncv=24, return_eigenvectors=False)
        _log("%s: ARPACK done in %.0f s, E0 = %r" % (wname, time.time() - t0, float(ev[0])))
        rows.append(("arpack", seed, 0, repr(float(ev[0]))))
    _write(name or wname, header, rows)


def batch34():
    rows = []
    bonds = torus_bonds(4, 4)
    for i, (u, n, seed) in enumerate(batch_instances(64, 1000)):
        if n not in (3, 4):
            continue
        m = Model(16, bonds, n, n, 1.0, u)
        x = start_vector(seed, m.dim)
        r = lanczos(m.hv, x, 400)
        ritz = ritz_lowest(r["a"], r["b"])
        stop = len(ritz)
        for j in range(2, len(ritz)):
            if abs(ritz[j] - ritz[j - 1]) < 1e-13 and abs(ritz[j - 1] - ritz[j - 2]) < 1e-13:
                stop = j + 1
                break
        rows.append(("batch", i, n, repr(float(u)), seed, stop, repr(float(ritz[stop - 1]))))
        _log("batch item %d: N = %d, U = %.4f, E0 = %r after %d steps" % (i, n, u, ritz[stop - 1], stop))
    header = ["the 64-instance batch draw (synth.batch_instances(64, 1000)), items with 3 or 4 particles per "
              "species: 4x4 periodic Hubbard, t = 1",
              "columns: kind, item index, N_up = N_dn, U, start seed, steps, E0 (Alg. 1 until |dE0| < 1e-13 "
              "twice in a row)",
              "written by tests/golden/make_energies.py from oracle/ only"]
    _write("batch34", header, rows)


CASES = {
    "torus4x4_5x5": lambda: lanczos_case("torus4x4_5x5", 2, 200, arpack=True),
    "torus4x4_8x8": lambda: lanczos_case("torus4x4_8x8", 5, 200),
    "torus4x4_8x8_seed55": lambda: lanczos_case("torus4x4_8x8", 55, 200, name="torus4x4_8x8_seed55"),
    "batch34": batch34,
}


if __name__ == "__main__":
    for case in sys.argv[1:] or sorted(CASES):
        CASES[case]()
