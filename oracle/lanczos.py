"""The Lanczos iteration (Alg. 1) and the tridiagonal projection T (Sec. 2.2).

``lanczos`` follows the paper's order exactly, in float64, with no
re-orthogonalisation: q = H f_j - b_j f_{j-1}; a_j = q.f_j; q = q - a_j f_j;
b_{j+1} = |q|; stop if b_{j+1} vanishes; f_{j+1} = q / b_{j+1}; b_1 = 0 and
f_0 = 0.  Inner products are f^dagger q: with complex hopping amplitudes the
vectors are complex, and a_j is the real part of f_j^dagger q (H is Hermitian,
so the imaginary part is rounding); with real hopping this is q^T f.

Readings:
* "b_{j+1} = 0" is tested as b_{j+1} <= 64 * eps * max_k(|a_k|, b_k) with
  eps = 2**-52; the iteration also stops after dim H steps.
* The start vector is supplied by the caller (seeded); it is normalised here.
* E0(j) is the lowest eigenvalue of T_j = tridiag(b_2..b_j; a_1..a_j; b_2..b_j),
  taken from LAPACK's tridiagonal solver.
* The ground-state vector is the standard two-pass construction: a second run
  from the same f_1 accumulates v = sum_k y_k f_k with y the lowest eigenvector
  of T_m, then v is normalised.  Gauge: the amplitude of a caller-chosen
  reference index is made positive; if it is below 1e-3 of the largest
  magnitude, the largest-magnitude entry (lowest index on ties) is used.
"""

import numpy as np
import scipy.linalg as sla

EPS64 = 2.0 ** -52


def _as_vector(f1) -> np.ndarray:
    return np.asarray(f1, dtype=np.complex128 if np.iscomplexobj(f1) else np.float64)


def _inner(u, v) -> float:
    """Re(u^dagger v)."""
    return float(np.real(np.vdot(u, v)))


def normalise(f1) -> np.ndarray:
    f = _as_vector(f1)
    n = np.sqrt(_inner(f, f))
    if not np.isfinite(n) or n == 0.0:
        raise ValueError("start vector has zero or non-finite norm")
    return f / n


def lanczos(hv, f1, m: int, vectors=False):
    """m steps of Alg. 1.  Returns dict(a, b, breakdown, f) with b[0] = b_1 = 0.

    a has the steps actually taken; b has one more entry (b_{j+1} of the last step).
    ``vectors=True`` also returns the Lanczos vectors f_1..f_j (small cases only).
    """
    f = normalise(f1)
    dim = f.size
    f_prev = np.zeros_like(f)
    a, b = [], [0.0]
    fs = [f.copy()] if vectors else None
    breakdown = False
    scale = 0.0
    for j in range(m):
        q = hv(f) - b[j] * f_prev
        aj = _inner(f, q)
        q = q - aj * f
        bj1 = float(np.sqrt(_inner(q, q)))
        a.append(aj)
        b.append(bj1)
        scale = max(scale, abs(aj), bj1)
        if bj1 <= 64.0 * EPS64 * scale or len(a) >= dim:
            breakdown = bj1 <= 64.0 * EPS64 * scale
            break
        f_prev, f = f, q / bj1
        if vectors:
            fs.append(f.copy())
    return {"a": np.array(a), "b": np.array(b), "breakdown": breakdown,
            "f": fs}


def tridiag_lowest(a, b_off) -> float:
    """Lowest eigenvalue of the symmetric tridiagonal matrix (diag a, offdiag b_off)."""
    a = np.asarray(a, dtype=np.float64)
    if a.size == 1:
        return float(a[0])
    w = sla.eigh_tridiagonal(a, np.asarray(b_off, dtype=np.float64),
                             eigvals_only=True, select="i", select_range=(0, 0))
    return float(w[0])


def ritz_lowest(a, b) -> np.ndarray:
    """E0(j) for j = 1..len(a), with b[0] = b_1 = 0 as returned by ``lanczos``."""
    return np.array([tridiag_lowest(a[:j], b[1:j]) for j in range(1, len(a) + 1)])


def ground_energy(hv, f1, m: int) -> float:
    r = lanczos(hv, f1, m)
    return tridiag_lowest(r["a"], r["b"][1:len(r["a"])])


def lowest_eigvec_T(a, b_off) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    if a.size == 1:
        return np.ones(1)
    w, v = sla.eigh_tridiagonal(a, np.asarray(b_off, dtype=np.float64),
                                select="i", select_range=(0, 0))
    return v[:, 0]


def ground_state_two_pass(hv, f1, m: int):
    """Returns (E0, v): pass 1 builds T_m, pass 2 replays and sums y_k f_k."""
    r = lanczos(hv, f1, m)
    a, b = r["a"], r["b"]
    k = len(a)
    y = lowest_eigvec_T(a, b[1:k])
    e0 = tridiag_lowest(a, b[1:k])
    f = normalise(f1)
    f_prev = np.zeros_like(f)
    v = y[0] * f
    for j in range(k - 1):
        q = hv(f) - b[j] * f_prev
        q = q - a[j] * f
        f_prev, f = f, q / b[j + 1]
        v = v + y[j + 1] * f
    v = v / np.sqrt(_inner(v, v))
    return e0, v


def fix_gauge(v: np.ndarray, ref_index: int) -> np.ndarray:
    mx = np.max(np.abs(v))
    k = ref_index if abs(v[ref_index]) >= 1e-3 * mx else int(np.argmax(np.abs(v)))
    return v if v[k] > 0 else -v
