"""Pins of the stored ground-state energies (tests/golden/e0_*.txt, written from the oracle alone).

Each stored value is checked against what fixes it independently of the run that produced it:
a second algorithm (ARPACK), a second start vector, the convergence of the Ritz sequence
(interlacing: E0(j) non-increasing), and for the batch draw the bounds and shape that the
variational principle puts on E0(U) (Hellmann-Feynman: non-decreasing; a minimum of functions
linear in U: concave; between the U = 0 band sum and the energy of a U = 0 determinant).
"""

import numpy as np

from tests.golden.load import arpack_e0, batch34, energies, lanczos_e0


def _ritz(name):
    return np.array([float(e) for kind, _s, j, e in energies(name) if kind == "lanczos"])


def test_c2_lanczos_agrees_with_arpack():
    """4x4 5+5, U = 4: Alg. 1 after 200 steps and ARPACK's implicitly restarted iteration agree."""
    e_l, e_a = lanczos_e0("torus4x4_5x5", 200), arpack_e0("torus4x4_5x5")
    assert abs(e_l - e_a) <= 1e-12 * abs(e_a)
    assert -24.0 <= e_a <= -24.0 + 4.0 * 25 / 16   # band sum <= E0 <= U = 0 determinant energy


def test_c5_two_starts_agree():
    """4x4 8+8, U = 4: runs from two independent start vectors reach the same E0."""
    e5, e55 = lanczos_e0("torus4x4_8x8", 200), lanczos_e0("torus4x4_8x8_seed55", 200)
    assert abs(e5 - e55) <= 1e-12 * abs(e5)
    assert -24.0 <= e5 <= -24.0 + 4.0 * 64 / 16


def test_ritz_sequences_converge_monotonically():
    for name in ("torus4x4_5x5", "torus4x4_8x8", "torus4x4_8x8_seed55"):
        e = _ritz(name)
        assert np.all(np.diff(e) <= 1e-12 * abs(e[-1])), name
        assert abs(e[-1] - e[-3]) <= 1e-13 * abs(e[-1]), name   # converged over the last 20 steps


def test_batch34_energy_shape_in_u():
    rows = batch34()
    assert len(rows) >= 20
    band = {3: -16.0, 4: -20.0}   # sum of the N lowest levels -2t(cos kx + cos ky) per species, twice
    for n in (3, 4):
        pts = sorted((u, e) for _, nn, u, _, _, e in rows if nn == n)
        us = np.array([p[0] for p in pts])
        es = np.array([p[1] for p in pts])
        assert np.all(es >= band[n] - 1e-12)
        assert np.all(es <= band[n] + us * n * n / 16.0 + 1e-12)
        assert np.all(np.diff(es) >= -1e-12)                       # dE0/dU = double occupancy >= 0
        slopes = np.diff(es) / np.maximum(np.diff(us), 1e-300)
        keep = np.diff(us) > 1e-3
        s = slopes[keep]
        assert np.all(np.diff(s) <= 1e-9)                          # concave in U
