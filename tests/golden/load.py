"""Readers for the text fixtures in this folder (no arithmetic of the method)."""

import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def ell_fig2():
    out = {}
    with open(os.path.join(HERE, "ell_fig2.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, vals = line.split(":")
            parts = head.split()
            name, shape = parts[0], tuple(int(s) for s in parts[1:])
            arr = np.array([float(v) for v in vals.split()])
            out[name] = arr.reshape(shape)
    return out


def paper_sizes():
    rows = []
    with open(os.path.join(HERE, "paper_sizes.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            kind, ns, nu, nd, val, tol = line.split()
            rows.append((kind, int(ns), int(nu), int(nd), float(val), float(tol)))
    return rows


def energies(name):
    """Rows of e0_<name>.txt (written by make_energies.py from the oracle): lists of fields."""
    rows = []
    with open(os.path.join(HERE, "e0_%s.txt" % name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def lanczos_e0(name, steps):
    """E0 of T_steps from the oracle's Alg. 1 run recorded in e0_<name>.txt."""
    for kind, _seed, j, e in energies(name):
        if kind == "lanczos" and int(j) == steps:
            return float(e)
    raise KeyError((name, steps))


def arpack_e0(name):
    for kind, _seed, _j, e in energies(name):
        if kind == "arpack":
            return float(e)
    raise KeyError(name)


def batch34():
    """(item index, N, U, start seed, steps, E0) of the batch items with 3 or 4 particles per species."""
    return [(int(i), int(n), float(u), int(s), int(k), float(e)) for _, i, n, u, s, k, e in energies("batch34")]
