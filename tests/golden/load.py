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
