"""Parsers for the text fixtures in this folder."""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _num(tok: str):
    tok = tok.strip()
    try:
        return Fraction(tok)
    except ValueError:
        return complex(tok)


def _matrix(text: str, n: int):
    rows = [r.split() for r in text.split(";")]
    if len(rows) != n or any(len(r) != n for r in rows):
        raise ValueError("bad matrix row count in fixture: %r" % text)
    vals = [[_num(t) for t in r] for r in rows]
    cplx = any(isinstance(v, complex) for r in vals for v in r)
    dt = np.complex128 if cplx else np.float64
    out = np.zeros((n, n), dtype=dt)
    for i in range(n):
        for j in range(n):
            v = vals[i][j]
            out[i, j] = complex(v) if cplx else float(v)
    return out, vals


def closed_forms():
    """Yield (name, T, U, U_exact_entries) from closed_forms.txt."""
    cases = []
    cur = {}
    with open(os.path.join(HERE, "closed_forms.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(" ")
            if key == "case":
                if cur:
                    cases.append(cur)
                cur = {"name": rest}
            elif key == "n":
                cur["n"] = int(rest)
            elif key in ("T", "U"):
                cur[key] = _matrix(rest, cur["n"])
    if cur:
        cases.append(cur)
    for c in cases:
        yield c["name"], c["T"][0], c["U"][0], c["U"][1]
