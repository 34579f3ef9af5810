"""Discrete velocity sets used by the oracle (Sec. II.A).

The paper fixes c_s^2 = 1/3 for the standard velocity sets (Sec. II.A, after
eq. Maxwellian); the velocities and weights of D2Q9, D3Q19 and D3Q27 are the textbook
Gauss-Hermite quadratures.  Direction order (shared by contract with the C-ABI,
so that a (node, dir) pair means the same thing on both sides):

D2Q9   0:(0,0) 1:(1,0) 2:(-1,0) 3:(0,1) 4:(0,-1) 5:(1,1) 6:(1,-1) 7:(-1,1) 8:(-1,-1)
D3Q19  0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..10 = (+-1,+-1,0); 11..14 = (+-1,0,+-1);
       15..18 = (0,+-1,+-1); each pair group in sign order (+,+),(+,-),(-,+),(-,-).
D3Q27  0..18 as D3Q19; 19..26 = the corners (+-1,+-1,+-1), sign order
       (+,+,+),(+,+,-),(+,-,+),(+,-,-),(-,+,+),(-,+,-),(-,-,+),(-,-,-).

Status: pinned (moment identities and isotropy, tests/test_oracle_lattice.py).
"""
from fractions import Fraction

import numpy as np

from . import precision as prec

CS2 = 1.0 / 3.0


class Lattice:
    """A velocity set: integer velocities c (Q x 3), weights w (Q), opposite index."""

    def __init__(self, name, dim, velocities, weights):
        self.name = name
        self.d = dim
        self.c = np.array(velocities, dtype=np.int64)
        self.q = len(velocities)
        self.w_exact = [Fraction(x) for x in weights]
        # opposite direction: the unique j with c_j = -c_i
        self.opp = np.array(
            [int(np.flatnonzero((self.c == -self.c[i]).all(axis=1))[0]) for i in range(self.q)],
            dtype=np.int64,
        )

    @property
    def w(self):
        """Weights in the oracle's current arithmetic type (each fraction rounded once)."""
        cache = self.__dict__.setdefault("_w", {})
        if prec.REAL not in cache:
            cache[prec.REAL] = np.array([prec.scalar(x) for x in self.w_exact], dtype=prec.REAL)
            cache[prec.REAL].setflags(write=False)
        return cache[prec.REAL]

    @property
    def cs2(self):
        """c_s^2 = 1/3 in the current arithmetic type."""
        return prec.scalar(Fraction(1, 3))


def _d2q9():
    c = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
         (1, 1, 0), (1, -1, 0), (-1, 1, 0), (-1, -1, 0)]
    w = ["4/9"] + ["1/9"] * 4 + ["1/36"] * 4
    return Lattice("D2Q9", 2, c, w)


def _d3q19():
    c = [(0, 0, 0)]
    c += [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    signs = [(1, 1), (1, -1), (-1, 1), (-1, -1)]
    c += [(a, b, 0) for a, b in signs]
    c += [(a, 0, b) for a, b in signs]
    c += [(0, a, b) for a, b in signs]
    w = ["1/3"] + ["1/18"] * 6 + ["1/36"] * 12
    return Lattice("D3Q19", 3, c, w)


def _d3q27():
    c = [tuple(v) for v in _d3q19().c.tolist()]
    c += [(a, b, g) for a in (1, -1) for b in (1, -1) for g in (1, -1)]
    w = ["8/27"] + ["2/27"] * 6 + ["1/54"] * 12 + ["1/216"] * 8
    return Lattice("D3Q27", 3, c, w)


D2Q9 = _d2q9()
D3Q19 = _d3q19()
D3Q27 = _d3q27()


def get(name):
    return {"D2Q9": D2Q9, "D3Q19": D3Q19, "D3Q27": D3Q27}[name]
