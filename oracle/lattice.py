"""Cartesian coset decomposition of an integer lattice (oracle; test infrastructure only).

Sec. 4.1 of the paper writes the lattice L Z^s as a union of M shifted copies
of a sub-lattice GL Z^s and, for the GPU, picks G so that GL = D is diagonal:
each coset is then a plain s-dimensional array.  The oracle uses the scalar
choice D I with the smallest positive integer D for which D Z^s is a
sub-lattice of L Z^s, and orders the shifts l_k in [0, D)^s by the integer
sum_a l_a D^a (last coordinate most significant), which puts the zero shift
first.  Coset array index i corresponds to the lattice site D i + l_k.
"""

from fractions import Fraction
from itertools import product

import numpy as np

from .boxspline import _frac_det, _frac_solve


class CosetLattice:
    def __init__(self, L):
        L = np.asarray(L, dtype=np.int64)
        s = L.shape[0]
        if L.shape != (s, s):
            raise ValueError("L must be square")
        det = _frac_det(L.tolist())
        if det == 0:
            raise ValueError("L must have full rank")
        self.L, self.s, self.det = L, s, abs(int(det))
        cols = _frac_solve(L.tolist(), [[int(a == b) for a in range(s)] for b in range(s)])
        Linv = [[cols[b][a] for b in range(s)] for a in range(s)]      # L^{-1}
        self._Linv = Linv
        den = 1
        for row in Linv:
            for v in row:
                den = den * v.denominator // np.gcd(den, v.denominator)
        self.D = int(den)
        shifts = [v for v in product(range(self.D), repeat=s) if self.contains(v)]
        shifts.sort(key=lambda v: sum(c * self.D ** a for a, c in enumerate(v)))
        self.shifts = [np.array(v, dtype=np.int64) for v in shifts]
        self.M = len(self.shifts)
        if self.M * self.det != self.D ** s:
            raise AssertionError("coset count does not match D^s / |det L|")

    def contains(self, v):
        """True iff the integer vector v lies on L Z^s (L^{-1} v integral)."""
        for row in self._Linv:
            if sum(Fraction(r) * int(c) for r, c in zip(row, v)).denominator != 1:
                return False
        return True
