"""Integer lattice helpers for the offline table generator.

Cartesian coset decomposition (Sec. 4.1): the lattice L Z^s is the union of
M cosets D Z^s + l_k where D is the smallest positive integer with
D Z^s contained in L Z^s (GL = D I).  Shifts l_k in [0, D)^s are ordered by
sum_a l_a D^a (last coordinate most significant), so l_0 = 0.
"""

from fractions import Fraction
from itertools import product
from math import gcd


def _frac_rows(M):
    return [[Fraction(v) for v in row] for row in M]


def int_det(M):
    A = _frac_rows(M)
    n = len(A)
    det = Fraction(1)
    for c in range(n):
        p = next((r for r in range(c, n) if A[r][c] != 0), None)
        if p is None:
            return 0
        if p != c:
            A[c], A[p] = A[p], A[c]
            det = -det
        det *= A[c][c]
        for r in range(c + 1, n):
            f = A[r][c] / A[c][c]
            if f:
                for k in range(c, n):
                    A[r][k] -= f * A[c][k]
    assert det.denominator == 1
    return int(det)


def int_rank(M):
    A = _frac_rows(M)
    if not A:
        return 0
    rows, cols = len(A), len(A[0])
    r = 0
    for c in range(cols):
        p = next((i for i in range(r, rows) if A[i][c] != 0), None)
        if p is None:
            continue
        A[r], A[p] = A[p], A[r]
        for i in range(rows):
            if i != r and A[i][c] != 0:
                f = A[i][c] / A[r][c]
                A[i] = [x - f * y for x, y in zip(A[i], A[r])]
        r += 1
        if r == rows:
            break
    return r


def primitive_normal(vecs, s):
    """Primitive integer normal of the hyperplane spanned by s-1 vectors
    (first nonzero entry positive), or None if they do not span one."""
    if s == 1:
        return (1,)
    nu = []
    for a in range(s):
        minor = [[v[b] for b in range(s) if b != a] for v in vecs]
        nu.append((-1) ** a * int_det(minor))
    if not any(nu):
        return None
    g = 0
    for v in nu:
        g = gcd(g, abs(v))
    nu = [v // g for v in nu]
    if next(v for v in nu if v) < 0:
        nu = [-v for v in nu]
    return tuple(nu)


def inverse(M):
    n = len(M)
    A = [list(map(Fraction, M[i])) + [Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[p] = A[p], A[c]
        piv = A[c][c]
        A[c] = [v / piv for v in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return [row[n:] for row in A]


class Lattice:
    def __init__(self, L):
        self.L = [[int(v) for v in row] for row in L]
        self.s = len(self.L)
        self.det = abs(int_det(self.L))
        if self.det == 0:
            raise ValueError("singular lattice matrix")
        self.Linv = inverse(self.L)
        D = 1
        for row in self.Linv:
            for v in row:
                D = D * v.denominator // gcd(D, v.denominator)
        self.D = D
        shifts = [v for v in product(range(D), repeat=self.s) if self.contains(v)]
        shifts.sort(key=lambda v: sum(c * D ** a for a, c in enumerate(v)))
        self.shifts = shifts
        self.M = len(shifts)
        assert self.M * self.det == D ** self.s

    def contains(self, v):
        return all(sum(r * int(c) for r, c in zip(row, v)).denominator == 1 for row in self.Linv)
