"""Sparse multivariate polynomials with exact rational coefficients.

Used offline by the table generator only.  A polynomial in ``nv`` variables
is a dict mapping exponent tuples to ``fractions.Fraction``.
"""

from fractions import Fraction
from math import comb


class Poly:
    __slots__ = ("nv", "t")

    def __init__(self, nv, terms=None):
        self.nv = nv
        self.t = {} if terms is None else {e: c for e, c in terms.items() if c != 0}

    # ------------------------------------------------------------- builders
    @staticmethod
    def const(nv, c):
        return Poly(nv, {(0,) * nv: Fraction(c)})

    @staticmethod
    def affine(coef, const):
        """sum_a coef[a] z_a + const."""
        nv = len(coef)
        terms = {(0,) * nv: Fraction(const)}
        for a, c in enumerate(coef):
            if c:
                e = [0] * nv
                e[a] = 1
                terms[tuple(e)] = Fraction(c)
        return Poly(nv, terms)

    def is_zero(self):
        return not self.t

    def degree(self):
        return max((sum(e) for e in self.t), default=-1)

    # ------------------------------------------------------------- algebra
    def __add__(self, o):
        r = dict(self.t)
        for e, c in o.t.items():
            v = r.get(e, 0) + c
            if v:
                r[e] = v
            else:
                r.pop(e, None)
        return Poly(self.nv, r)

    def __sub__(self, o):
        return self + o.scale(-1)

    def scale(self, k):
        k = Fraction(k)
        if k == 0:
            return Poly(self.nv)
        return Poly(self.nv, {e: c * k for e, c in self.t.items()})

    def scale_vars(self, k):
        """Q(z) = P(k z) for a scalar k."""
        k = Fraction(k)
        return Poly(self.nv, {e: c * k ** sum(e) for e, c in self.t.items()})

    def __mul__(self, o):
        r = {}
        for e1, c1 in self.t.items():
            for e2, c2 in o.t.items():
                e = tuple(a + b for a, b in zip(e1, e2))
                r[e] = r.get(e, 0) + c1 * c2
        return Poly(self.nv, r)

    def __call__(self, point):
        tot = Fraction(0)
        for e, c in self.t.items():
            v = c
            for x, k in zip(point, e):
                if k:
                    v *= Fraction(x) ** k
            tot += v
        return tot

    def shift(self, d):
        """Q(z) = P(z + d) for a constant vector d."""
        r = Poly(self.nv)
        cache = {}
        for e, c in self.t.items():
            term = Poly.const(self.nv, c)
            for a, k in enumerate(e):
                if k == 0:
                    continue
                key = (a, k)
                if key not in cache:
                    cache[key] = _power(Poly.affine([int(b == a) for b in range(self.nv)], d[a]), k)
                term = term * cache[key]
            r = r + term
        return r

    def __eq__(self, o):
        return isinstance(o, Poly) and self.nv == o.nv and self.t == o.t

    def __repr__(self):
        return f"Poly({self.nv}, {self.t})"


def _power(p, k):
    r = Poly.const(p.nv, 1)
    for _ in range(k):
        r = r * p
    return r


def integrate_along(P, xi, lo, hi):
    """I(z) = int_{lo(z)}^{hi(z)} P(z - t xi) dt, with lo/hi affine in z
    (given as Poly of degree <= 1).  Exact."""
    s = P.nv
    # R(z, t) = int_0^t P(z - tau xi) dtau, stored as {k: poly in z} for t^k
    R = {}
    for e, c in P.t.items():
        # prod_a (z_a - t xi_a)^{e_a} = sum over j_a C(e_a, j_a) z_a^{e_a-j_a} (-xi_a t)^{j_a}
        parts = [((), Fraction(c), 0)]
        for a in range(s):
            new = []
            for ze, co, tk in parts:
                for j in range(e[a] + 1):
                    f = comb(e[a], j) * (-xi[a]) ** j
                    if f == 0:
                        continue
                    new.append((ze + (e[a] - j,), co * f, tk + j))
            parts = new
        for ze, co, tk in parts:
            # integral of t^tk from 0 to t is t^(tk+1)/(tk+1)
            k = tk + 1
            bucket = R.setdefault(k, {})
            bucket[ze] = bucket.get(ze, 0) + co / k
    out = Poly(s)
    for bound, sign in ((hi, 1), (lo, -1)):
        pw = Poly.const(s, 1)
        powers = {0: pw}
        for k in sorted(R):
            while max(powers) < k:
                powers[max(powers) + 1] = powers[max(powers)] * bound
            zpart = Poly(s, R[k])
            out = out + (zpart * powers[k]).scale(sign)
    return out


def monomials(nv, deg):
    """Exponent tuples of total degree <= deg in graded order (degree, then
    reverse-lexicographic), the layout used by the emitted tables."""
    out = []
    for d in range(deg + 1):
        out.extend(_exps(nv, d))
    return out


def _exps(nv, d):
    if nv == 1:
        return [(d,)]
    res = []
    for k in range(d, -1, -1):
        for rest in _exps(nv - 1, d - k):
            res.append((k,) + rest)
    return res
