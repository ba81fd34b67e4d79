"""Exact piecewise-polynomial (PP) form of a box spline, derived offline from
the paper's convolution definition (Sec. 3).

The paper defines M_Xi by convolving along one direction at a time,

    M_Xi(z) = int_0^1 M_{Xi\\xi}(z - t xi) dt          (n > s),

with the base case n = s: 1/|det Xi| on the parallelepiped Xi [0,1)^s.
(The printed integrand argument has its sign reversed; this is the form that
agrees with the stated support, the Minkowski sum of the directions.)

`BoxSplinePP.piece(q)` returns the polynomial that equals M_Xi on the mesh
cell containing the generic rational point q.  It integrates symbolically:
along the segment q - t xi, t in [0,1], the integrand is polynomial between
consecutive crossings of the mesh planes of M_{Xi\\xi} (Sec. 3: pieces are
delimited by hyperplanes spanned by s-1 directions, shifted by sums of
directions).  Each crossing parameter is an affine function of z, so every
sub-integral is an exact polynomial in z.  Results are memoised per
(direction subset, mesh cell).

This is independent of the recurrence used elsewhere for testing: it
implements the defining integral.
"""

from bisect import bisect_right
from fractions import Fraction
from itertools import combinations

import numpy as np

from .poly import Poly, integrate_along
from .lattice import int_det, int_rank, primitive_normal


_THETA = Fraction(38197, 100003)


class DegeneratePoint(Exception):
    """q lies on a mesh plane or two crossings coincide; perturb and retry."""


class BoxSplinePP:
    def __init__(self, Xi):
        self.Xi = [tuple(int(v) for v in col) for col in zip(*Xi)]   # list of directions
        self.n = len(self.Xi)
        self.s = len(self.Xi[0])
        if int_rank(list(zip(*self.Xi))) != self.s:
            raise ValueError("Xi must span")
        self._mesh = {}
        self._memo = {}
        self._span = {}
        self._rng = np.random.default_rng(2021)

    # ------------------------------------------------------------ mesh data
    def cols(self, mask):
        return [j for j in range(self.n) if (mask >> j) & 1]

    def spans(self, mask):
        r = self._span.get(mask)
        if r is None:
            cols = self.cols(mask)
            r = len(cols) >= self.s and int_rank([[self.Xi[j][a] for j in cols] for a in range(self.s)]) == self.s
            self._span[mask] = r
        return r

    def mesh(self, mask):
        """[(normal, sorted offsets)] of the planes carrying breakpoints of M_mask."""
        m = self._mesh.get(mask)
        if m is not None:
            return m
        cols = self.cols(mask)
        normals = set()
        for sub in combinations(cols, self.s - 1):
            vecs = [self.Xi[j] for j in sub]
            nu = primitive_normal(vecs, self.s)
            if nu is not None:
                normals.add(nu)
        sums = set()
        for r in range(len(cols) + 1):
            for sub in combinations(cols, r):
                sums.add(tuple(sum(self.Xi[j][a] for j in sub) for a in range(self.s)))
        m = []
        for nu in sorted(normals):
            offs = sorted({sum(a * b for a, b in zip(nu, sm)) for sm in sums})
            m.append((nu, offs))
        self._mesh[mask] = m
        return m

    def cell_key(self, mask, q):
        key = [mask]
        for nu, offs in self.mesh(mask):
            v = sum(Fraction(a) * b for a, b in zip(nu, q))
            pos = bisect_right(offs, v)
            if pos and offs[pos - 1] == v:
                raise DegeneratePoint()
            key.append(pos)
        return tuple(key)

    def _cuts(self, sub, xi, q):
        """Sorted crossings (t, t(z)) of the segment q - t xi, t in (0,1), with
        the mesh planes of M_sub; None if two different planes coincide."""
        cuts = []
        for nu, offs in self.mesh(sub):
            den = sum(a * b for a, b in zip(nu, xi))
            if den == 0:
                continue
            nq = sum(Fraction(a) * b for a, b in zip(nu, q))
            for off in offs:
                t = (nq - off) / den
                if 0 < t < 1:
                    # affine crossing parameter t(z) = (nu.z - off) / den
                    cuts.append((t, Poly.affine([Fraction(a, den) for a in nu], Fraction(-off, den))))
        cuts.sort(key=lambda c: c[0])
        for a, b in zip(cuts, cuts[1:]):
            if a[0] == b[0] and a[1] != b[1]:
                return None
        return cuts

    # ------------------------------------------------------------ pieces
    def piece(self, q, mask=None):
        mask = (1 << self.n) - 1 if mask is None else mask
        q = tuple(Fraction(v) for v in q)
        key = self.cell_key(mask, q)
        hit = self._memo.get(key)
        if hit is not None:
            return hit
        cols = self.cols(mask)
        s = self.s
        if len(cols) == s:
            B = [[self.Xi[j][a] for j in cols] for a in range(s)]
            det = int_det(B)
            # u = B^{-1} q by Cramer's rule; inside iff 0 < u_i < 1 (q generic)
            inside = True
            for i in range(s):
                Bi = [row[:] for row in B]
                for a in range(s):
                    Bi[a][i] = q[a]
                ui = _det_frac(Bi) / det
                if ui <= 0 or ui >= 1:
                    if ui == 0 or ui == 1:
                        raise DegeneratePoint()
                    inside = False
                    break
            res = Poly.const(s, Fraction(1, abs(det)) if inside else 0)
        else:
            j = next(j for j in reversed(cols) if self.spans(mask & ~(1 << j)))
            sub = mask & ~(1 << j)
            xi = self.Xi[j]
            cuts = self._cuts(sub, xi, q)
            # Two different planes crossing the segment at the same t: the
            # point sits on a (non-mesh) hyperplane where the crossing order
            # flips.  M_mask is one polynomial on the whole cell, so any point
            # of the same cell will do: move q to a random nearby point.
            scale = Fraction(1, 10 ** 6)
            while cuts is None:
                d = tuple(Fraction(int(self._rng.integers(-10 ** 6, 10 ** 6)), 10 ** 6) * scale for _ in range(s))
                q2 = tuple(a + b for a, b in zip(q, d))
                try:
                    same = self.cell_key(mask, q2) == key
                except DegeneratePoint:
                    same = False
                if same:
                    q = q2
                    cuts = self._cuts(sub, xi, q)
                else:
                    scale /= 10
            pts = [(Fraction(0), Poly.const(s, 0))] + cuts + [(Fraction(1), Poly.const(s, 1))]
            res = Poly(s)
            for (ta, fa), (tb, fb) in zip(pts, pts[1:]):
                if ta == tb:
                    continue
                # an interior point of the interval; not the midpoint, which
                # for parallel planes lands on the integer-offset planes halfway
                tm = ta + _THETA * (tb - ta)
                qm = tuple(qa - tm * x for qa, x in zip(q, xi))
                pm = self.piece(qm, sub)
                if pm.is_zero():
                    continue
                res = res + integrate_along(pm, xi, fa, fb)
        self._memo[key] = res
        return res


def _det_frac(M):
    A = [[Fraction(v) for v in row] for row in M]
    n = len(A)
    det = Fraction(1)
    for c in range(n):
        p = next((r for r in range(c, n) if A[r][c] != 0), None)
        if p is None:
            return Fraction(0)
        if p != c:
            A[c], A[p] = A[p], A[c]
            det = -det
        det *= A[c][c]
        for r in range(c + 1, n):
            f = A[r][c] / A[c][c]
            if f:
                for k in range(c, n):
                    A[r][k] -= f * A[c][k]
    return det
