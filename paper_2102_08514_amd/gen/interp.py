"""Slow CPU interpreter of the fast evaluation scheme over generated tables.

It executes, per query and per coset, exactly the steps the GPU kernels take
(the paper's Algorithm 1 with the symmetry fold in place of the sigma
table): shift into the coset cell, fold into the fundamental chamber, find
the sub-region from the splitting planes, rename the stencil sites through
the fold, gather, and evaluate the sub-region's polynomials.  Used offline
to check tables exactly (Fractions) and, in FP64, against independent
evaluations.
"""

from fractions import Fraction
from math import floor

import numpy as np


def fold_point(u, fold):
    """Signed permutation T with u' = T u in the fundamental chamber.
    Returns (u', perm, tau) with u'_r = tau_r * u[perm[r]]."""
    s = len(u)
    sg = [1 if v >= 0 else -1 for v in u]
    a = [abs(v) for v in u]
    perm = sorted(range(s), key=lambda i: (-a[i], i))
    tau = [sg[p] for p in perm]
    if fold == "D":
        neg = sum(1 for v in sg if v < 0)
        if neg % 2 == 1:
            tau[-1] = -tau[-1]
    up = [tau[r] * u[perm[r]] for r in range(s)]
    return up, perm, tau


def site_offset(j, perm, tau):
    """Original-frame offset o of folded-frame site j: o - 1/2 = T^{-1}(j - 1/2)."""
    s = len(j)
    o = [0] * s
    for r in range(s):
        o[perm[r]] = j[r] if tau[r] > 0 else 1 - j[r]
    return o


def orbit_of(tables, up):
    from .analysis import plane_ties
    ties = plane_ties(tables)
    code = 0
    for i, (nu, off) in enumerate(tables.planes):
        v = sum(a * b for a, b in zip(nu, up)) - off
        if v > 0 or (v == 0 and ties[i]):
            code |= 1 << i
    sig = getattr(tables, "sigma", None)
    if sig:
        return sig["table"][code % sig["r"]]          # Sec. 4.2: sigma(q mod r)
    return tables.orbit_table[code]


def eval_exact(tables, coef, x):
    """f(x) in exact arithmetic; coef(k, i) returns the coefficient of coset k
    at array index i (a tuple), or 0 outside the stored data."""
    s, D = tables.s, tables.D
    x = [Fraction(v) for v in x]
    h = Fraction(D, 2)
    total = Fraction(0)
    for k, l in enumerate(tables.lat.shifts):
        xp = [a - b for a, b in zip(x, l)]
        i = [floor(v / D) for v in xp]
        u = [v - D * ii - h for v, ii in zip(xp, i)]
        up, perm, tau = fold_point(u, tables.fold)
        orb = tables.orbits[orbit_of(tables, up)]
        for j, P in zip(orb["stencil"], orb["polys"]):
            o = site_offset(j, perm, tau)
            idx = tuple(a + b for a, b in zip(i, o))
            total += coef(k, idx) * P(up)
    return total


class FloatTables:
    """FP64 arrays extracted from exact tables for the vectorised interpreter."""

    def __init__(self, tables):
        self.t = tables
        self.mons = tables.monomials()
        self.A = [np.array([[float(v) for v in row] for row in tables.coefficient_matrix(k)])
                  for k in range(tables.K)]
        self.stencil = [np.array(o["stencil"], dtype=np.int64) for o in tables.orbits]
        self.planes = [(np.array(nu, dtype=float), float(off)) for nu, off in tables.planes]
        from .analysis import plane_ties
        self.ties = plane_ties(tables)
        self.orbit_table = np.array(tables.orbit_table, dtype=np.int64)
        sig = getattr(tables, "sigma", None)
        self.sigma = (sig["r"], np.array(sig["table"], dtype=np.int64)) if sig else None


def eval_fp64(ft, coeffs, X):
    """Vectorised FP64 interpreter.  coeffs: list of M arrays (n_{s-1},...,n_0)."""
    t = ft.t
    s, D = t.s, t.D
    X = np.asarray(X, dtype=np.float64).reshape(-1, s)
    dims = tuple(reversed(coeffs[0].shape))
    f = np.zeros(len(X))
    for k, l in enumerate(t.lat.shifts):
        xp = X - np.array(l, dtype=float)
        i = np.floor(xp / D).astype(np.int64)
        u = xp - D * i - D / 2.0
        sg = np.where(u >= 0, 1, -1)
        a = np.abs(u)
        perm = np.argsort(-a, axis=1, kind="stable")
        tau = np.take_along_axis(sg, perm, axis=1)
        if t.fold == "D":
            odd = (np.sum(sg < 0, axis=1) % 2) == 1
            tau[odd, -1] *= -1
        up = tau * np.take_along_axis(u, perm, axis=1)
        code = np.zeros(len(X), dtype=np.int64)
        for b, ((nu, off), tie) in enumerate(zip(ft.planes, ft.ties)):
            v = up @ nu - off
            code |= ((v > 0) | ((v == 0) & tie)).astype(np.int64) << b
        orbit = ft.orbit_table[code] if ft.sigma is None else ft.sigma[1][code % ft.sigma[0]]
        mono = np.stack([np.prod(up ** np.array(e), axis=1) for e in ft.mons], axis=1)
        flat_c = coeffs[k].reshape(-1)
        for ob in range(t.K):
            sel = np.nonzero(orbit == ob)[0]
            if len(sel) == 0:
                continue
            w = mono[sel] @ ft.A[ob].T                        # (q, stencil)
            for r, j in enumerate(ft.stencil[ob]):
                o = np.empty((len(sel), s), dtype=np.int64)
                for rr in range(s):
                    p = perm[sel, rr]
                    o[np.arange(len(sel)), p] = np.where(tau[sel, rr] > 0, j[rr], 1 - j[rr])
                idx = i[sel] + o
                ok = np.all((idx >= 0) & (idx < np.array(dims)), axis=1)
                flat = np.zeros(len(sel), dtype=np.int64)
                stride = 1
                for aa in range(s):
                    flat += idx[:, aa] * stride
                    stride *= dims[aa]
                cv = np.where(ok, flat_c[np.where(ok, flat, 0)], 0.0)
                f[sel] += cv * w[:, r]
    return f
