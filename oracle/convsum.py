"""Convolution sum f(x) = sum_n c_n phi(x - n) on a lattice (oracle; test infrastructure only).

Follows the paper's Eq. conv_sum (h = 1) in its per-coset form (Eq.
coset_form): the sum runs over every lattice site n of every Cartesian coset
whose shifted support contains x.  Nothing of the fast scheme (region of
evaluation, splitting planes, symmetry) is used: candidates are all coset
sites in the bounding box of x - supp(phi), pruned by the zonotope facets
of the support (Sec. 3: the support is the Minkowski sum of the
directions), and every remaining site's phi is evaluated by the box-spline
recurrence.

Basis: phi(w) = |det L| * M_Xi(w + c0), c0 = (1/2) sum_j xi_j.  Scaling by
|det L| gives partition of unity on L when every direction lies on L (the
requirement of Sec. 4.1); the shift by c0 centres phi at the origin so that
phi(-w) = phi(w).

Data layout (shared convention of the whole project): coset k stores its
values in an array indexed by i = (i_0, ..., i_{s-1}), site D i + l_k; the
numpy array has shape (n_{s-1}, ..., n_0) (x fastest in memory).  Sites
outside the stored arrays contribute zero (zero extension).
"""

from itertools import product

import numpy as np

from .boxspline import BoxSplineOracle, facet_normals, _frac_rank, _frac_solve
from .lattice import CosetLattice


class ConvolutionSumOracle:
    def __init__(self, L, Xi):
        self.lat = CosetLattice(L)
        self.bs = BoxSplineOracle(Xi)
        s = self.lat.s
        if self.bs.s != s:
            raise ValueError("Xi and L dimensions differ")
        for j in range(self.bs.n):
            if not self.lat.contains(self.bs.Xi[:, j]):
                raise ValueError("every direction of Xi must lie on the lattice L Z^s")
        self.s = s
        Xi = self.bs.Xi
        self.c0 = 0.5 * Xi.sum(axis=1).astype(float)
        self.half = 0.5 * np.abs(Xi).sum(axis=1).astype(float)       # bbox half widths
        self.normals = np.array(facet_normals(Xi), dtype=float)
        self.bounds = 0.5 * np.abs(self.normals @ Xi.astype(float)).sum(axis=1)
        D = self.lat.D
        self.window = [int(np.ceil(2 * h / D)) + 2 for h in self.half]

    # ----------------------------------------------------------------- basis
    def phi(self, W, want_grad=False):
        """phi at the rows of W (P x s)."""
        W = np.asarray(W, dtype=float).reshape(-1, self.s)
        r = self.bs.eval(W + self.c0, want_grad=want_grad)
        det = float(self.lat.det)
        if want_grad:
            return det * r[0], det * r[1]
        return det * r

    def phi_exact(self, w):
        from fractions import Fraction
        z = [Fraction(a) + Fraction(int(2 * c), 2) for a, c in zip(w, self.c0)]
        return self.lat.det * self.bs.eval_exact(z)

    # ------------------------------------------------------------ candidates
    def _candidates(self, X, dims):
        """All (query, coset, flat index, w = x - site) with site in the closed
        support of phi(x - .) and inside the stored arrays."""
        X = np.asarray(X, dtype=float).reshape(-1, self.s)
        D = self.lat.D
        dims = tuple(int(d) for d in dims)
        offs = np.array(list(product(*[range(w) for w in self.window])), dtype=np.int64)
        qs, ks, flats, Ws = [], [], [], []
        for k, l in enumerate(self.lat.shifts):
            lo = np.floor((X - l - self.half) / D).astype(np.int64)      # (Q, s)
            I = lo[:, None, :] + offs[None, :, :]                        # (Q, C, s)
            site = D * I + l
            W = X[:, None, :] - site
            inside = np.all(np.abs(W @ self.normals.T) <= self.bounds, axis=2)
            inb = np.all((I >= 0) & (I < np.array(dims)), axis=2)
            keep = inside & inb
            qi, ci = np.nonzero(keep)
            Ik = I[qi, ci]
            flat = np.zeros(len(qi), dtype=np.int64)
            stride = 1
            for a in range(self.s):
                flat += Ik[:, a] * stride
                stride *= dims[a]
            qs.append(qi)
            ks.append(np.full(len(qi), k))
            flats.append(flat)
            Ws.append(W[qi, ci])
        return (np.concatenate(qs), np.concatenate(ks), np.concatenate(flats),
                np.concatenate(Ws).reshape(-1, self.s))

    @staticmethod
    def _dims_of(coeffs):
        return tuple(reversed(coeffs[0].shape))

    # ------------------------------------------------------------- forward
    def eval(self, coeffs, X, want_grad=False, chunk=4096):
        """f(x) (and grad f) at the rows of X for coefficient arrays ``coeffs``
        (list of M arrays of shape (n_{s-1}, ..., n_0))."""
        X = np.asarray(X, dtype=float).reshape(-1, self.s)
        if len(coeffs) != self.lat.M:
            raise ValueError("need one coefficient array per coset")
        dims = self._dims_of(coeffs)
        flatc = [np.asarray(c, dtype=float).reshape(-1) for c in coeffs]
        f = np.zeros(len(X))
        g = np.zeros((len(X), self.s)) if want_grad else None
        for q0 in range(0, len(X), chunk):
            Xc = X[q0:q0 + chunk]
            qi, ki, flat, W = self._candidates(Xc, dims)
            cv = np.zeros(len(qi))
            for k in range(self.lat.M):
                sel = ki == k
                cv[sel] = flatc[k][flat[sel]]
            if want_grad:
                ph, dph = self.phi(W, want_grad=True)
                for a in range(self.s):
                    g[q0:q0 + len(Xc), a] = np.bincount(qi, weights=cv * dph[:, a], minlength=len(Xc))
            else:
                ph = self.phi(W)
            f[q0:q0 + len(Xc)] = np.bincount(qi, weights=cv * ph, minlength=len(Xc))
        return (f, g) if want_grad else f

    def eval_exact(self, coeffs, x):
        """f(x) exactly (Fractions) for one query x; coefficients are converted
        exactly from their stored binary values."""
        from fractions import Fraction
        dims = self._dims_of(coeffs)
        qi, ki, flat, W = self._candidates(np.asarray(x, dtype=float)[None, :], dims)
        xf = [Fraction(float(v)) for v in x]
        total = Fraction(0)
        for k, fl in zip(ki, flat):
            l = self.lat.shifts[k]
            idx = []
            rem = int(fl)
            for a in range(self.s):
                idx.append(rem % dims[a])
                rem //= dims[a]
            site = [self.lat.D * i + int(li) for i, li in zip(idx, l)]
            w = [a - b for a, b in zip(xf, site)]
            c = Fraction(float(np.asarray(coeffs[k]).reshape(-1)[fl]))
            total += c * self.phi_exact(w)
        return total

    # ------------------------------------------------------------- adjoint
    def adjoint(self, X, gout, dims, chunk=4096):
        """Transpose of c -> f: returns M arrays r_k[i] = sum_q g_q phi(x_q - site)."""
        X = np.asarray(X, dtype=float).reshape(-1, self.s)
        gout = np.asarray(gout, dtype=float).reshape(-1)
        dims = tuple(int(d) for d in dims)
        size = int(np.prod(dims))
        out = [np.zeros(size) for _ in range(self.lat.M)]
        for q0 in range(0, len(X), chunk):
            Xc = X[q0:q0 + chunk]
            qi, ki, flat, W = self._candidates(Xc, dims)
            ph = self.phi(W)
            contrib = gout[q0 + qi] * ph
            for k in range(self.lat.M):
                sel = ki == k
                out[k] += np.bincount(flat[sel], weights=contrib[sel], minlength=size)
        return [o.reshape(tuple(reversed(dims))) for o in out]

    def adjoint_at(self, X, gout, sites):
        """The transpose of c -> f at chosen sites only.  For every (k, i) in
        ``sites`` (coset k, array index i as an s-tuple) returns
        sum_q g_q phi(x_q - m) with m = D i + l_k, summed over every query
        whose x_q lies in the support of phi(. - m): the column of Eq.
        conv_sum that belongs to c_m.  Queries are found by sorting them
        along axis 0 once and keeping those inside the support's bounding
        box around m; the rest is the plain definition."""
        X = np.asarray(X, dtype=float).reshape(-1, self.s)
        gout = np.asarray(gout, dtype=float).reshape(-1)
        order = np.argsort(X[:, 0], kind="stable")
        xs = X[order, 0]
        out = np.zeros(len(sites))
        for j, (k, idx) in enumerate(sites):
            m = self.lat.D * np.asarray(idx, dtype=float) + np.asarray(self.lat.shifts[k], dtype=float)
            lo = np.searchsorted(xs, m[0] - self.half[0], side="left")
            hi = np.searchsorted(xs, m[0] + self.half[0], side="right")
            cand = order[lo:hi]
            W = X[cand] - m
            keep = np.all(np.abs(W) <= self.half, axis=1)
            cand, W = cand[keep], W[keep]
            if len(cand):
                out[j] = float(np.sum(gout[cand] * self.phi(W)))
        return out

    def nonzero_count(self, X, dims):
        """Number of sites with phi(x - site) != 0 per query (Table 1's
        '# Lookups' reading: sites with nonzero weight)."""
        X = np.asarray(X, dtype=float).reshape(-1, self.s)
        qi, ki, flat, W = self._candidates(X, dims)
        ph = self.phi(W)
        return np.bincount(qi[ph != 0], minlength=len(X))
