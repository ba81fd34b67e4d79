"""Box spline M_Xi by the de Boor--Hoellig recurrence (oracle; test infrastructure only).

Definition followed: Sec. 3 of the paper defines M_Xi for an s x n direction
matrix Xi (n >= s, rank s) by convolution along one direction at a time,
down to the base case n = s where M_Xi is 1/|det Xi| on the half-open
parallelepiped Xi [0,1)^s and 0 elsewhere.  (The printed convolution
argument has its sign reversed; the standard form M_{Xi\\xi}(x - t xi) is
used, which is the one consistent with the stated support.)

The oracle evaluates that function with the classical recurrence of de Boor
and Hoellig (de Boor, Hoellig & Riemenschneider, "Box Splines", 1993): for
any t with Xi t = z,

    (n - s) M_Xi(z) = sum_xi  t_xi M_{Xi\\xi}(z) + (1 - t_xi) M_{Xi\\xi}(z - xi).

Terms whose remaining matrix Xi\\xi does not span R^s are singular measures
carried by mesh planes and vanish at the generic (perturbed) point, so they
are dropped.  Its directional derivative is D_xi M_Xi = M_{Xi\\xi} -
M_{Xi\\xi}(. - xi).

Ties.  The paper points out (Sec. 2) that a recursive evaluator is only
stable when every decision on a separating plane is taken consistently.
Here every base-case membership test is decided for z + eps v with one fixed
lexicographic direction v = (1, 2^-10, 2^-20, ...) shared by all nodes and all
sites, i.e. the oracle returns lim_{eps->0+} M_Xi(z + eps v).  The test is
exact: with A = sign(det B) adj(B) and d = |det B|, z is inside B[0,1)^s iff
0 <= (A z)_i < d for all i; A has small integer entries and every input the
oracle sees is an FP32 value minus an integer, so A z is computed without
rounding in FP64.  Only the recurrence weights t carry rounding error.

Memoisation: for a batch of points Z the recursion is a DAG over
(direction subset, accumulated integer shift); each node is evaluated once,
vectorised over all points of the batch.
"""

from fractions import Fraction
from itertools import combinations

import numpy as np


# ---------------------------------------------------------------- exact helpers
def _frac_matrix(M):
    return [[Fraction(int(v)) for v in row] for row in M]


def _frac_det(M):
    """Exact determinant by Gaussian elimination over the rationals."""
    A = [row[:] for row in _frac_matrix(M)] if not isinstance(M[0][0], Fraction) else [row[:] for row in M]
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


def _frac_rank(M):
    A = _frac_matrix(M)
    rows, cols = len(A), len(A[0]) if A else 0
    r = 0
    for c in range(cols):
        p = next((i for i in range(r, rows) if A[i][c] != 0), None)
        if p is None:
            continue
        A[r], A[p] = A[p], A[r]
        for i in range(rows):
            if i != r and A[i][c] != 0:
                f = A[i][c] / A[r][c]
                for k in range(c, cols):
                    A[i][k] -= f * A[r][k]
        r += 1
        if r == rows:
            break
    return r


def _frac_solve(A, B):
    """Solve A X = B exactly (A square, invertible); B is a list of columns."""
    n = len(A)
    aug = [list(map(Fraction, A[i])) + [Fraction(b[i]) for b in B] for i in range(n)]
    m = len(B)
    for c in range(n):
        p = next(r for r in range(c, n) if aug[r][c] != 0)
        aug[c], aug[p] = aug[p], aug[c]
        piv = aug[c][c]
        aug[c] = [v / piv for v in aug[c]]
        for r in range(n):
            if r != c and aug[r][c] != 0:
                f = aug[r][c]
                aug[r] = [a - f * b for a, b in zip(aug[r], aug[c])]
    return [[aug[i][n + j] for i in range(n)] for j in range(m)]  # columns


def _int_adjugate(B):
    """Integer adjugate adj(B) (so that B adj(B) = det(B) I)."""
    s = len(B)
    adj = [[0] * s for _ in range(s)]
    for i in range(s):
        for j in range(s):
            minor = [[B[r][c] for c in range(s) if c != j] for r in range(s) if r != i]
            cof = int(_frac_det(minor)) if s > 1 else 1
            adj[j][i] = (-1) ** (i + j) * cof
    return adj


# ---------------------------------------------------------------- the oracle
class _LazyMap(dict):
    """dict that fills a missing key with make(key)."""

    def __init__(self, make):
        super().__init__()
        self._make = make

    def __missing__(self, key):
        val = self._make(key)
        self[key] = val
        return val


class BoxSplineOracle:
    """M_Xi for an integer s x n direction matrix Xi (columns are directions)."""

    def __init__(self, Xi):
        X = np.asarray(Xi, dtype=np.int64)
        if X.ndim != 2:
            raise ValueError("Xi must be a 2-D s x n matrix")
        s, n = X.shape
        if n < s or _frac_rank(X.tolist()) < s:
            raise ValueError("Xi must have n >= s columns and rank s")
        self.Xi, self.s, self.n = X, s, n
        self.dirs = [tuple(int(v) for v in X[:, j]) for j in range(n)]
        self.full = (1 << n) - 1
        # one fixed generic perturbation direction (exact binary fractions)
        self.v = np.array([2.0 ** (-10 * a) for a in range(s)])
        self._v_frac = [Fraction(1, 2 ** (10 * a)) for a in range(s)]

        self.spanning = _LazyMap(self._is_spanning)
        self.pinv = _LazyMap(self._make_pinv)      # mask -> float (k x s) least-norm right inverse
        self.pinv_frac = {}                         # mask -> exact version (lazily)
        self.base = _LazyMap(self._make_base)      # mask -> (A int s x s, d int, tie_lo, tie_hi)
        # gradient coefficients: e_a = sum_j g[j, a] xi_j using only removable j
        removable = [j for j in range(n) if self.spanning[self.full & ~(1 << j)]]
        self.removable = removable
        Xr = X[:, removable].astype(float)
        if removable and np.linalg.matrix_rank(Xr) == s:
            self.grad_coef = Xr.T @ np.linalg.inv(Xr @ Xr.T)   # (len(removable), s)
        else:
            self.grad_coef = None

    def _is_spanning(self, mask):
        cols = self.cols(mask)
        return len(cols) >= self.s and _frac_rank(self.Xi[:, cols].tolist()) == self.s

    def _make_pinv(self, mask):
        Xf = self.Xi[:, self.cols(mask)].astype(float)
        return Xf.T @ np.linalg.inv(Xf @ Xf.T)

    def _make_base(self, mask):
        Bm = self.Xi[:, self.cols(mask)].tolist()
        det = int(_frac_det(Bm))
        adj = np.array(_int_adjugate(Bm), dtype=np.int64)
        A = adj * (1 if det > 0 else -1)
        Av = A.astype(float) @ self.v          # exact: powers of two
        return (A, abs(det), Av > 0, Av < 0)

    def cols(self, mask):
        return [j for j in range(self.n) if (mask >> j) & 1]

    # ------------------------------------------------------------ FP64 batch
    def _node(self, Z, mask, shift, memo):
        key = (mask, shift)
        hit = memo.get(key)
        if hit is not None:
            return hit
        z = Z - np.asarray(shift, dtype=float)
        cols = self.cols(mask)
        k = len(cols)
        if k == self.s:
            A, d, tie_lo, tie_hi = self.base[mask]
            num = z @ A.T.astype(float)
            ok = ((num > 0) | ((num == 0) & tie_lo)) & ((num < d) | ((num == d) & tie_hi))
            res = np.where(ok.all(axis=1), 1.0 / d, 0.0)
        else:
            t = z @ self.pinv[mask].T                 # (P, k): Xi_mask t = z
            res = np.zeros(len(Z))
            for idx, j in enumerate(cols):
                sub = mask & ~(1 << j)
                if not self.spanning[sub]:
                    continue
                a = self._node(Z, sub, shift, memo)
                b = self._node(Z, sub, tuple(u + v for u, v in zip(shift, self.dirs[j])), memo)
                tj = t[:, idx]
                res += tj * a + (1.0 - tj) * b
            res /= (k - self.s)
        memo[key] = res
        return res

    def eval(self, Z, want_grad=False):
        """M_Xi at the rows of Z (P x s, float64).  Returns values (P,) and,
        if requested, the gradient (P, s)."""
        Z = np.ascontiguousarray(Z, dtype=float).reshape(-1, self.s)
        memo = {}
        zero = (0,) * self.s
        val = self._node(Z, self.full, zero, memo)
        if not want_grad:
            return val
        if self.grad_coef is None:
            raise ValueError("gradient needs the removable directions to span")
        grad = np.zeros((len(Z), self.s))
        for r, j in enumerate(self.removable):
            sub = self.full & ~(1 << j)
            dj = self._node(Z, sub, zero, memo) - self._node(Z, sub, self.dirs[j], memo)
            grad += dj[:, None] * self.grad_coef[r][None, :]
        return val, grad

    # ------------------------------------------------------------ exact mode
    def _pinv_exact(self, mask):
        P = self.pinv_frac.get(mask)
        if P is None:
            Xm = [[Fraction(int(v)) for v in row] for row in self.Xi[:, self.cols(mask)]]
            k = len(Xm[0])
            G = [[sum(Xm[a][c] * Xm[b][c] for c in range(k)) for b in range(self.s)] for a in range(self.s)]
            # P = Xm^T G^{-1}; columns of G^{-1} solve G y = e_b
            Ginv_cols = _frac_solve(G, [[Fraction(int(a == b)) for a in range(self.s)] for b in range(self.s)])
            Ginv = [[Ginv_cols[b][a] for b in range(self.s)] for a in range(self.s)]
            P = [[sum(Xm[a][c] * Ginv[a][b] for a in range(self.s)) for b in range(self.s)] for c in range(k)]
            self.pinv_frac[mask] = P
        return P

    def eval_exact(self, z):
        """M_Xi(z) exactly for one rational point z (sequence of Fractions/ints)."""
        z = [Fraction(v) for v in z]
        memo = {}

        def node(mask, shift):
            key = (mask, shift)
            if key in memo:
                return memo[key]
            w = [a - b for a, b in zip(z, shift)]
            cols = self.cols(mask)
            k = len(cols)
            if k == self.s:
                A, d, tie_lo, tie_hi = self.base[mask]
                ok = True
                for i in range(self.s):
                    num = sum(int(A[i, c]) * w[c] for c in range(self.s))
                    lo_ok = num > 0 or (num == 0 and bool(tie_lo[i]))
                    hi_ok = num < d or (num == d and bool(tie_hi[i]))
                    if not (lo_ok and hi_ok):
                        ok = False
                        break
                res = Fraction(1, d) if ok else Fraction(0)
            else:
                P = self._pinv_exact(mask)
                res = Fraction(0)
                for idx, j in enumerate(cols):
                    sub = mask & ~(1 << j)
                    if not self.spanning[sub]:
                        continue
                    tj = sum(P[idx][b] * w[b] for b in range(self.s))
                    a = node(sub, shift)
                    b = node(sub, tuple(u + v for u, v in zip(shift, self.dirs[j])))
                    res += tj * a + (1 - tj) * b
                res /= (k - self.s)
            memo[key] = res
            return res

        return node(self.full, (0,) * self.s)


def facet_normals(Xi):
    """Integer normals of the hyperplanes spanned by (s-1)-subsets of Xi
    (primitive, first nonzero entry positive).  These are the facet normals
    of the zonotope that supports M_Xi (Sec. 3, support of a box spline)."""
    X = np.asarray(Xi, dtype=np.int64)
    s, n = X.shape
    out = set()
    for cols in combinations(range(n), s - 1):
        sub = X[:, list(cols)]
        if s > 1 and _frac_rank(sub.tolist()) < s - 1:
            continue
        # generalized cross product: nu_a = (-1)^a det(sub without row a)
        nu = []
        for a in range(s):
            minor = [list(sub[r]) for r in range(s) if r != a]
            nu.append((-1) ** a * int(_frac_det(minor)) if s > 1 else 1)
        g = 0
        for v in nu:
            g = np.gcd(g, abs(v))
        nu = [v // g for v in nu]
        first = next(v for v in nu if v != 0)
        if first < 0:
            nu = [-v for v in nu]
        out.add(tuple(nu))
    return sorted(out)
