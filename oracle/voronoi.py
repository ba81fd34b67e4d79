"""Voronoi splines (oracle; test infrastructure only).

Definition followed (Sec. 3, Voronoi splines): with V the Voronoi cell of a
lattice L_v (the points at least as close to the origin as to any other site
of L_v), chi = 1/|det L_v| on V and 0 elsewhere, and

    V_0 = chi,    V_n = chi * V_{n-1}    (convolution).

The basis used on a lattice L that contains L_v is phi = |det L| V_n: the
Voronoi cells tile space under L_v, so sum_{m in L_v} chi(x - m) = 1/|det L_v|,
and summing over the |det L_v| / |det L| cosets of L_v in L gives
sum_{m in L} phi(x - m) = 1 (partition of unity, the requirement of Sec. 4.1).
The Voronoi cell is centrally symmetric, so phi is centred at the origin.

Two independent evaluations:

* `OverlapPhi` (n = 1 only): V_1(w) = int chi(y) chi(w - y) dy
  = vol(V n (V + w)) / |det L_v|^2, since V = -V.  The volume of the convex
  polytope V n (V + w) is computed from its vertices (every triple of bounding
  planes, solved and kept when feasible) face by face: each face polygon is
  ordered around its centroid, and the volume is the sum over faces of
  height x area / s.  Its gradient is the rate at which the translated cell
  V + w gains volume inside V: grad vol = sum over faces F of V + w of
  area(F n V) times F's outward unit normal.
* `BoxSumPhi` (any n): the paper's route.  V is a zonotope sum_j [-1/2,1/2] g_j
  for the lattices here; a tiling of the zonotope into parallelepipeds
  t_B + G_B [0,1)^s (one per basis B of the generators, read off the lower
  faces of the zonotope lifted by generic heights, see `zonotope_tiles`)
  writes chi as a sum of constant box splines, |det G_B| M_{G_B}(. - t_B)
  / |det L_v|, and the multinomial theorem expands chi^{*(n+1)} into shifted
  box splines whose directions are the union of the factors' (the
  convolution of box splines is the box spline of the joined directions).
  Each is evaluated by the de Boor--Hoellig recurrence of `boxspline.py`.

The two agree for n = 1 (a test pins one against the other), and `BoxSumPhi`
carries the higher orders.
"""

from collections import Counter
from fractions import Fraction
from itertools import combinations, combinations_with_replacement, product
from math import factorial

import numpy as np

from .boxspline import BoxSplineOracle, _frac_det
from .lattice import CosetLattice


# ------------------------------------------------------------------ the cell
def voronoi_halfspaces(Lv, reach=2):
    """(A, b) with V = {x : A x <= b}: one row n, |n|^2 / 2 per nonzero site n
    of L_v with integer coordinates k in [-reach, reach]^s of the basis;
    redundant rows are kept (they do not change the polytope)."""
    L = np.asarray(Lv, dtype=np.int64)
    s = L.shape[0]
    rows = []
    for k in product(range(-reach, reach + 1), repeat=s):
        n = L @ np.array(k, dtype=np.int64)
        if np.any(n):
            rows.append(tuple(int(v) for v in n))
    rows = sorted(set(rows))
    A = np.array(rows, dtype=float)
    b = 0.5 * np.sum(A * A, axis=1)
    return A, b


def in_voronoi(X, A, b):
    X = np.asarray(X, dtype=float).reshape(-1, A.shape[1])
    return np.all(X @ A.T <= b, axis=1)


def _polytope_faces(A, b, tol=1e-10):
    """Vertices of {x : A x <= b} (3-D, bounded) grouped per bounding plane:
    returns [(row index into A, ordered vertex array, unit normal)] for the
    faces of positive area, and the vertices."""
    # coincident half-spaces (V and V + w share a bounding plane when n.w = 0)
    # would contribute their face twice: keep the first of each
    # (the tolerances here and below are far under the spacing of FP32 inputs)
    An = A / np.linalg.norm(A, axis=1)[:, None]
    bn = b / np.linalg.norm(A, axis=1)
    sc = 1.0 + np.abs(bn).max()
    keep = []
    for i in range(A.shape[0]):
        if not any(np.max(np.abs(An[i] - An[j])) < 1e-12 and abs(bn[i] - bn[j]) < 1e-9 * sc for j in keep):
            keep.append(i)
    keep = np.array(keep)
    A, b = A[keep], b[keep]
    m = A.shape[0]
    idx = np.array(list(combinations(range(m), 3)), dtype=np.int64)
    M = A[idx]                                   # (T, 3, 3)
    det = np.linalg.det(M)
    ok = np.abs(det) > 1e-12
    idx, M = idx[ok], M[ok]
    rhs = b[idx]
    P = np.linalg.solve(M, rhs[..., None])[..., 0]
    scale = 1.0 + np.abs(b).max()
    feas = np.all(P @ A.T <= b + tol * scale, axis=1)
    P = P[feas]
    if len(P) == 0:
        return [], P
    # merge repeated vertices (points where more than three planes meet)
    key = np.round(P / (1e-9 * scale)).astype(np.int64)
    _, first = np.unique(key, axis=0, return_index=True)
    V = P[np.sort(first)]
    faces = []
    on = np.abs(V @ A.T - b) <= 1e-9 * scale      # (nv, m)
    for i in range(m):
        F = V[on[:, i]]
        if len(F) < 3:
            continue
        n = A[i] / np.linalg.norm(A[i])
        c = F.mean(axis=0)
        e1 = F[0] - c
        if np.linalg.norm(e1) < 1e-14:
            e1 = F[1] - c
        e1 = e1 / np.linalg.norm(e1)
        e2 = np.cross(n, e1)
        ang = np.arctan2((F - c) @ e2, (F - c) @ e1)
        faces.append((int(keep[i]), F[np.argsort(ang)], n))
    return faces, V


def _area(poly, n):
    """Area of a planar convex polygon (ordered vertices) with unit normal n."""
    tot = np.zeros(3)
    for a, c in zip(poly, np.roll(poly, -1, axis=0)):
        tot += np.cross(a, c)
    return abs(float(tot @ n)) / 2.0


class OverlapPhi:
    """phi(w) = (|det L| / |det L_v|^2) vol(V n (V + w)) for 3-D lattices."""

    def __init__(self, L, Lv):
        self.lat = CosetLattice(L)
        self.vlat = CosetLattice(Lv)
        if self.lat.s != 3:
            raise ValueError("the overlap evaluation is written for 3-D cells")
        self.A, self.b = voronoi_halfspaces(Lv)
        faces, verts = _polytope_faces(self.A, self.b)
        self.cell_vertices = verts
        self.scale = float(self.lat.det) / float(self.vlat.det) ** 2
        # keep only the facet-defining rows of V
        self.A = np.array([self.A[i] for i, _, _ in faces])
        self.b = np.array([self.b[i] for i, _, _ in faces])
        self.half = np.abs(verts).max(axis=0) * 2.0           # support bbox half widths

    def _one(self, w, want_grad):
        A, b = self.A, self.b
        # V + w = {x : A x <= b + A w}; w/2 is interior iff w lies in 2 V (open)
        if not np.all(A @ (0.5 * w) < b):
            return 0.0, np.zeros(3)
        AA = np.vstack([A, A])
        bb = np.concatenate([b, b + A @ w])
        faces, _ = _polytope_faces(AA, bb)
        c = 0.5 * w
        vol = 0.0
        grad = np.zeros(3)
        nA = len(A)
        for i, poly, n in faces:
            ar = _area(poly, n)
            h = (bb[i] - AA[i] @ c) / np.linalg.norm(AA[i])
            vol += h * ar / 3.0
            if want_grad and i >= nA:
                grad += ar * n          # a face of V + w: its outward normal
        return vol, grad

    def __call__(self, W, want_grad=False):
        W = np.asarray(W, dtype=float).reshape(-1, 3)
        val = np.zeros(len(W))
        grad = np.zeros((len(W), 3))
        for r, w in enumerate(W):
            v, g = self._one(w, want_grad)
            val[r], grad[r] = v, g
        val *= self.scale
        grad *= self.scale
        return (val, grad) if want_grad else val


# ------------------------------------------------------------------ box-spline sum
def zonotope_tiles(G, heights):
    """Tiles (basis B, corner t_B) of the zonotope sum_j [0, 1] g_j: for every
    basis B, the normal n_B of the lifted vectors (g_j, h_j), j in B, with a
    positive last entry; the lower face it supports is t_B + G_B [0,1]^s with
    t_B the sum of the lifted generators on which n_B is negative."""
    s = len(G[0])
    m = len(G)
    tiles = []
    for B in combinations(range(m), s):
        GB = [[G[j][a] for j in B] for a in range(s)]
        if _frac_det(GB) == 0:
            continue
        lifted = [list(G[j]) + [heights[j]] for j in B]
        nB = []
        for col in range(s + 1):
            minor = [[row[c] for c in range(s + 1) if c != col] for row in lifted]
            nB.append((-1) ** col * _frac_det(minor))
        if nB[s] < 0:
            nB = [-v for v in nB]
        t = [Fraction(0)] * s
        for j in range(m):
            if j in B:
                continue
            val = sum(nB[a] * G[j][a] for a in range(s)) + nB[s] * heights[j]
            if val == 0:
                raise ValueError("lifting heights not generic")
            if val < 0:
                t = [x + y for x, y in zip(t, G[j])]
        tiles.append((B, tuple(t), abs(_frac_det(GB))))
    return tiles


class BoxSumPhi:
    """phi = |det L| V_n through the box-spline expansion.  Generators are
    given as integer vectors W with G = W / sigma."""

    def __init__(self, L, Lv, W, sigma, n):
        self.lat = CosetLattice(L)
        self.vlat = CosetLattice(Lv)
        s = self.lat.s
        self.s = s
        G = [tuple(Fraction(int(v), sigma) for v in w) for w in W]
        heights = [Fraction((j + 1) ** 3 + 5 * j, 7) for j in range(len(G))]
        self.tiles = zonotope_tiles(G, heights)
        centre = [sum(g[a] for g in G) / 2 for a in range(s)]
        k = n + 1
        acc = {}
        for combo in combinations_with_replacement(range(len(self.tiles)), k):
            mult = factorial(k)
            for v in Counter(combo).values():
                mult //= factorial(v)
            coef = Fraction(mult)
            cols, shift = [], [k * c for c in centre]
            for t in combo:
                B, tB, vol = self.tiles[t]
                coef *= vol
                cols.extend(tuple(int(W[j][a]) for a in range(s)) for j in B)
                shift = [x - y for x, y in zip(shift, tB)]
            key = (tuple(sorted(cols)), tuple(shift))
            acc[key] = acc.get(key, Fraction(0)) + coef
        # V_n = sum coef / |det L_v|^k M_{G cols}(w + shift); M_G(z) = sigma^s M_W(sigma z)
        norm = Fraction(self.lat.det * sigma ** s, self.vlat.det ** k)
        self.terms = []
        self._bs = {}
        for (cols, shift), coef in sorted(acc.items()):
            if cols not in self._bs:
                self._bs[cols] = BoxSplineOracle(np.array(cols, dtype=np.int64).T)
            self.terms.append((cols, np.array([float(sigma * v) for v in shift]), float(coef * norm)))
        self.sigma = sigma
        self.n_tiles = len(self.tiles)
        self.n_products = sum(1 for _ in combinations_with_replacement(range(len(self.tiles)), k))
        wmax = np.abs(np.array(W, dtype=float)).sum(axis=0) / (2.0 * sigma)
        self.half = k * wmax

    def __call__(self, Wq, want_grad=False):
        Wq = np.asarray(Wq, dtype=float).reshape(-1, self.s)
        val = np.zeros(len(Wq))
        grad = np.zeros((len(Wq), self.s))
        for cols, shift, coef in self.terms:
            Z = self.sigma * Wq + shift
            r = self._bs[cols].eval(Z, want_grad=want_grad)
            if want_grad:
                val += coef * r[0]
                grad += coef * self.sigma * r[1]
            else:
                val += coef * r
        return (val, grad) if want_grad else val


# ------------------------------------------------------------------ the lattice sum
class VoronoiSumOracle:
    """f(x) = sum_m c_m phi(x - m) over every site m of L (per coset, zero
    outside the stored arrays), phi = |det L| V_n of the Voronoi cell of L_v.
    Same interface as `ConvolutionSumOracle` (eval, adjoint, adjoint_at,
    nonzero_count)."""

    def __init__(self, L, Lv, n=1, W=None, sigma=None, method=None):
        self.lat = CosetLattice(L)
        self.s = self.lat.s
        method = method or ("overlap" if n == 1 and self.s == 3 else "boxsum")
        if method == "overlap":
            if n != 1:
                raise ValueError("the overlap form is V_1 only")
            self.phi_fn = OverlapPhi(L, Lv)
        else:
            self.phi_fn = BoxSumPhi(L, Lv, W, sigma, n)
        self.half = np.asarray(self.phi_fn.half, dtype=float)
        D = self.lat.D
        self.window = [int(np.ceil(2 * h / D)) + 2 for h in self.half]

    def phi(self, W, want_grad=False):
        return self.phi_fn(W, want_grad=want_grad)

    def _candidates(self, X, dims):
        X = np.asarray(X, dtype=float).reshape(-1, self.s)
        D = self.lat.D
        dims = tuple(int(d) for d in dims)
        offs = np.array(list(product(*[range(w) for w in self.window])), dtype=np.int64)
        qs, ks, flats, Ws = [], [], [], []
        for k, l in enumerate(self.lat.shifts):
            lo = np.floor((X - l - self.half) / D).astype(np.int64)
            I = lo[:, None, :] + offs[None, :, :]
            W = X[:, None, :] - (D * I + l)
            inside = np.all(np.abs(W) < self.half, axis=2)
            inb = np.all((I >= 0) & (I < np.array(dims)), axis=2)
            qi, ci = np.nonzero(inside & inb)
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

    def eval(self, coeffs, X, want_grad=False, chunk=2048):
        X = np.asarray(X, dtype=float).reshape(-1, self.s)
        if len(coeffs) != self.lat.M:
            raise ValueError("need one coefficient array per coset")
        dims = tuple(reversed(coeffs[0].shape))
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

    def adjoint(self, X, gout, dims, chunk=2048):
        X = np.asarray(X, dtype=float).reshape(-1, self.s)
        gout = np.asarray(gout, dtype=float).reshape(-1)
        dims = tuple(int(d) for d in dims)
        size = int(np.prod(dims))
        out = [np.zeros(size) for _ in range(self.lat.M)]
        for q0 in range(0, len(X), chunk):
            Xc = X[q0:q0 + chunk]
            qi, ki, flat, W = self._candidates(Xc, dims)
            contrib = gout[q0 + qi] * self.phi(W)
            for k in range(self.lat.M):
                sel = ki == k
                out[k] += np.bincount(flat[sel], weights=contrib[sel], minlength=size)
        return [o.reshape(tuple(reversed(dims))) for o in out]

    def nonzero_count(self, X, dims):
        qi, ki, flat, W = self._candidates(X, dims)
        ph = self.phi(W)
        return np.bincount(qi[ph > 0], minlength=len(np.asarray(X).reshape(-1, self.s)))
