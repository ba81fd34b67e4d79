"""The basis function phi of the lattice sum, as the table generator sees it.

phi(y) = |det L| F(y), centred at the origin, with F one of

* a box spline, F(y) = M_Xi(y + c0), c0 = 1/2 sum xi (Sec. 3);
* a Voronoi spline, F = V_n, the (n+1)-fold self-convolution of the
  normalised indicator chi of the Voronoi cell of a lattice L_v (Sec. 3,
  Voronoi splines).  Following the paper's route, chi is rewritten as a sum
  of constant box splines and the multinomial theorem expands chi^{*(n+1)}
  into a sum of shifted box splines, each the convolution of n+1 of them.

The Voronoi cells handled here are zonotopes Z(G) = sum_j [-1/2, 1/2] g_j
(true for the Cartesian, BCC and FCC lattices; `VoronoiPhi` checks it).  A
zonotope is tiled by one parallelepiped per basis B of its generators (a
fine zonotopal tiling, taken here from the lower faces of a generically
lifted zonotope), and the indicator of the parallelepiped s_B + G_B [0,1)^s
is |det G_B| M_{G_B}(. - s_B).  The number of tiles is the number of bases:
16 for the BCC Voronoi cell (truncated octahedron), 4 for the FCC one
(rhombic dodecahedron).  For BCC, the (n+1)-fold products then give 136
(V_1) and 816 (V_2) distinct box splines, the counts the paper quotes.

Generators are rational; they are handled as integer directions W = sigma G
with M_G(z) = sigma^s M_W(sigma z).

Every object exposes what the analysis needs: the dimension, the directions
whose (s-1)-subsets give the mesh normals, the breakpoint offsets of phi
along each normal, the polynomial piece of phi on the mesh cell holding a
generic point, the degree, the approximation order, and the generator set
whose symmetry the fold relies on.
"""

from collections import Counter
from fractions import Fraction
from itertools import combinations, combinations_with_replacement, product
from math import factorial

from .lattice import Lattice, int_det, int_rank, primitive_normal
from .poly import Poly
from .pp import BoxSplinePP, DegeneratePoint  # noqa: F401  (DegeneratePoint re-exported)


def _subset_sums(cols, s):
    sums = set()
    for r in range(len(cols) + 1):
        for sub in combinations(cols, r):
            sums.add(tuple(sum(c[a] for c in sub) for a in range(s)))
    return sums


def _normals(cols, s):
    out = set()
    for sub in combinations(cols, s - 1):
        nu = primitive_normal(list(sub), s)
        if nu is not None:
            out.add(nu)
    return out


def _dot(nu, v):
    return sum(Fraction(a) * b for a, b in zip(nu, v))


def _approx_order(cols, s):
    """Smallest number of directions whose removal leaves a non-spanning set."""
    n = len(cols)
    for r in range(1, n + 1):
        for rem in combinations(range(n), r):
            keep = [c for j, c in enumerate(cols) if j not in rem]
            if int_rank([[c[a] for c in keep] for a in range(s)] if keep else [[0]]) < s:
                return r
    return n


class BoxPhi:
    """phi(y) = |det L| M_Xi(y + c0)."""

    kind = "box"

    def __init__(self, Xi, det):
        Xi = [[int(v) for v in row] for row in Xi]
        self.Xi_rows = Xi
        self.s = s = len(Xi)
        self.cols = [tuple(Xi[a][j] for a in range(s)) for j in range(len(Xi[0]))]
        self.det = det
        self.c0 = tuple(Fraction(sum(c[a] for c in self.cols), 2) for a in range(s))
        self.degree = len(self.cols) - s
        self.order = _approx_order(self.cols, s)
        self.pp = BoxSplinePP(Xi)
        self._sums = _subset_sums(self.cols, s)
        # support bounding box of the centred spline
        self.reach = [Fraction(sum(abs(c[a]) for c in self.cols), 2) for a in range(s)]

    def symmetry_generators(self):
        return list(self.cols)

    def mesh_directions(self):
        return list(self.cols)

    def normals(self):
        return sorted(_normals(self.cols, self.s))

    def offsets(self, nu):
        """Offsets b with breakpoints of phi on nu.y = b."""
        return {_dot(nu, sm) - _dot(nu, self.c0) for sm in self._sums}

    def piece(self, y):
        """Polynomial (in y) equal to phi on the mesh cell of the generic point y."""
        q = tuple(Fraction(v) + c for v, c in zip(y, self.c0))
        return self.pp.piece(q).shift(self.c0).scale(self.det)


# ------------------------------------------------------------------ Voronoi
def voronoi_relevant(Lv):
    """Nonzero lattice vectors n of L_v with n.n <= 4 r^2 where r bounds the
    cell: enough half-spaces x.n <= n.n/2 to cut out the Voronoi cell."""
    s = Lv.s
    pts = []
    for k in product(range(-3, 4), repeat=s):
        v = tuple(sum(Lv.L[a][b] * k[b] for b in range(s)) for a in range(s))
        if any(v):
            pts.append(v)
    pts = sorted(set(pts), key=lambda v: sum(a * a for a in v))
    return pts


def _in_voronoi(x, rel):
    return all(2 * _dot(n, x) <= sum(a * a for a in n) for n in rel)


def zonotope_tiling(G, s, heights):
    """Tiles (basis B, shift s_B) of the zonotope sum_j [0,1] g_j: the lower
    facets of the zonotope of the lifted generators (g_j, heights_j).  For a
    basis B the facet normal n_B is orthogonal to the lifted g_j, j in B,
    with positive last coordinate; the tile is s_B + G_B [0,1)^s with s_B
    the sum of the generators on which n_B is negative."""
    m = len(G)
    tiles = []
    for B in combinations(range(m), s):
        M = [[G[j][a] for j in B] for a in range(s)]
        if int_det([[v * 4 for v in row] for row in M]) == 0:   # integer-scaled det test
            continue
        # normal in R^{s+1}: cofactors of the s x (s+1) matrix of lifted rows
        rows = [list(G[j]) + [heights[j]] for j in B]
        n = []
        for col in range(s + 1):
            minor = [[r[c] for c in range(s + 1) if c != col] for r in rows]
            n.append((-1) ** col * _det_frac(minor))
        if n[s] < 0:
            n = [-v for v in n]
        assert n[s] > 0
        shift = [Fraction(0)] * s
        for j in range(m):
            if j in B:
                continue
            val = sum(n[a] * G[j][a] for a in range(s)) + n[s] * heights[j]
            assert val != 0, "lifting heights are not generic"
            if val < 0:
                shift = [a + b for a, b in zip(shift, G[j])]
        tiles.append((B, tuple(shift)))
    return tiles


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


class VoronoiPhi:
    """phi(y) = |det L| V_n(y) for the Voronoi cell of L_v (L_v a sublattice of L)."""

    kind = "voronoi"

    def __init__(self, L, Lv, W, sigma, n):
        """W: integer generators with G = W / sigma spanning the Voronoi cell of L_v."""
        self.lat = Lattice(L)
        self.vlat = Lattice(Lv)
        self.s = s = self.lat.s
        self.n = n
        self.sigma = sigma
        self.W = [tuple(int(v) for v in w) for w in W]
        G = [tuple(Fraction(v, sigma) for v in w) for w in self.W]
        self.G = G
        self.det = self.lat.det
        # L_v must be a sublattice of L (partition of unity on L)
        for b in range(s):
            if not self.lat.contains([self.vlat.L[a][b] for a in range(s)]):
                raise ValueError("the Voronoi lattice is not a sublattice of L")
        # the zonotope Z(G) is the Voronoi cell: equal volume and every vertex inside
        tiles = zonotope_tiling(G, s, heights=[Fraction(3 ** j + 7 * j * j, 11) for j in range(len(G))])
        vols = [abs(_det_frac([[G[j][a] for j in B] for a in range(s)])) for B, _ in tiles]
        if sum(vols) != self.vlat.det:
            raise ValueError("generator zonotope volume differs from |det L_v|")
        rel = voronoi_relevant(self.vlat)
        for sg in product((-1, 1), repeat=len(G)):
            v = tuple(sum(Fraction(sg[j], 2) * G[j][a] for j in range(len(G))) for a in range(s))
            if not _in_voronoi(v, rel):
                raise ValueError("generator zonotope is not the Voronoi cell")
        self.tiles = tiles
        c = tuple(sum(g[a] for g in G) / 2 for a in range(s))   # centre of Z(G)
        # chi(y) = (1/|det L_v|) sum_B |det G_B| M_{G_B}(y + c - s_B); expand (n+1) factors
        k = n + 1
        terms = {}
        for combo in combinations_with_replacement(range(len(tiles)), k):
            cnt = Counter(combo)
            mult = factorial(k)
            for v in cnt.values():
                mult //= factorial(v)
            coef = Fraction(mult, self.vlat.det ** k)
            dirs = []
            arg = [k * ca for ca in c]
            for t in combo:
                B, sh = tiles[t]
                coef *= vols[t]
                dirs.extend(self.W[j] for j in B)
                arg = [a - b for a, b in zip(arg, sh)]
            key = (tuple(sorted(dirs)), tuple(arg))
            terms[key] = terms.get(key, Fraction(0)) + coef
        # phi = |det L| * V_n; M_G(z) = sigma^s M_W(sigma z)
        self.terms = [(dirs, arg, coef * self.det * sigma ** s) for (dirs, arg), coef in sorted(terms.items())]
        self.n_box = len(self.terms)
        self._pp = {}
        for dirs, _, _ in self.terms:
            if dirs not in self._pp:
                Xi = [[d[a] for d in dirs] for a in range(s)]
                self._pp[dirs] = BoxSplinePP(Xi)
        self._term_normals = {dirs: _normals(list(dirs), s) for dirs in self._pp}
        self._term_sums = {dirs: _subset_sums(list(dirs), s) for dirs in self._pp}
        self.degree = k * s - s
        self.order = k
        # reach: the support is (n+1) times the Voronoi cell
        self.reach = [k * sum(abs(g[a]) for g in G) / 2 for a in range(s)]
        # per-term support boxes in y: sigma (y + arg) in [0, sum |w|] per axis, loosely
        self._box = []
        for dirs, arg, _ in self.terms:
            lo = [Fraction(sum(min(d[a], 0) for d in dirs), sigma) - arg[a] for a in range(s)]
            hi = [Fraction(sum(max(d[a], 0) for d in dirs), sigma) - arg[a] for a in range(s)]
            self._box.append((lo, hi))

    def symmetry_generators(self):
        return list(self.W)

    def mesh_directions(self):
        return sorted(set(self.W))

    def normals(self):
        out = set()
        for v in self._term_normals.values():
            out |= v
        return sorted(out)

    def offsets(self, nu):
        # term t: breakpoints of M_W(sigma (y + arg)) on nu.(sigma (y + arg)) = nu.(subset sum)
        out = set()
        for dirs, arg, _ in self.terms:
            if nu not in self._term_normals[dirs]:
                continue
            na = _dot(nu, arg)
            for sm in self._term_sums[dirs]:
                out.add(Fraction(_dot(nu, sm), self.sigma) - na)
        return out

    def piece(self, y):
        y = tuple(Fraction(v) for v in y)
        s, sg = self.s, self.sigma
        res = Poly(s)
        for (dirs, arg, coef), (lo, hi) in zip(self.terms, self._box):
            if any(y[a] < lo[a] or y[a] > hi[a] for a in range(s)):
                continue                      # outside the term's support box
            q = tuple(sg * (y[a] + arg[a]) for a in range(s))
            P = self._pp[dirs].piece(q)
            if P.is_zero():
                continue
            # P(sigma (Y + arg)) as a polynomial in Y
            res = res + P.shift(tuple(sg * a for a in arg)).scale_vars(sg).scale(coef)
        return res
