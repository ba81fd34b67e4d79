"""Offline analysis of a (lattice, box spline) pair into evaluation tables.

Steps (Sec. 4 of the paper, specialised to a symmetry fold):

1. Cartesian coset decomposition D Z^s + l_k of the lattice (Sec. 4.1,
   GL = D diagonal).  Every coset uses the same tables.
2. Region of evaluation: the cell [0, D)^s of the coset's own array; a
   query x on coset k is shifted by rho(x) = D floor((x - l_k)/D) into it
   (Sec. 4.1, the map rho), u = x - l_k - rho - (D/2)1 is the offset from the
   cell centre p.
3. Symmetry (Sec. 4.3): phi is invariant under a signed-permutation group
   G (all signed permutations B_s when T Xi = Xi up to column order and
   signs for every T in B_s, else the even-sign subgroup D_s).  Every T in G
   maps the cell's half-integer site grid onto itself, so the per-coset sum
   at u equals the one at u' = T u with renamed coefficients pi(n) = T^{-1}
   (n - 1/2) + 1/2, a rigid renaming as the paper reports.  A query is
   folded into the fundamental chamber F (h >= u'_1 >= ... >= u'_s >= 0 for
   B_s; h >= u'_1 >= ... >= u'_{s-1} >= |u'_s| for D_s), which replaces the
   general sigma lookup table by a sorting network.
4. Splitting planes (Sec. 4.2): the mesh planes of all site-shifted copies
   of phi that cross the interior of F.  They cut F into K sub-regions; no
   two are related by G (F is a fundamental domain), so K is the number of
   non-equivalent polynomial sets (the paper's K, Sec. 4.3).
5. For each sub-region: the stencil (sites whose support contains it; its
   size summed over cosets is the Table 1 lookup count) and, per site, the
   exact polynomial phi(u' - D(j - 1/2 1)) in u' (Sec. 4.1, psi_j).

Everything is exact (rationals).  The polynomial pieces come from
`BoxSplinePP`, the symbolic form of the paper's convolution definition.
"""

from fractions import Fraction
from itertools import combinations, permutations, product

import numpy as np

from .lattice import Lattice, primitive_normal
from .poly import Poly, monomials
from .phi import BoxPhi
from .pp import DegeneratePoint


# ------------------------------------------------------------------ symmetry
def _signed_perms(s, even):
    for perm in permutations(range(s)):
        for sg in product((1, -1), repeat=s):
            if even and np.prod(sg) < 0:
                continue
            yield perm, sg


def _invariant(Xi_cols, perm, sg):
    """T Xi equals Xi up to column order and column signs (T: (Tv)_r = sg_r v_perm[r])."""
    def canon(v):
        v = tuple(v)
        neg = tuple(-a for a in v)
        return max(v, neg)
    want = sorted(canon(c) for c in Xi_cols)
    got = sorted(canon([sg[r] * c[perm[r]] for r in range(len(c))]) for c in Xi_cols)
    return want == got


def symmetry_fold(Xi_cols, s):
    if all(_invariant(Xi_cols, p, g) for p, g in _signed_perms(s, False)):
        return "B"
    if all(_invariant(Xi_cols, p, g) for p, g in _signed_perms(s, True)):
        return "D"
    raise ValueError("box spline lacks the signed-permutation symmetry the fold needs")


def chamber_constraints(s, fold, h):
    """F as rows (a, b) meaning a.u + b >= 0."""
    rows = [([-1] + [0] * (s - 1), h)]                  # h - u_1 >= 0
    for r in range(s - 1):
        a = [0] * s
        a[r], a[r + 1] = 1, -1
        if fold == "D" and r == s - 2:
            rows.append((a, 0))                         # u_{s-1} - u_s >= 0
            b = [0] * s
            b[r], b[r + 1] = 1, 1
            rows.append((b, 0))                         # u_{s-1} + u_s >= 0
        else:
            rows.append((a, 0))
    if fold == "B":
        a = [0] * s
        a[s - 1] = 1
        rows.append((a, 0))                             # u_s >= 0
    return rows


def chamber_vertices(s, fold, h):
    vs = []
    for k in range(s + 1):
        vs.append(tuple([h] * k + [0] * (s - k)))
    if fold == "D":
        vs.append(tuple([h] * (s - 1) + [-h]))
    return vs


def plane_ties(t):
    """Per splitting plane of tables t: True when a point exactly on the plane
    takes its >= side (the side of the chamber's generic tie point)."""
    from .select import tie_sides
    h = Fraction(t.D, 2)
    return tie_sides(t.planes, chamber_constraints(t.s, t.fold, h), chamber_vertices(t.s, t.fold, h))


# ------------------------------------------------------------------ analysis
class SplineTables:
    def __init__(self, name, L, Xi=None, seed=1, phi=None):
        """Tables for phi on the lattice L: the box spline M_Xi when `phi` is
        None, else the given basis function object (see `phi.py`)."""
        self.name = name
        self.lat = Lattice(L)
        s = self.lat.s
        if phi is None:
            phi = BoxPhi(Xi, self.lat.det)
            for c in phi.cols:
                if not self.lat.contains(c):
                    raise ValueError("direction not on the lattice: partition of unity fails")
        self.phi = phi
        self.s = s
        self.voronoi = None
        if phi.kind == "voronoi":
            self.voronoi = {"Lv": phi.vlat.L, "W": [list(w) for w in phi.W], "sigma": phi.sigma, "n": phi.n,
                            "terms": phi.n_box}
        dirs = phi.mesh_directions()
        self.Xi_rows = [[d[a] for d in dirs] for a in range(s)]
        self.n = len(dirs)
        self.cols = [tuple(d) for d in dirs]
        self.D = self.lat.D
        self.h = Fraction(self.D, 2)
        self.degree = phi.degree
        self.order = phi.order
        self.fold = symmetry_fold(phi.symmetry_generators(), s)
        self._rng = np.random.default_rng(seed)
        self.normals = phi.normals()
        self.planes = self._splitting_planes()
        self.cells = self._cells()
        self.K = len(self.cells)
        self.orbit_table = self._orbit_table()
        self.sigma = self._sigma()
        self.orbits = [self._orbit(c) for c in self.cells]

    def _splitting_planes(self):
        """Mesh planes nu.u' = off crossing the interior of F.  Site j's copy of
        phi has breakpoints at nu.(u - D(j - 1/2) + c0) = nu.(sum of a subset)."""
        s, D = self.s, self.D
        verts = chamber_vertices(s, self.fold, self.h)
        planes = []
        for nu in self.normals:
            vals = [sum(Fraction(a) * b for a, b in zip(nu, v)) for v in verts]
            lo, hi = min(vals), max(vals)
            # nu.u = b + D nu.(j - 1/2 1), j integer, b a breakpoint offset of phi
            base = {b - self.h * sum(nu) for b in self.phi.offsets(nu)}
            offs = set()
            for off in base:
                # nu is primitive, so nu.(D Z^s) = D Z
                k = (lo - off) // D
                t = off + k * D
                while t < hi:
                    if t > lo:
                        offs.add(t)
                    t += D
            for off in sorted(offs):
                planes.append((nu, off))
        return planes

    # ----------------------------------------------------------------- cells
    def _cells(self):
        """Sub-regions of F cut by the splitting planes: feasible sign vectors,
        each with an exact generic interior point."""
        from scipy.optimize import linprog
        s = self.s
        F = chamber_constraints(s, self.fold, self.h)
        planes = self.planes
        Q = len(planes)
        cells = []

        def lp(signs):
            # maximise d: sign*(nu.u - off) >= d, F rows >= d
            A, b = [], []
            for (nu, off), sg in zip(planes, signs):
                A.append([-sg * float(v) for v in nu] + [1.0])
                b.append(-sg * float(off))
            for a, c in F:
                A.append([-float(v) for v in a] + [1.0])
                b.append(float(c))
            res = linprog(c=[0.0] * s + [-1.0], A_ub=A, b_ub=b, bounds=[(None, None)] * s + [(None, 1.0)],
                          method="highs")
            if res.status != 0 or -res.fun <= 1e-9:
                return None
            return res.x[:s]

        def dfs(prefix):
            if len(prefix) == Q:
                x = lp(prefix)
                if x is not None:
                    cells.append((tuple(prefix), self._exact_point(x, prefix)))
                return
            for sg in (1, -1):
                p2 = prefix + [sg]
                sub_planes = planes[:len(p2)]
                # partial feasibility
                ok = _partial_lp(sub_planes, p2, F, s)
                if ok:
                    dfs(p2)

        dfs([])
        return cells

    def _inside(self, u, signs):
        for (nu, off), sg in zip(self.planes, signs):
            if sg * (sum(Fraction(a) * b for a, b in zip(nu, u)) - off) <= 0:
                return False
        for a, c in chamber_constraints(self.s, self.fold, self.h):
            if sum(Fraction(x) * y for x, y in zip(a, u)) + c <= 0:
                return False
        return True

    def _exact_point(self, x, signs):
        for scale in (10 ** 6, 10 ** 7, 10 ** 8):
            u = tuple(Fraction(float(v)).limit_denominator(scale) for v in x)
            if self._inside(u, signs):
                return u
        raise RuntimeError("could not find an exact interior point")

    def _generic(self, u, signs):
        """Perturb u by a small random rational keeping it inside its cell."""
        for _ in range(100):
            d = [Fraction(int(self._rng.integers(-10 ** 6, 10 ** 6)), 99991 * 10 ** 4) for _ in range(self.s)]
            v = tuple(a + b for a, b in zip(u, d))
            if self._inside(v, signs):
                return v
        raise RuntimeError("could not perturb inside the cell")

    # ------------------------------------------------------------- orbits
    def _orbit_table(self):
        Q = len(self.planes)
        table = []
        sig = {tuple(1 if b == 1 else 0 for b in c[0]): k for k, c in enumerate(self.cells)}
        for code in range(1 << Q):
            bits = tuple((code >> i) & 1 for i in range(Q))
            if bits in sig:
                table.append(sig[bits])
            else:
                # infeasible pattern (reachable only through rounding next to an
                # intersection of planes): take a feasible neighbour
                best = min(sig, key=lambda b: (sum(x != y for x, y in zip(b, bits)), sig[b]))
                table.append(sig[best])
        return table

    def feasible_codes(self):
        return {sum(1 << i for i, b in enumerate(c[0]) if b == 1): k for k, c in enumerate(self.cells)}

    def _sigma(self):
        """Sec. 4.2 table sigma(q mod r) when the full 2^Q table no longer fits
        one 64-bit word of 4-bit entries (Q > 4); None otherwise."""
        from .select import sigma_table
        Q = len(self.planes)
        if 4 * (1 << Q) <= 64:
            return None
        r, table = sigma_table(self.feasible_codes(), Q)
        return {"r": r, "table": table, "feasible": sorted(self.feasible_codes())}

    def _orbit(self, cell):
        signs, u0 = cell
        s, D = self.s, self.D
        R = [int((self.phi.reach[a] + self.h) / D) + 2 for a in range(s)]
        cand = list(product(*[range(-R[a], R[a] + 2) for a in range(s)]))
        for attempt in range(20):
            try:
                u = self._generic(u0, signs)
                stencil, polys = [], []
                for j in cand:
                    # site j of the cell sits at D (j - 1/2 1) from the cell centre
                    shift = tuple(-D * (Fraction(j[a]) - Fraction(1, 2)) for a in range(s))
                    P = self.phi.piece(tuple(u[a] + shift[a] for a in range(s)))
                    if P.is_zero():
                        continue
                    stencil.append(tuple(j))
                    polys.append(P.shift(shift))
                return {"stencil": stencil, "polys": polys, "point": u}
            except DegeneratePoint:
                continue
        raise RuntimeError("no generic point found")

    # --------------------------------------------------------------- checks
    def verify(self, points=40):
        """Exact checks of the tables through the interpreter of the fast
        scheme, at random rational points: partition of unity and linear
        precision of the whole lattice sum (Sec. 4.1 requirement on phi), and
        the lookup count per query."""
        from .interp import eval_exact
        s, D = self.s, self.D
        for orb in self.orbits:
            for P in orb["polys"]:
                assert P.degree() <= self.degree
        rng = np.random.default_rng(99)
        shifts = self.lat.shifts
        for _ in range(points):
            x = [Fraction(int(v), 7919) for v in rng.integers(0, 7919 * 8 * D, s)]
            one = eval_exact(self, lambda k, i: 1, x)
            assert one == 1, "partition of unity fails"
            for a in range(s):
                lin = eval_exact(self, lambda k, i, a=a: D * i[a] + shifts[k][a], x)
                assert lin == x[a], "linear precision fails"
        return True

    def lookups_per_coset(self):
        return [len(o["stencil"]) for o in self.orbits]

    def monomials(self):
        return monomials(self.s, self.degree)

    def coefficient_matrix(self, k):
        """A[j][m]: coefficient of monomial m in site j's polynomial (sub-region k)."""
        mons = self.monomials()
        idx = {e: i for i, e in enumerate(mons)}
        A = [[Fraction(0)] * len(mons) for _ in self.orbits[k]["stencil"]]
        for r, P in enumerate(self.orbits[k]["polys"]):
            for e, c in P.t.items():
                A[r][idx[e]] = c
        return A


def _partial_lp(planes, signs, F, s):
    from scipy.optimize import linprog
    A, b = [], []
    for (nu, off), sg in zip(planes, signs):
        A.append([-sg * float(v) for v in nu] + [1.0])
        b.append(-sg * float(off))
    for a, c in F:
        A.append([-float(v) for v in a] + [1.0])
        b.append(float(c))
    res = linprog(c=[0.0] * s + [-1.0], A_ub=A, b_ub=b, bounds=[(None, None)] * s + [(None, 1.0)], method="highs")
    return res.status == 0 and -res.fun > 1e-9
