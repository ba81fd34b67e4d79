"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's own recurrence: each compares it with an
independent statement -- a closed form, the paper's defining convolution
integral, a moment identity, printed counts, exact rational arithmetic,
finite differences or the adjoint identity.
"""

import os
from fractions import Fraction
from itertools import combinations, permutations, product

import numpy as np
import pytest

from oracle import BoxSplineOracle, ConvolutionSumOracle
from oracle.boxspline import facet_normals
from workloads import configs as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(12345)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


# ------------------------------------------------------------------ closed forms
def bspline(k, t):
    """Cardinal B-spline of order k (support [0, k]) by the explicit truncated
    power formula (1/(k-1)!) sum_j (-1)^j C(k, j) (t - j)_+^(k-1)."""
    from math import comb, factorial
    t = np.asarray(t, dtype=float)
    out = np.zeros_like(t)
    for j in range(k + 1):
        out += (-1) ** j * comb(k, j) * np.where(t > j, (t - j), 0.0) ** (k - 1)
    return out / factorial(k - 1)


def test_univariate_bsplines():
    # s = 1, Xi = [1, 1, ..., 1] (k ones) is the cardinal B-spline of order k
    for k in (2, 3, 4, 5):
        bs = BoxSplineOracle(np.ones((1, k), dtype=int))
        t = f32(RNG.uniform(-0.5, k + 0.5, 400))
        np.testing.assert_allclose(bs.eval(t[:, None]), bspline(k, t), atol=1e-13)


@pytest.mark.parametrize("reps", [2, 3, 4])
def test_tensor_product_bsplines(reps):
    # Xi = [I3]^{:reps} (Table 1 CC Voronoi 1/2/3) is the tensor-product B-spline
    bs = BoxSplineOracle(np.hstack([np.eye(3, dtype=int)] * reps))
    Z = f32(RNG.uniform(-0.3, reps + 0.3, (300, 3)))
    want = np.prod(bspline(reps, Z), axis=1)
    np.testing.assert_allclose(bs.eval(Z), want, atol=1e-13)


def test_trilinear_interpolation():
    # centred Xi = [I3 | -I3]: phi(y) = prod(1 - |y_i|)_+, f = trilinear interpolation
    o = ConvolutionSumOracle(np.eye(3, dtype=int), np.hstack([np.eye(3, dtype=int), -np.eye(3, dtype=int)]))
    Y = f32(RNG.uniform(-1.2, 1.2, (300, 3)))
    np.testing.assert_allclose(o.phi(Y), np.prod(np.clip(1 - np.abs(Y), 0, None), axis=1), atol=1e-14)
    c = RNG.uniform(-1, 1, (6, 6, 6))
    X = f32(RNG.uniform(1, 4, (200, 3)))
    f = o.eval([c], X)
    i = np.floor(X).astype(int)
    t = X - i
    want = np.zeros(len(X))
    for d in product((0, 1), repeat=3):
        w = np.prod([t[:, a] if d[a] else 1 - t[:, a] for a in range(3)], axis=0)
        want += w * c[i[:, 2] + d[2], i[:, 1] + d[1], i[:, 0] + d[0]]
    np.testing.assert_allclose(f, want, atol=1e-13)


def slice_length_box_spline(Xi, z):
    """n = s + 1 box spline as the length of the slice {t in [0,1):
    B^{-1}(z - t xi) in [0,1)^s} / |det B|, B = first s columns (the paper's
    convolution definition, evaluated by exact interval intersection)."""
    Xi = [[Fraction(int(v)) for v in row] for row in Xi]
    s = len(Xi)
    B = [row[:s] for row in Xi]
    xi = [row[s] for row in Xi]
    Bf = np.array(B, dtype=float)
    inv = np.linalg.inv(Bf)
    det = abs(round(np.linalg.det(Bf)))
    Binv = [[Fraction(round(inv[i, j] * det), det) for j in range(s)] for i in range(s)]
    a = [sum(Binv[i][j] * Fraction(z[j]) for j in range(s)) for i in range(s)]
    b = [-sum(Binv[i][j] * xi[j] for j in range(s)) for i in range(s)]
    lo, hi = Fraction(0), Fraction(1)
    for ai, bi in zip(a, b):
        if bi == 0:
            if not (0 <= ai < 1):
                return Fraction(0)
            continue
        t0, t1 = sorted(((0 - ai) / bi, (1 - ai) / bi))
        lo, hi = max(lo, t0), min(hi, t1)
    return max(Fraction(0), hi - lo) / det


def test_slice_length_form_n_equals_s_plus_1():
    for Xi in (W.XI_BCC_LINEAR, np.array([[1, 0, 1], [0, 1, 1]]), np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 1]])):
        bs = BoxSplineOracle(Xi)
        s = Xi.shape[0]
        Z = f32(RNG.uniform(-2.2, 2.2, (120, s)))
        got = bs.eval(Z)
        want = np.array([float(slice_length_box_spline(Xi, z)) for z in Z])
        np.testing.assert_allclose(got, want, atol=1e-14)


def test_c1_is_barycentric_interpolation():
    cfg = W.get("c1")
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    # interpolation at the sites: phi(0) = 1, phi(other sites) = 0
    sites = [np.array(p) for p in product(range(-4, 5), repeat=3) if len({v % 2 for v in p}) == 1]
    vals = o.phi(np.array(sites, dtype=float))
    assert vals[[i for i, p in enumerate(sites) if not p.any()][0]] == 1.0
    assert np.count_nonzero(vals) == 1
    # barycentric weights of the 4 nonzero sites
    X = f32(RNG.uniform(-1, 1, (300, 3)))
    S = np.array(sites, dtype=float)
    for x in X:
        w = o.phi(x[None, :] - S)
        nz = np.nonzero(w)[0]
        assert len(nz) == 4
        A = np.vstack([S[nz].T, np.ones(4)])
        lam = np.linalg.solve(A, np.append(x, 1.0))
        np.testing.assert_allclose(w[nz], lam, atol=1e-13)


# ------------------------------------------------------- the defining convolution
def _mesh_breakpoints(Xi_sub, x, xi):
    """Parameters t in (0,1) where x - t xi crosses a mesh plane of M_{Xi_sub}:
    planes nu.z = nu.(sum of a subset of Xi_sub), nu normal to an (s-1)-subset."""
    X = np.asarray(Xi_sub)
    n = X.shape[1]
    sums = {tuple(X[:, list(c)].sum(axis=1)) for r in range(n + 1) for c in combinations(range(n), r)}
    ts = {0.0, 1.0}
    for nu in facet_normals(X):
        nu = np.array(nu, dtype=float)
        den = nu @ xi
        if den == 0:
            continue
        for sm in sums:
            t = (nu @ x - nu @ np.array(sm, dtype=float)) / den
            if 0 < t < 1:
                ts.add(t)
    return sorted(ts)


@pytest.mark.parametrize("name", ["c1", "c2", "c4", "c5", "d4", "cc_linear_rd", "bcc_quintic_rd"])
def test_convolution_definition(name):
    """M_Xi(x) = int_0^1 M_{Xi\\xi}(x - t xi) dt (Sec. 3, sign corrected),
    integrated exactly: the integrand is a polynomial of degree n-1-s between
    consecutive mesh crossings, so Gauss-Legendre with enough nodes is exact."""
    Xi = W.get(name).Xi
    s, n = Xi.shape
    full = BoxSplineOracle(Xi)
    gx, gw = np.polynomial.legendre.leggauss(4)
    for j in (0, n - 1):
        sub = np.delete(Xi, j, axis=1)
        subo = BoxSplineOracle(sub)
        xi = Xi[:, j].astype(float)
        X = RNG.uniform(Xi.clip(max=0).sum(1), Xi.clip(min=0).sum(1), (25, s))
        want = full.eval(X)
        got = []
        for x in X:
            ts = _mesh_breakpoints(sub, x, xi)
            acc = 0.0
            for a, b in zip(ts[:-1], ts[1:]):
                tt = 0.5 * (a + b) + 0.5 * (b - a) * gx
                acc += 0.5 * (b - a) * np.dot(gw, subo.eval(x[None, :] - tt[:, None] * xi[None, :]))
            got.append(acc)
        np.testing.assert_allclose(got, want, atol=1e-12)


# ------------------------------------------------------------- moment identities
def _centred_moment(Xi, alpha):
    """E[(Xi v)^alpha] for v uniform on [-1/2, 1/2]^n (exact)."""
    Xi = np.asarray(Xi)
    n = Xi.shape[1]
    axes = [a for a, k in enumerate(alpha) for _ in range(k)]
    mom = {0: Fraction(1), 1: Fraction(0), 2: Fraction(1, 12), 3: Fraction(0), 4: Fraction(1, 80)}
    total = Fraction(0)
    for js in product(range(n), repeat=len(axes)):
        coef = 1
        for a, j in zip(axes, js):
            coef *= int(Xi[a, j])
        if coef == 0:
            continue
        e = Fraction(1)
        for j in set(js):
            e *= mom[js.count(j)]
        total += coef * e
    return total


def _order(Xi):
    """Approximation order m: fewest directions whose removal leaves a non-spanning set."""
    Xi = np.asarray(Xi)
    s, n = Xi.shape
    for r in range(1, n + 1):
        for c in combinations(range(n), r):
            if np.linalg.matrix_rank(np.delete(Xi, list(c), axis=1)) < s:
                return r
    return n


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5", "d4", "cc_linear_rd", "bcc_quintic_rd"])
def test_moment_identities(name):
    """For |alpha| < m (Strang--Fix), sum_{n in L} (x-n)^alpha phi(x-n) equals
    int y^alpha phi(y) dy / ... = E[(Xi v)^alpha], v ~ U[-1/2,1/2]^n, at every x."""
    cfg = W.get(name)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    s = cfg.s
    m = _order(cfg.Xi)
    # orders printed in Table 1; the D4 spline is fourth order (Sec. 5.2)
    assert m == {"c1": 2, "c2": 4, "c3": 4, "c4": 3, "c5": 4, "d4": 4, "cc_linear_rd": 2, "bcc_quintic_rd": 4}[name]
    dims = (12,) * s
    X = f32(RNG.uniform(4.5, 2 * 12 - 6.5 if cfg.D == 2 else 12 - 4.5, (8 if s == 4 else 30, s)))
    qi, ki, flat, Wd = o._candidates(X, dims)
    ph = o.phi(Wd)
    for deg in range(m):
        for alpha in product(range(deg + 1), repeat=s):
            if sum(alpha) != deg:
                continue
            mono = np.prod([Wd[:, a] ** alpha[a] for a in range(s)], axis=0)
            got = np.bincount(qi, weights=mono * ph, minlength=len(X))
            want = float(_centred_moment(cfg.Xi, alpha))
            np.testing.assert_allclose(got, want, atol=1e-11, err_msg=str(alpha))


# ------------------------------------------------------------ structure pins
def _read_table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_lookups.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, lat, xi, cnt = line.split()
                rows.append((name, lat, xi, int(cnt)))
    return rows


def _xi_of(tag):
    if tag.startswith("I3:"):
        return np.hstack([np.eye(3, dtype=int)] * int(tag[3:]))
    return {"bcc_diag": W.BCC_DIAG, "I3|bcc_diag": W.XI_ZP, "2I3|bcc_diag": W.XI_BCC_QUARTIC,
            "bcc_diag:2": np.hstack([W.BCC_DIAG] * 2), "fcc6": W.XI_FCC6,
            "xi_d4": np.array([[1, 1, 1, 1, -1, -1, -1, -1], [1, 1, -1, -1, 1, 1, -1, -1],
                               [1, -1, 1, -1, 1, -1, 1, -1], [1, 1, 1, 1, 1, 1, 1, 1]])}[tag]


@pytest.mark.parametrize("row", _read_table1(), ids=lambda r: r[0])
def test_lookup_counts(row):
    name, lat, xi, want = row
    L = {"CC": W.L_CC, "BCC": W.L_BCC, "FCC": W.L_FCC, "D4": W.L_D4, "D4S": W.L_D4S}[lat]
    Xi = _xi_of(xi)
    o = ConvolutionSumOracle(L, Xi)
    s = Xi.shape[0]
    dims = (24,) * s
    X = f32(RNG.uniform(12, 16, (3 if s == 4 else 20, s)))
    assert set(o.nonzero_count(X, dims).tolist()) == {want}


def _group(s, even):
    for perm in permutations(range(s)):
        for sg in product((1, -1), repeat=s):
            if even and np.prod(sg) < 0:
                continue
            T = np.zeros((s, s))
            for i, j in enumerate(perm):
                T[i, j] = sg[i]
            yield T


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
def test_symmetry_and_support(name):
    cfg = W.get(name)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    s = cfg.s
    Y = f32(RNG.uniform(-3.2, 3.2, (60 if s == 4 else 200, s)))
    base = o.phi(Y)
    Ts = list(_group(s, even=(s == 4)))
    for T in Ts[:: (7 if s == 4 else 3)]:
        np.testing.assert_allclose(o.phi(Y @ T.T), base, atol=1e-14)
    # support = open zonotope: positive strictly inside, zero outside
    lhs = np.abs(Y @ o.normals.T)
    inside = np.all(lhs < o.bounds - 1e-9, axis=1)
    outside = np.any(lhs > o.bounds + 1e-9, axis=1)
    assert np.all(base[inside] > 0) and np.all(base[outside] == 0)


def test_exact_mode_matches_fp64():
    for name in ("c1", "c2", "c4"):
        cfg = W.get(name)
        o = ConvolutionSumOracle(cfg.L, cfg.Xi)
        Y = f32(RNG.uniform(-2, 2, (6, cfg.s)))
        got = o.phi(Y)
        for y, g in zip(Y, got):
            assert abs(float(o.phi_exact(y)) - g) < 1e-13
        # points exactly on mesh planes: exact and FP64 agree (consistent ties)
        for y in ([0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [1.0, 0.0, 0.0], [0.25, 0.25, 0.5]):
            assert abs(float(o.phi_exact(y)) - o.phi(np.array([y]))[0]) < 1e-13


def test_ties_are_consistent_on_mesh_planes():
    # queries exactly on lattice sites and mesh planes still give PoU = 1
    cfg = W.get("c2")
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    X = np.array([[5, 5, 5], [5.5, 5.5, 5.5], [5.5, 5, 5], [5.25, 5.25, 5.5], [6, 5.5, 5.0]])
    f = o.eval([np.ones((12, 12, 12))], X)
    np.testing.assert_allclose(f, 1.0, atol=1e-14)


# ----------------------------------------------------------- derivatives, adjoint
@pytest.mark.parametrize("name", ["c2", "c3", "c4", "c5"])
def test_gradient_matches_finite_differences(name):
    cfg = W.get(name)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    s = cfg.s
    dims = (10,) * s
    rng = np.random.default_rng(7)
    c = [rng.uniform(-1, 1, tuple(reversed(dims))) for _ in range(cfg.M)]
    hi = cfg.D * 9 - o.half.max() - 0.5
    X = rng.uniform(o.half.max() + cfg.D, hi, (5 if s == 4 else 12, s))
    f, g = o.eval(c, X, want_grad=True)
    h = 1e-5
    for a in range(s):
        e = np.zeros(s)
        e[a] = h
        fd = (o.eval(c, X + e) - o.eval(c, X - e)) / (2 * h)
        np.testing.assert_allclose(g[:, a], fd, atol=1e-7)


def test_linear_data_has_constant_gradient():
    cfg = W.get("c3")
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    dims = (10,) * 3
    a = np.array([0.3, -1.1, 0.7])
    c = []
    for l in o.lat.shifts:
        idx = np.indices(tuple(reversed(dims))).astype(float)
        site = np.stack([2 * idx[2 - k] + l[k] for k in range(3)], axis=-1)
        c.append(site @ a + 0.25)
    X = RNG.uniform(5, 13, (20, 3))
    f, g = o.eval(c, X, want_grad=True)
    np.testing.assert_allclose(f, X @ a + 0.25, atol=1e-12)
    np.testing.assert_allclose(g, np.broadcast_to(a, g.shape), atol=1e-12)


@pytest.mark.parametrize("name", ["c1", "c4"])
def test_adjoint_identity(name):
    cfg = W.get(name)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    dims = (7,) * cfg.s
    rng = np.random.default_rng(3)
    c = [rng.uniform(-1, 1, tuple(reversed(dims))) for _ in range(cfg.M)]
    X = rng.uniform(-1, 2 * 7, (400, cfg.s))          # includes partially outside queries
    g = rng.normal(size=len(X))
    lhs = np.dot(o.eval(c, X), g)
    r = o.adjoint(X, g, dims)
    rhs = sum(np.sum(ci * ri) for ci, ri in zip(c, r))
    assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs))


@pytest.mark.parametrize("name", ["c4", "c5"])
def test_adjoint_at_sites_is_a_column_of_the_forward(name):
    """adjoint_at enumerates queries per site (column-wise); its value at
    site m must equal <A e_m, g>: the forward sum with the single unit
    coefficient c_m = 1 (found row-wise, per query), dotted with g.  It must
    also agree with the full adjoint at every sampled site."""
    cfg = W.get(name)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    dims = (6,) * cfg.s
    rng = np.random.default_rng(17)
    X = rng.uniform(-1, 2 * 6, (300, cfg.s))
    g = rng.normal(size=len(X))
    full = o.adjoint(X, g, dims)
    sites = [(int(rng.integers(cfg.M)), tuple(int(v) for v in rng.integers(0, 6, cfg.s))) for _ in range(12)]
    sites += [(0, (0,) * cfg.s), (cfg.M - 1, (5,) * cfg.s)]
    got = o.adjoint_at(X, g, sites)
    for (k, idx), v in zip(sites, got):
        e = [np.zeros(tuple(reversed(dims))) for _ in range(cfg.M)]
        e[k][tuple(reversed(idx))] = 1.0
        want = float(np.dot(o.eval(e, X), g))
        assert abs(v - want) <= 1e-12 * max(1.0, abs(want))
        assert abs(v - full[k][tuple(reversed(idx))]) <= 1e-12 * max(1.0, abs(v))
