"""Pins of the Voronoi-spline oracle (Sec. 3, Voronoi splines; Table 1 Voronoi rows).

The oracle has two evaluations of V_1 (the overlap volume of the cell with
its translate, straight from the definition V_1 = chi * chi, and the paper's
route through a sum of box splines); each is checked against the other and
both against facts that do not depend on either: the geometry of the cells,
partition of unity, linear precision, the lookup counts the paper prints,
lattice symmetry, values at lattice sites and the slope at the origin given
by the cell's projected area.
"""

import os
from itertools import permutations, product

import numpy as np
import pytest

from oracle.voronoi import (BoxSumPhi, OverlapPhi, VoronoiSumOracle, _polytope_faces, in_voronoi,
                            voronoi_halfspaces, zonotope_tiles)
from workloads import configs as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_voronoi_lookups.txt")
RNG = np.random.default_rng(2102)
V1 = ["vor_bcc1", "vor_fcc1", "vor_cc_bcc1", "vor_cc_fcc1"]


def _gen(lat):
    from fractions import Fraction
    return [tuple(Fraction(v, W.VORONOI_SIGMA) for v in w) for w in W.VORONOI_GEN[lat]]


@pytest.mark.parametrize("lat", ["BCC", "FCC"])
def test_generators_span_the_voronoi_cell(lat):
    """The zonotope sum_j [-1/2, 1/2] g_j has exactly the vertices of the
    Voronoi cell computed from the lattice's half-spaces."""
    A, b = voronoi_halfspaces(W.LATTICES[lat])
    _, verts = _polytope_faces(A, b)
    G = np.array([[float(v) for v in g] for g in _gen(lat)])
    pts = np.array([0.5 * np.array(sg) @ G for sg in product((-1, 1), repeat=len(G))])
    # extreme points of the zonotope: those not inside the hull of the others
    # are the cell vertices; every cell vertex must be a zonotope point and
    # every zonotope point inside the cell
    assert np.all(in_voronoi(pts, A, b + 1e-12))
    for v in verts:
        assert np.min(np.abs(pts - v).sum(axis=1)) < 1e-12
    assert len(verts) == {"BCC": 24, "FCC": 14}[lat]     # truncated octahedron / rhombic dodecahedron


@pytest.mark.parametrize("lat,ntiles", [("BCC", 16), ("FCC", 4)])
def test_tiling_partitions_the_cell(lat, ntiles):
    """One parallelepiped per basis; they cover the cell exactly once (the
    paper: the BCC V_0 is a sum of 16 box splines)."""
    from fractions import Fraction
    G = _gen(lat)
    tiles = zonotope_tiles(G, [Fraction((j + 1) ** 3 + 5 * j, 7) for j in range(len(G))])
    assert len(tiles) == ntiles
    det = abs(int(round(np.linalg.det(np.asarray(W.LATTICES[lat], dtype=float)))))
    assert sum(v for _, _, v in tiles) == det
    A, b = voronoi_halfspaces(W.LATTICES[lat])
    centre = np.array([float(sum(g[a] for g in G)) / 2 for a in range(3)])
    X = RNG.uniform(-1.6, 1.6, (4000, 3))
    count = np.zeros(len(X), dtype=int)
    for B, t, _ in tiles:
        M = np.array([[float(G[j][a]) for j in B] for a in range(3)])
        u = np.linalg.solve(M, (X + centre - np.array([float(v) for v in t])).T).T
        count += np.all((u >= 0) & (u < 1), axis=1)
    assert np.array_equal(count, in_voronoi(X, A, b).astype(int))


def test_product_counts_match_the_paper():
    """BCC: V_0 has 16 terms; V_1, V_2, V_3 expand into 136, 816 and 3876
    box-spline products (Sec. 3)."""
    from math import comb
    assert [comb(16 + k - 1, k) for k in (2, 3, 4)] == [136, 816, 3876]
    b = BoxSumPhi(W.L_BCC, W.L_BCC, W.VORONOI_GEN["BCC"], W.VORONOI_SIGMA, 1)
    assert b.n_tiles == 16 and b.n_products == 136


@pytest.mark.parametrize("name", V1)
def test_overlap_volume_matches_box_spline_sum(name):
    cfg = W.get(name)
    op = OverlapPhi(cfg.L, cfg.Lv)
    bs = BoxSumPhi(cfg.L, cfg.Lv, cfg.voronoi_gen, W.VORONOI_SIGMA, 1)
    Wq = RNG.uniform(-2.2, 2.2, (300, 3))
    a, ga = op(Wq, want_grad=True)
    b, gb = bs(Wq, want_grad=True)
    assert np.max(np.abs(a - b)) < 1e-13
    assert np.max(np.abs(ga - gb)) < 1e-12
    assert np.count_nonzero(a) > 30


@pytest.mark.parametrize("name", V1 + ["vor_fcc2"])
def test_partition_of_unity_and_linear_precision(name):
    cfg = W.get(name)
    o = VoronoiSumOracle(cfg.L, cfg.Lv, cfg.voronoi[1], W=cfg.voronoi_gen, sigma=W.VORONOI_SIGMA)
    dims = (12, 12, 12)
    D = cfg.D
    X = RNG.uniform(D * 5, D * 6 + 1, (4 if cfg.voronoi[1] == 2 else 12 if D == 1 else 30, 3))
    X[:6] = np.floor(2 * X[:6]) / 2           # lattice sites and half-integers: planes of V and V + w coincide
    ones = [np.ones(dims) for _ in range(cfg.M)]
    assert np.max(np.abs(o.eval(ones, X) - 1)) < 1e-12
    for a in range(3):
        lin = []
        for l in cfg.shifts:
            idx = np.indices(dims)[2 - a]           # array axis of coordinate a (x fastest)
            lin.append(D * idx + l[a])
        assert np.max(np.abs(o.eval(lin, X) - X[:, a])) < 1e-11


def _read_golden():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, lat, cell, n, want = line.split()
                rows.append((name, lat, cell, int(n), int(want)))
    return rows


@pytest.mark.parametrize("row", _read_golden(), ids=lambda r: r[0])
def test_voronoi_lookup_counts(row):
    """Sites with nonzero weight = sites m with x - m in the open support (n+1) V
    (V_n is positive inside its support: a convolution of positive functions)."""
    name, lat, cell, n, want = row
    L = W.LATTICES[lat]
    A, b = voronoi_halfspaces(W.LATTICES[cell])
    from oracle.lattice import CosetLattice
    cl = CosetLattice(L)
    X = RNG.uniform(20, 21, (40, 3))
    D = cl.D
    offs = np.array(list(product(range(-8, 9), repeat=3)))
    for x in X:
        cnt = 0
        for l in cl.shifts:
            base = np.floor((x - l) / D)
            sites = D * (base + offs) + l
            w = x - sites
            cnt += int(np.count_nonzero(np.all(w @ A.T < (n + 1) * b, axis=1)))
        assert cnt == want


def _oh():
    for perm in permutations(range(3)):
        for sg in product((1, -1), repeat=3):
            T = np.zeros((3, 3))
            for i, j in enumerate(perm):
                T[i, j] = sg[i]
            yield T


@pytest.mark.parametrize("name", ["vor_bcc1", "vor_fcc1"])
def test_symmetry_sites_and_slope(name):
    cfg = W.get(name)
    op = OverlapPhi(cfg.L, cfg.Lv)
    Wq = RNG.uniform(-2, 2, (20, 3))
    base = op(Wq)
    for T in _oh():
        assert np.max(np.abs(op(Wq @ T.T) - base)) < 1e-13
    det, detv = abs(round(np.linalg.det(cfg.L))), abs(round(np.linalg.det(cfg.Lv)))
    assert abs(op(np.zeros((1, 3)))[0] - det / detv) < 1e-13
    # other sites of L_v: the cells meet in a face at most
    A, _ = voronoi_halfspaces(cfg.Lv, reach=1)
    assert np.max(np.abs(op(A))) < 1e-13
    # slope along e_1 at the origin: -(area of the cell's projection along e_1) det / det_v^2;
    # truncated octahedron |y|,|z| <= 1, |y|+|z| <= 3/2: 3.5; rhombic dodecahedron |y|+|z| <= 1: 2
    area = {"BCC": 3.5, "FCC": 2.0}[cfg.voronoi[0]]
    _, g = op(np.array([[1e-6, 0.0, 0.0]]), want_grad=True)
    assert abs(g[0, 0] + area * det / detv ** 2) < 1e-5


@pytest.mark.parametrize("name", ["vor_bcc1", "vor_cc_fcc1"])
def test_gradient_matches_finite_differences(name):
    cfg = W.get(name)
    op = OverlapPhi(cfg.L, cfg.Lv)
    Wq = RNG.uniform(-1.8, 1.8, (60, 3))
    _, g = op(Wq, want_grad=True)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (op(Wq + e) - op(Wq - e)) / (2 * h)
        assert np.max(np.abs(fd - g[:, a])) < 1e-6
