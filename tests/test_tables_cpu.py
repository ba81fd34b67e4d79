"""The committed generated tables against the oracle, on the CPU.

The tables come from the exact symbolic form of the paper's convolution
definition; the oracle from the de Boor--Hoellig recurrence.  The slow
interpreter executes the fast scheme (fold, sub-region, renamed stencil,
polynomial) in FP64 exactly as the kernels do.
"""

import hashlib
import os

import numpy as np
import pytest

from oracle import ConvolutionSumOracle, VoronoiSumOracle
from paper_2102_08514_amd.gen.interp import FloatTables, eval_fp64
from paper_2102_08514_amd.gen.specs import SPECS
from paper_2102_08514_amd.gen.tables import GENERATED, load
from workloads import configs as W

NAMES = {"c1": "bcc_linear", "c2": "cc_zp", "c3": "bcc_quartic", "c4": "fcc_6dir", "c5": "d4s_8dir", "d4": "d4_8dir",
         "cc_tp2": "cc_tp2", "cc_tp3": "cc_tp3", "cc_tp4": "cc_tp4", "cc_linear_rd": "cc_linear_rd",
         "bcc_quintic_rd": "bcc_quintic_rd", "vor_bcc1": "bcc_voronoi1", "vor_fcc1": "fcc_voronoi1",
         "vor_cc_bcc1": "cc_bcc_voronoi1", "vor_cc_fcc1": "cc_fcc_voronoi1", "vor_fcc2": "fcc_voronoi2",
         "vor_cc_fcc2": "cc_fcc_voronoi2"}


def oracle_for(cfg):
    if cfg.voronoi:
        # the box-spline form (pinned equal to the overlap-volume definition
        # for V_1 in test_voronoi_oracle_cpu.py) evaluates batches much faster
        return VoronoiSumOracle(cfg.L, cfg.Lv, cfg.voronoi[1], W=cfg.voronoi_gen, sigma=W.VORONOI_SIGMA,
                                method="boxsum")
    return ConvolutionSumOracle(cfg.L, cfg.Xi)


@pytest.mark.parametrize("cfg_name", list(NAMES))
def test_tables_match_oracle(cfg_name):
    cfg = W.get(cfg_name)
    t = load(NAMES[cfg_name])
    ft = FloatTables(t)
    s = cfg.s
    dims = (9,) * s
    rng = np.random.default_rng(11)
    coeffs = [rng.uniform(-1, 1, tuple(reversed(dims))) for _ in range(cfg.M)]
    ext = cfg.D * (dims[0] - 1) + 1
    # fewer points where the oracle is slow (12 directions, sums of up to 121 box splines)
    n = 150 if s == 4 else (40 if cfg.voronoi and cfg.voronoi[1] > 1 else
                            150 if cfg_name in ("cc_tp4", "vor_cc_bcc1") else 300 if cfg.voronoi else 600)
    X = rng.uniform(-1.5, ext + 0.5, (n, s)).astype(np.float32).astype(np.float64)
    X[:20] = np.floor(X[:20]) + rng.integers(0, 2, (20, s)) * 0.5   # sites, half-integers
    o = oracle_for(cfg)
    want = o.eval(coeffs, X)
    got = eval_fp64(ft, coeffs, X)
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("cfg_name", list(NAMES))
def test_table_facts(cfg_name):
    """Counts the paper prints: Table 1 lookups; the FCC 6-direction spline
    needs several non-equivalent sub-regions (Sec. 4.3); Q <= 9 planes for
    3-D box splines (Sec. 4.2)."""
    cfg = W.get(cfg_name)
    t = load(NAMES[cfg_name])
    per_query = cfg.M * sum(t.lookups_per_coset()) / t.K
    assert per_query == cfg.lookups
    if cfg_name == "c4":
        assert t.K > 1
    if cfg.s == 3:
        assert t.K >= 1 and len(t.planes) <= 9
    # the stored record is the one the header was emitted from
    blob = open(os.path.join(GENERATED, f"{t.name}.json")).read()
    head = open(os.path.join(GENERATED, f"{t.name}.inc")).readline()
    assert hashlib.sha256(blob.encode()).hexdigest()[:16] in head
    # lattice and spline are the configuration's
    _, L, what = SPECS[t.name]
    assert np.array_equal(np.array(L), cfg.L)
    if cfg.voronoi:
        assert np.array_equal(np.array(what.Lv), cfg.Lv) and what.n == cfg.voronoi[1]
        assert sorted(map(tuple, what.W)) == sorted(map(tuple, cfg.voronoi_gen))
    else:
        assert np.array_equal(np.array(what), cfg.Xi)


@pytest.mark.parametrize("name", ["bcc_voronoi1"])
def test_sigma_table_separates_the_subregions(name):
    """Sec. 4.2: r is smaller than 2^Q and sigma(q mod r) names every
    sub-region from its own code."""
    t = load(name)
    assert t.sigma is not None and t.sigma["r"] < 1 << len(t.planes)
    res = [c % t.sigma["r"] for c in t.sigma["feasible"]]
    assert len(set(res)) == len(res) == t.K
    for c in t.sigma["feasible"]:
        assert t.sigma["table"][c % t.sigma["r"]] == t.orbit_table[c]


@pytest.mark.parametrize("cfg_name", ["c1", "c2", "c4", "vor_bcc1", "vor_fcc1"])
def test_exact_partition_of_unity(cfg_name):
    from fractions import Fraction
    from paper_2102_08514_amd.gen.interp import eval_exact
    t = load(NAMES[cfg_name])
    rng = np.random.default_rng(3)
    for _ in range(10):
        x = [Fraction(int(v), 997) for v in rng.integers(0, 997 * 10, t.s)]
        assert eval_exact(t, lambda k, i: 1, x) == 1
        lin = eval_exact(t, lambda k, i: t.D * i[0] + t.lat.shifts[k][0], x)
        assert lin == x[0]
