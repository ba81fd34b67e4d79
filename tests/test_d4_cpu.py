"""The paper's 4-D experiment (Sec. 5.2): the 8-direction box spline on the D4
lattice with its quasi-interpolation prefilter, pinned on the CPU oracle.

- The prefilter (7/3 at the origin, -1/18 at the 24 sites at distance sqrt 2)
  turns sampling into a scheme that reproduces every cubic exactly, which is
  what fourth-order approximation (error / 16 per halving of h) rests on.
  Plain sampling does not reproduce cubics.
- The spline touches 240 lattice sites at a generic point (Sec. 5.2).
"""

import itertools

import numpy as np

from oracle import ConvolutionSumOracle
from workloads import configs as W
from workloads.d4 import D4_ROOTS, PREFILTER_CENTRE, PREFILTER_ROOT, prefilter_samples

CFG = W.get("d4")
RNG = np.random.default_rng(2024)


def _cubic():
    mons = [a for a in itertools.product(range(4), repeat=4) if sum(a) <= 3]
    coef = RNG.normal(size=len(mons))

    def p(P):
        P = np.asarray(P, dtype=np.float64)
        return sum(cf * np.prod(P ** np.array(a), axis=-1) for cf, a in zip(coef, mons))
    return p


def _coset_arrays(values_at, dims):
    out = []
    for k in range(CFG.M):
        idx = np.indices(tuple(reversed(dims)), dtype=np.float64)
        P = np.stack([2 * idx[3 - a] + CFG.shifts[k][a] for a in range(4)], axis=-1)
        out.append(values_at(P))
    return out


def test_prefilter_weights():
    # 24 roots of D4 (norm sqrt 2) and weights summing to one
    assert len(D4_ROOTS) == 24
    assert all(sum(v * v for v in m) == 2 and sum(m) % 2 == 0 for m in D4_ROOTS)
    assert abs(PREFILTER_CENTRE + 24 * PREFILTER_ROOT - 1.0) < 1e-15


def test_prefiltered_sampling_reproduces_cubics():
    p = _cubic()
    o = ConvolutionSumOracle(CFG.L, CFG.Xi)
    dims = (8, 8, 8, 8)
    X = RNG.uniform(5.0, 10.0, size=(16, 4))
    f = o.eval(_coset_arrays(lambda P: prefilter_samples(p, P), dims), X)
    scale = np.abs(p(X)).max()
    assert np.abs(f - p(X)).max() <= 1e-12 * scale
    # plain sampling is only second order: cubics are not reproduced
    f2 = o.eval(_coset_arrays(p, dims), X)
    assert np.abs(f2 - p(X)).max() > 1e-3 * scale


def test_lookups_240():
    o = ConvolutionSumOracle(CFG.L, CFG.Xi)
    X = RNG.uniform(5.0, 10.0, size=(8, 4))
    counts = o.nonzero_count(X, (8, 8, 8, 8))
    assert np.all(np.asarray(counts) == 240)
