"""Inputs of the D4 approximation study (Sec. 5.2): the quasi-interpolation
prefilter and the Gaussian test function.  Plain arithmetic on sample values;
none of the spline's arithmetic lives here."""

import itertools

import numpy as np

# the 24 D4 sites at distance sqrt 2 from the origin (+-e_i +- e_j)
D4_ROOTS = tuple(v for v in itertools.product((-1, 0, 1), repeat=4) if sum(t * t for t in v) == 2)
PREFILTER_CENTRE = 7.0 / 3.0
PREFILTER_ROOT = -1.0 / 18.0
GAUSS_SIGMA = 0.125


def prefilter_samples(f, P, h=1.0):
    """c_n = 7/3 f(h n) - 1/18 sum over the 24 roots m of f(h (n + m)), at the
    sites n given as rows of P (lattice units)."""
    P = np.asarray(P, dtype=np.float64)
    out = PREFILTER_CENTRE * f(h * P)
    for m in D4_ROOTS:
        out = out + PREFILTER_ROOT * f(h * (P + np.asarray(m, dtype=np.float64)))
    return out


def gaussian(P, sigma=GAUSS_SIGMA):
    """exp(-|x|^2 / (2 sigma^2)) at the rows of P (last axis = coordinates)."""
    P = np.asarray(P, dtype=np.float64)
    return np.exp(-(P * P).sum(axis=-1) / (2.0 * sigma * sigma))
