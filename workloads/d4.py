"""Inputs of the D4 approximation study (Sec. 5.2): the quasi-interpolation
prefilter and the Gaussian test function.  Plain arithmetic on sample values
(numpy or torch arrays alike); none of the spline's arithmetic lives here."""

import itertools

import numpy as np

# the 24 D4 sites at distance sqrt 2 from the origin (+-e_i +- e_j)
D4_ROOTS = tuple(v for v in itertools.product((-1, 0, 1), repeat=4) if sum(t * t for t in v) == 2)
PREFILTER_CENTRE = 7.0 / 3.0
PREFILTER_ROOT = -1.0 / 18.0
GAUSS_SIGMA = 0.125


def _like(v, P):
    """The tuple v as an array of P's kind (numpy, or a torch tensor on P's device)."""
    if isinstance(P, np.ndarray):
        return np.asarray(v, dtype=np.float64)
    import torch
    return torch.tensor(v, dtype=P.dtype, device=P.device)


def prefilter_samples(f, P, h=1.0):
    """c_n = 7/3 f(h n) - 1/18 sum over the 24 roots m of f(h (n + m)), at the
    sites n given as rows of P (lattice units, last axis = coordinates)."""
    out = PREFILTER_CENTRE * f(h * P)
    for m in D4_ROOTS:
        out = out + PREFILTER_ROOT * f(h * (P + _like(m, P)))
    return out


def gaussian(P, sigma=GAUSS_SIGMA):
    """exp(-|x|^2 / (2 sigma^2)) at the rows of P (last axis = coordinates)."""
    r2 = (P * P).sum(-1)
    if isinstance(P, np.ndarray):
        return np.exp(-r2 / (2.0 * sigma * sigma))
    return (-r2 / (2.0 * sigma * sigma)).exp()


def study_grid(h, cfg, margin=5):
    """Array geometry of one level: coset k's index i holds site n = 2 (i - o) + l_k
    (lattice units, world position h n); N^4 entries per coset cover every site
    within `margin` of [-0.5/h, 0.5/h]^4.  Returns (o, N)."""
    half = int(np.ceil(0.5 / h)) + margin
    o = (half + 1) // 2
    return o, 2 * o + 1
