"""Shared case builders of the GPU parity tests (seeded inputs only; no
arithmetic of the method)."""

import numpy as np

from workloads import configs as W

SMALL = {"c1": (12, 12, 12), "c2": (20, 20, 20), "c3": (12, 12, 12), "c4": (10, 10, 10), "c5": (7, 7, 7, 7),
         "d4": (8, 8, 8, 8), "cc_tp2": (20, 20, 20), "cc_tp3": (20, 20, 20), "cc_tp4": (20, 20, 20),
         "cc_linear_rd": (20, 20, 20), "bcc_quintic_rd": (12, 12, 12),
         "vor_bcc1": (12, 12, 12), "vor_fcc1": (10, 10, 10), "vor_cc_bcc1": (20, 20, 20), "vor_cc_fcc1": (20, 20, 20),
         "vor_fcc2": (10, 10, 10), "vor_cc_fcc2": (14, 14, 14)}
NQ = {"c1": 1301, "c2": 1301, "c3": 1301, "c4": 1301, "c5": 601, "d4": 401, "cc_tp2": 1301, "cc_tp3": 1301,
      "cc_tp4": 96, "cc_linear_rd": 1301, "bcc_quintic_rd": 1301,   # cc_tp4: 12 directions make the oracle slow
      "vor_bcc1": 601, "vor_fcc1": 601, "vor_cc_bcc1": 401, "vor_cc_fcc1": 601, "vor_fcc2": 301, "vor_cc_fcc2": 201}


def voronoi_oracle(cfg):
    """The oracle of a Voronoi-spline configuration (the box-spline expansion,
    pinned against the overlap-volume definition on the CPU)."""
    from oracle import VoronoiSumOracle
    return VoronoiSumOracle(cfg.L, cfg.Lv, cfg.voronoi[1], W=cfg.voronoi_gen, sigma=W.VORONOI_SIGMA,
                            method="boxsum")


def small_case(name, n=None, seed=0):
    """Coefficients U[-1, 1] on small arrays and n float32 queries: half in the
    interior, the rest straddling and leaving the stored arrays, and 48 on
    lattice sites, half-integers and quarter points."""
    cfg = W.get(name)
    dims = SMALL[name]
    rng = np.random.default_rng(1000 + seed)
    coeffs = [rng.uniform(-1, 1, tuple(reversed(dims))) for _ in range(cfg.M)]
    n = NQ[name] if n is None else n
    ext = cfg.D * (dims[0] - 1) + 1
    X = rng.uniform(-2.0, ext + 1.0, (n, cfg.s))
    X[: n // 2] = rng.uniform(cfg.D * 2, ext - cfg.D * 2 - 1, (n // 2, cfg.s))
    special = rng.integers(3, ext - 4, (48, cfg.s)).astype(float)
    special[16:32] += 0.5
    special[32:40] += rng.integers(0, 2, (8, cfg.s)) * 0.25
    X[-48:] = special
    return cfg, coeffs, X.astype(np.float32)


def bf16_round(a):
    """Values rounded to bfloat16 (nearest, ties to even) through float32, in
    float64: what a round-to-nearest-even device conversion stores."""
    b = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def to_dev(arrs, dtype):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda() for a in arrs]


def rounded(dev):
    """The stored values of device arrays (after the RNE conversion), in FP64."""
    return [d.float().cpu().numpy().astype(np.float64) for d in dev]


def normwise(a, b, coeffs):
    scale = max(float(np.max(np.abs(c))) for c in coeffs)
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)))) / scale


def tile_pixels(rays, W):
    """Pixel index u + W v of ray r (8 x 8 tiles, row-major tile order)."""
    r = np.asarray(rays)
    tile, within = r >> 6, r & 63
    u = (tile % (W // 8)) * 8 + (within & 7)
    v = (tile // (W // 8)) * 8 + (within >> 3)
    return u + W * v


def interior_sites(cfg, count, lo_idx, hi_idx, seed):
    """count random (coset, index) sites with every index in [lo_idx, hi_idx)."""
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(cfg.M)), tuple(int(v) for v in rng.integers(lo_idx, hi_idx, cfg.s)))
            for _ in range(count)]
