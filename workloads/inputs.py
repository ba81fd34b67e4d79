"""Seeded input generators.

Seeds: numpy PCG64 with seed 1000 * (config number) + stream, where stream
0 = coefficients, 1 = queries, 2 = targets, 3 = field parameters.

Smooth field (stand-in for the paper's Marschner--Lobb test volume, Sec.
5.1, which is not reproduced): g(p) = (1/8) sum_{i=1..8} sin(2 pi k_i . p +
theta_i) with k_i = f_i u_i / D, f_i ~ U[0, 0.2] cycles per coset-array
spacing D, u_i uniform on the unit sphere, theta_i ~ U[0, 2 pi); optional
additive N(0, noise^2) noise.  Values are generated in float64 and stored in
the configuration's dtype.
"""

import numpy as np

from .configs import CONFIGS


def _seed_index(name):
    """c1..c5 keep their number; the other workloads follow in table order."""
    if name[0] == "c" and name[1:].isdigit():
        return int(name[1:])
    others = [n for n in CONFIGS if not (n[0] == "c" and n[1:].isdigit())]
    return 6 + others.index(name)


def _rng(cfg, stream):
    return np.random.Generator(np.random.PCG64(1000 * _seed_index(cfg.name) + stream))


def field_params(cfg, stream=3, count=8):
    rng = _rng(cfg, stream)
    s = cfg.s
    u = rng.normal(size=(count, s))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    f = rng.uniform(0.0, 0.2, size=count)
    theta = rng.uniform(0.0, 2 * np.pi, size=count)
    k = (f[:, None] * u) / cfg.D
    return k, theta


def smooth_field(cfg, P, stream=3):
    """g at the rows of P (world coordinates), float64."""
    k, theta = field_params(cfg, stream)
    P = np.asarray(P, dtype=np.float64)
    out = np.zeros(P.shape[:-1])
    for ki, th in zip(k, theta):
        out += np.sin(2 * np.pi * (P @ ki) + th)
    return out / len(k)


def site_coordinates(cfg, k, dims=None):
    """World coordinates D i + l_k of coset k's array, shape (n_{s-1},...,n_0, s)."""
    dims = tuple(dims or cfg.dims)
    idx = np.indices(tuple(reversed(dims)), dtype=np.float64)      # (s, n_{s-1}, ..., n_0)
    coords = [cfg.D * idx[cfg.s - 1 - a] + cfg.shifts[k][a] for a in range(cfg.s)]
    return np.stack(coords, axis=-1)


def coefficients(cfg, dims=None, dtype=None):
    """List of M coefficient arrays of shape (n_{s-1}, ..., n_0)."""
    dims = tuple(dims or cfg.dims)
    shape = tuple(reversed(dims))
    rng = _rng(cfg, 0)
    out = []
    if cfg.coeff_kind == "uniform":
        for _ in range(cfg.M):
            out.append(rng.uniform(-1.0, 1.0, size=shape))
        dt = dtype or np.float64
    else:
        for k in range(cfg.M):
            v = np.zeros(shape)
            # slab-wise to bound memory for the big volumes
            idx_last = np.arange(shape[0])
            for z0 in range(0, shape[0], 16):
                zs = idx_last[z0:z0 + 16]
                sub = np.indices((len(zs),) + shape[1:], dtype=np.float64)
                sub[0] += z0
                coords = [cfg.D * sub[cfg.s - 1 - a] + cfg.shifts[k][a] for a in range(cfg.s)]
                v[z0:z0 + 16] = smooth_field(cfg, np.stack(coords, axis=-1))
            if cfg.noise:
                v += rng.normal(0.0, cfg.noise, size=shape)
            out.append(v)
        dt = dtype or np.float32
    return [np.ascontiguousarray(o.astype(dt)) for o in out]


def queries(cfg, n=None, lo=None, hi=None):
    """n uniform queries in [lo, hi]^s, rounded to float32 (the values every
    implementation sees)."""
    n = cfg.n_queries if n is None else n
    rng = _rng(cfg, 1)
    lo = cfg.lo if lo is None else lo
    hi = cfg.hi if hi is None else hi
    return rng.uniform(lo, hi, size=(n, cfg.s)).astype(np.float32)


def targets(cfg, X):
    """MSE targets y = g_T(x) from an independent field (stream 2), float32."""
    return smooth_field(cfg, np.asarray(X, dtype=np.float64), stream=2).astype(np.float32)


def ray_params(cfg, primary=True):
    """Orthographic ray grid through the volume: p = c + R a (2(u+1/2)/W - 1,
    2(v+1/2)/H - 1, 2(j+1/2)/S - 1), u < W, v < H, j < S.  Primary rays use
    R = Rz(30 deg) Rx(20 deg) and a = 187.5/sqrt(3) (every sample interior and
    oblique to the lattice); secondary rays are axis aligned with a = 187.5.
    Returns (centre, columns of R*a as a 3x3 matrix) in float64."""
    centre = np.full(3, 191.5)
    if primary:
        a = 187.5 / np.sqrt(3.0)
        cz, sz = np.cos(np.radians(30.0)), np.sin(np.radians(30.0))
        cx, sx = np.cos(np.radians(20.0)), np.sin(np.radians(20.0))
        Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
        Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
        R = Rz @ Rx
    else:
        a = 187.5
        R = np.eye(3)
    return centre, R * a


def ray_samples(cfg, pixels, steps, W=1024, H=1024, S=512, primary=True, params=None):
    """World positions of the samples (pixel index u + W v, step j), computed
    in float32 exactly as the GPU ray generator does: p = c + A t with
    t = 2(q + 1/2)/n - 1 per axis, each float32 operation rounded.
    params: (c, A) instead of the workload's own ray grid."""
    c, A = ray_params(cfg, primary) if params is None else (np.asarray(params[0]), np.asarray(params[1]))
    c32 = c.astype(np.float32)
    A32 = A.astype(np.float32)
    pixels = np.asarray(pixels, dtype=np.int64)
    steps = np.asarray(steps, dtype=np.int64)
    u = (pixels % W).astype(np.float32)
    v = (pixels // W).astype(np.float32)
    j = steps.astype(np.float32)
    two = np.float32(2.0)
    half = np.float32(0.5)
    one = np.float32(1.0)
    tu = (two * (u + half)) / np.float32(W) - one
    tv = (two * (v + half)) / np.float32(H) - one
    tj = (two * (j + half)) / np.float32(S) - one
    out = np.empty(np.broadcast(tu, tj).shape + (3,), dtype=np.float32)
    for a in range(3):
        acc = c32[a] + A32[a, 0] * tu
        acc = acc + A32[a, 1] * tv
        acc = acc + A32[a, 2] * tj
        out[..., a] = acc
    return out
