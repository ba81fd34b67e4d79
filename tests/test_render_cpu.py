"""Pins of the rendering oracle (front-to-back compositing of Sec. 5.1's
volume renderer) against closed forms.

- Constant data: partition of unity makes f constant and grad f zero, so
  every sample has the same alpha and colour and the opacity after S samples
  is 1 - (1 - alpha)^S (a geometric series); the colour is that opacity times
  the shaded colour.
- Linear data: f = a.x + b exactly (linear precision), grad f = a, so the
  shading is the constant ambient + diffuse |a.d| / |a|, and every sample's
  transfer-function value is known in closed form.
- Early termination stops at the first sample whose opacity reaches the bound.
"""

import numpy as np

from oracle import ConvolutionSumOracle
from oracle.render import composite, render_rays, transfer
from workloads import configs as W

CFG = W.get("c3")
DIMS = (10, 10, 10)


def _sites(k):
    idx = np.indices(tuple(reversed(DIMS)), dtype=np.float64)
    return np.stack([CFG.D * idx[2 - a] + CFG.shifts[k][a] for a in range(3)], axis=-1)


def _rays(R=5, S=7, seed=0):
    rng = np.random.default_rng(seed)
    start = rng.uniform(5.0, 8.0, (R, 1, 3))
    d = np.array([0.3, -0.2, 0.9])
    t = np.linspace(0.0, 4.0, S)[None, :, None]
    return (start + t * d).astype(np.float32).astype(np.float64), d


def test_transfer_function_lookup():
    tf = np.array([[0, 0, 0, 0], [1, 0, 0, 0.5], [1, 1, 0, 1.0]], dtype=np.float64)
    np.testing.assert_allclose(transfer(tf, -1.0, 1.0, -5.0), tf[0])
    np.testing.assert_allclose(transfer(tf, -1.0, 1.0, 0.5), (tf[1] + tf[2]) / 2)
    np.testing.assert_allclose(transfer(tf, -1.0, 1.0, 3.0), tf[2])


def test_constant_volume_geometric_series():
    o = ConvolutionSumOracle(CFG.L, CFG.Xi)
    v = 0.25
    coeffs = [np.full(tuple(reversed(DIMS)), v) for _ in range(CFG.M)]
    P, d = _rays()
    tf = np.array([[0.2, 0.4, 0.6, 0.1], [0.8, 0.6, 0.4, 0.3]])
    out = render_rays(o, coeffs, P, d, tf, 0.0, 1.0, ambient=0.25, diffuse=0.5)
    rgba = tf[0] * 0.75 + tf[1] * 0.25
    S = P.shape[1]
    A = 1.0 - (1.0 - rgba[3]) ** S
    np.testing.assert_allclose(out[:, 3], A, rtol=1e-12)
    np.testing.assert_allclose(out[:, :3], np.tile(A * 0.75 * rgba[:3], (len(out), 1)), rtol=1e-10)


def test_linear_volume_closed_form():
    o = ConvolutionSumOracle(CFG.L, CFG.Xi)
    a, b = np.array([0.05, -0.02, 0.03]), 0.1
    coeffs = [_sites(k) @ a + b for k in range(CFG.M)]
    P, d = _rays(seed=1)
    tf = np.array([[0.0, 0.5, 1.0, 0.05], [1.0, 0.5, 0.0, 0.25]])
    f0, f1 = 0.0, 1.0
    out = render_rays(o, coeffs, P, d, tf, f0, f1, ambient=0.2, diffuse=0.8)
    shade = 0.2 + 0.8 * abs(a @ (d / np.linalg.norm(d))) / np.linalg.norm(a)
    want = np.zeros((P.shape[0], 4))
    for r in range(P.shape[0]):
        C, A = np.zeros(3), 0.0
        for j in range(P.shape[1]):
            s = np.clip((P[r, j] @ a + b - f0) / (f1 - f0), 0.0, 1.0)
            rgba = tf[0] * (1 - s) + tf[1] * s
            C += (1 - A) * rgba[3] * shade * rgba[:3]
            A += (1 - A) * rgba[3]
        want[r, :3], want[r, 3] = C, A
    np.testing.assert_allclose(out, want, rtol=1e-9, atol=1e-12)


def test_early_termination():
    f = np.zeros((1, 10))
    g = np.zeros((1, 10, 3))
    tf = np.array([[1.0, 1.0, 1.0, 0.5], [1.0, 1.0, 1.0, 0.5]])
    out = composite(f, g, [0, 0, 1], tf, 0.0, 1.0, 1.0, 0.0, 1e-6, alpha_stop=0.8)
    # opacities 0.5, 0.75, 0.875: the third sample is the last one composited
    assert abs(out[0, 3] - 0.875) < 1e-15
