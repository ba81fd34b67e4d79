"""GPU parity of the volume renderer (lsp_render) against the rendering
oracle: the same rays, samples, transfer function, shading and front-to-back
compositing, with f and grad f from the FP64 convolution-sum oracle."""

import numpy as np
import pytest

from oracle import ConvolutionSumOracle
from oracle.render import render_rays
from workloads import configs as W
from workloads import inputs as I

pytestmark = pytest.mark.gpu

CFG = W.get("c3")
DIMS = (24, 24, 24)


def _geometry():
    c, A = I.ray_params(CFG)
    return np.full(3, 23.5), A * (18.0 / 187.5)


def _pixel_of_ray(r, Wd):
    tile, within = r // 64, r % 64
    tiles_x = Wd // 8
    return (tile % tiles_x) * 8 + within % 8 + Wd * ((tile // tiles_x) * 8 + within // 8)


@pytest.mark.parametrize("alpha_stop", [2.0, 0.6])
def test_render_matches_oracle(lsp, alpha_stop):
    import torch
    rng = np.random.default_rng(31)
    coeffs = [rng.uniform(-1, 1, tuple(reversed(DIMS))) for _ in range(CFG.M)]
    c, A = _geometry()
    Wd, Hd, S = 64, 64, 24
    ray0, nrays = 64 * 5, 64
    tf = np.array([[0.1, 0.2, 0.9, 0.00], [0.2, 0.8, 0.3, 0.04], [0.9, 0.7, 0.1, 0.10], [1.0, 0.2, 0.1, 0.30]],
                  dtype=np.float32)
    f0, f1 = -0.6, 0.6
    sp = lsp.LatticeSpline(CFG.L, CFG.Xi)
    vol = sp.bind([torch.from_numpy(np.ascontiguousarray(a)).float().cuda() for a in coeffs])
    out = sp.render(vol, c.astype(np.float32), A.astype(np.float32), Wd, Hd, S, torch.from_numpy(tf).cuda(), f0, f1,
                    ambient=0.3, diffuse=0.7, grad_eps=1e-6, alpha_stop=alpha_stop, ray0=ray0,
                    nrays=nrays).cpu().numpy()
    pix = np.array([_pixel_of_ray(r, Wd) for r in range(ray0, ray0 + nrays)])
    P = I.ray_samples(CFG, pix[:, None], np.arange(S)[None, :], W=Wd, H=Hd, S=S,
                      params=(c.astype(np.float32), A.astype(np.float32)))
    o = ConvolutionSumOracle(CFG.L, CFG.Xi)
    c32 = [a.astype(np.float32).astype(np.float64) for a in coeffs]
    want = render_rays(o, c32, P.astype(np.float64), A[:, 2], tf.astype(np.float64), f0, f1, ambient=0.3,
                       diffuse=0.7, grad_eps=1e-6, alpha_stop=alpha_stop)
    err = float(np.max(np.abs(out - want)))
    print("render max abs err", err, "opacity range", float(want[:, 3].min()), float(want[:, 3].max()), flush=True)
    assert want[:, 3].max() > 0.2        # the rays do accumulate
    assert err <= 1e-4


def test_render_argument_errors(lsp):
    import torch
    sp = lsp.LatticeSpline(CFG.L, CFG.Xi)
    coeffs = [torch.zeros(tuple(reversed(DIMS)), device="cuda") for _ in range(CFG.M)]
    vol = sp.bind(coeffs)
    c, A = _geometry()
    tf = torch.zeros(1, 4, device="cuda")
    from paper_2102_08514_amd._lib import LspError
    with pytest.raises(LspError):
        sp.render(vol, c, A, 64, 64, 8, tf, 0.0, 1.0)              # one entry
    tf = torch.zeros(2, 4, device="cuda")
    with pytest.raises(LspError):
        sp.render(vol, c, A, 64, 64, 8, tf, 1.0, 0.0)              # empty domain
    with pytest.raises(LspError):
        sp.render(vol, c, A, 60, 64, 8, tf, 0.0, 1.0)              # W not a multiple of 8
