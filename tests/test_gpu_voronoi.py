"""GPU parity of the Voronoi splines (Sec. 3, Voronoi splines; Table 1 Voronoi
rows) through the C ABI against the FP64 oracle.

Expected values come from tests/golden/voronoi_expected.npz, which
make_voronoi_expected.py writes by calling oracle/ alone on the inputs that
gpu_cases.small_case regenerates from seeds (the oracle's box-spline form is
slow for these splines).  Tolerances as for the box splines (normwise,
relative to max |c|): FP32 1e-5, FP64 accumulation 1e-11, BF16 storage 1e-5
against the rounded coefficients and 2e-3 against the unrounded ones,
grad f 1e-4, dL/dc 1e-5 max_m sum_q |g_q| phi(x_q - m).  V_1 is only C^0:
its gradient is two-valued on the mesh planes, so the 48 queries placed on
sites and half-integers are left out of its gradient checks.
"""

import os

import numpy as np
import pytest

from gpu_cases import bf16_round, normwise, rounded, small_case, tile_pixels, to_dev, voronoi_oracle
from workloads import configs as W
from workloads import inputs as I

pytestmark = pytest.mark.gpu

VOR = ["vor_bcc1", "vor_fcc1", "vor_cc_bcc1", "vor_cc_fcc1", "vor_fcc2", "vor_cc_fcc2"]
TABLE = {"vor_bcc1": "bcc_voronoi1", "vor_fcc1": "fcc_voronoi1", "vor_cc_bcc1": "cc_bcc_voronoi1",
         "vor_cc_fcc1": "cc_fcc_voronoi1", "vor_fcc2": "fcc_voronoi2", "vor_cc_fcc2": "cc_fcc_voronoi2"}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "voronoi_expected.npz")
_EXP = {}


def expected(name, key):
    if not _EXP:
        with np.load(GOLDEN, allow_pickle=False) as z:
            _EXP.update({k: z[k] for k in z.files})
    return _EXP[f"{name}/{key}"]


def _torch():
    import torch
    return torch


def _spline(lsp, cfg):
    return lsp.LatticeSpline(cfg.L, voronoi=(cfg.Lv, cfg.voronoi[1]))


def _smooth_mask(name, n):
    keep = np.ones(n, dtype=bool)
    if W.get(name).voronoi[1] == 1:
        keep[-48:] = False
    return keep


@pytest.mark.parametrize("name", VOR)
def test_plan(lsp, name):
    cfg = W.get(name)
    sp = _spline(lsp, cfg)
    info = sp.info
    assert info["kind"] == "voronoi" and info["voronoi_n"] == cfg.voronoi[1]
    assert info["name"] == TABLE[name]
    assert info["n_cosets"] == cfg.M and info["lookups"] == cfg.lookups
    # a box-spline plan is never matched by a Voronoi spline's generators, and vice versa
    from paper_2102_08514_amd._lib import LspError
    with pytest.raises(LspError):
        lsp.LatticeSpline(cfg.L, voronoi=(cfg.Lv, 7))


@pytest.mark.parametrize("name", VOR)
def test_forward_fp32_given_and_scheduled(lsp, name):
    torch = _torch()
    cfg, coeffs, X = small_case(name)
    want = expected(name, "f")
    sp = _spline(lsp, cfg)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    x = torch.from_numpy(X).cuda()
    for sch in (None, sp.schedule(vol, x)):
        f = sp.eval(vol, x, schedule=sch).cpu().numpy()
        err = normwise(f, want, coeffs)
        print(name, "fp32", "scheduled" if sch else "given", f"{err:.2e}", flush=True)
        assert err <= 1e-5


@pytest.mark.parametrize("name", VOR)
def test_forward_fp64_check(lsp, name):
    torch = _torch()
    cfg, coeffs, X = small_case(name)
    want = expected(name, "f")
    sp = _spline(lsp, cfg)
    vol = sp.bind(to_dev(coeffs, torch.float64))
    x = torch.from_numpy(X).cuda()
    for sch in (None, sp.schedule(vol, x)):
        f = sp.eval(vol, x, schedule=sch)
        assert f.dtype == torch.float64
        err = normwise(f.cpu().numpy(), want, coeffs)
        print(name, "fp64", f"{err:.2e}", flush=True)
        assert err <= 1e-11


@pytest.mark.parametrize("name", VOR)
def test_forward_bf16_storage(lsp, name):
    torch = _torch()
    cfg, coeffs, X = small_case(name)
    sp = _spline(lsp, cfg)
    dev = to_dev(coeffs, torch.bfloat16)
    # the golden file rounds with the same round-to-nearest-even rule
    assert all(np.array_equal(a, bf16_round(c)) for a, c in zip(rounded(dev), coeffs))
    vol = sp.bind(dev)
    x = torch.from_numpy(X).cuda()
    for sch in (None, sp.schedule(vol, x)):
        f = sp.eval(vol, x, schedule=sch).cpu().numpy()
        assert normwise(f, expected(name, "f_bf16"), coeffs) <= 1e-5
        assert normwise(f, expected(name, "f"), coeffs) <= 2e-3


@pytest.mark.parametrize("name", VOR)
def test_gradient(lsp, name):
    torch = _torch()
    cfg, coeffs, X = small_case(name)
    keep = _smooth_mask(name, len(X))
    sp = _spline(lsp, cfg)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    x = torch.from_numpy(X).cuda()
    for sch in (None, sp.schedule(vol, x)):
        _, g = sp.eval(vol, x, grad=True, schedule=sch)
        err = normwise(g.cpu().numpy()[keep], expected(name, "grad")[keep], coeffs)
        print(name, "grad", f"{err:.2e}", flush=True)
        assert err <= 1e-4


@pytest.mark.parametrize("name", VOR)
def test_adjoint_given_and_scheduled(lsp, name):
    torch = _torch()
    cfg, coeffs, X = small_case(name)
    g = np.random.default_rng(5).normal(size=len(X)).astype(np.float32)
    want = expected(name, "adj")
    bound = float(np.max(expected(name, "adj_abs")))
    keep = _smooth_mask(name, len(X))
    sp = _spline(lsp, cfg)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    x, gd = torch.from_numpy(X).cuda(), torch.from_numpy(g).cuda()
    for sch in (None, sp.schedule(vol, x)):
        gc, gx = sp.adjoint(vol, x, gd, grad_x=True, schedule=sch)
        err = max(float(np.max(np.abs(a.cpu().numpy() - b))) for a, b in zip(gc, want)) / bound
        print(name, "adjoint", "scheduled" if sch else "given", f"{err:.2e}", flush=True)
        assert err <= 1e-5
        gw = g[:, None].astype(np.float64) * expected(name, "grad")
        assert normwise(gx.cpu().numpy()[keep], gw[keep], coeffs) <= 1e-4 * float(np.max(np.abs(g)))


@pytest.mark.parametrize("name", ["vor_bcc1", "vor_fcc1", "vor_cc_bcc1", "vor_fcc2"])
def test_mse_training_step(lsp, name):
    """Scheduled MSE forward + fused backward: the loss from f, and dL/dc
    against the given-order adjoint of the same dL/df (itself pinned against
    the oracle above)."""
    torch = _torch()
    cfg, coeffs, X = small_case(name)
    want = expected(name, "f")
    y = np.random.default_rng(9).uniform(-1, 1, len(X)).astype(np.float32)
    sp = _spline(lsp, cfg)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    x, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    sch = sp.schedule(vol, x)
    f, dldf, loss = sp.eval_mse(vol, x, yd, schedule=sch)
    assert normwise(f.cpu().numpy(), want, coeffs) <= 1e-5
    r = want - y
    assert abs(float(loss.item()) - float(np.mean(r * r))) <= 1e-4 * max(1.0, float(np.mean(r * r)))
    gc = sp.mse_backward(vol, x, sch)
    ref, _ = sp.adjoint(vol, x, dldf)
    bound = max(float(t.abs().max()) for t in sp.adjoint(vol, x, dldf.abs())[0])
    err = max(float((a - b).abs().max()) for a, b in zip(gc, ref)) / bound
    print(name, "fused backward vs given-order adjoint", f"{err:.2e}", flush=True)
    assert err <= 1e-5


def test_rays_per_sample_bcc_voronoi1(lsp):
    """The ray sampler with the BCC Voronoi spline: every sample's f and
    grad f against the oracle at the same float32 positions."""
    torch = _torch()
    cfg = W.get("vor_bcc1")
    dims = (16, 16, 16)
    rng = np.random.default_rng(71)
    coeffs = [rng.uniform(-1, 1, tuple(reversed(dims))) for _ in range(cfg.M)]
    _, A = I.ray_params(W.get("c3"))
    centre, A = np.full(3, 15.5, dtype=np.float32), (A * (11.0 / 187.5)).astype(np.float32)
    Wd, Hd, S = 16, 8, 19
    ray0, nrays = 5, 23
    sp = _spline(lsp, cfg)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    out, smp = sp.rays(vol, centre, A, Wd, Hd, S, ray0=ray0, nrays=nrays, samples=True)
    pix = tile_pixels(np.arange(ray0, ray0 + nrays), Wd)
    P = I.ray_samples(W.get("c3"), pix[:, None], np.arange(S)[None, :], W=Wd, H=Hd, S=S, params=(centre, A))
    P64 = P.reshape(-1, 3).astype(np.float64)
    f, g = voronoi_oracle(cfg).eval(coeffs, P64, want_grad=True)
    smp = smp.cpu().numpy().reshape(-1, 4)
    assert normwise(smp[:, 0], f, coeffs) <= 1e-5
    assert normwise(smp[:, 1:], g, coeffs) <= 1e-4
    # per-ray sums are the sums of the samples
    np.testing.assert_allclose(out.cpu().numpy()[:, 0], smp[:, 0].reshape(nrays, S).sum(axis=1), atol=1e-4)
