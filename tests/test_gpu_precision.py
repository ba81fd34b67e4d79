"""GPU parity of the reduced-precision storage forms and of the scheduled
(binned) adjoint, element by element against the FP64 oracle.

Tolerances (normwise, relative to max |c|):
  f      1e-5 against the oracle on the stored (rounded) coefficients,
         2e-3 against the unrounded ones (BF16 round-to-nearest-even storage
         errs by at most 2^-9 max |c|);
  grad f 1e-4 (one digit lost to differentiation);
  dL/dc  1e-5 max_m sum_q |g_q| phi(x_q - m) per site, plus, where g is the
         MSE head's dL/df = 2 (f - y) / n, the part that f's own 1e-5 error
         carries into g: (2/n) 1e-5 max|c| max_m sum_q phi(x_q - m).
The oracle never sees a value the GPU computed: upstream gradients are
seeded inputs, or the oracle's own dL/df.
"""

import numpy as np
import pytest

from gpu_cases import SMALL, interior_sites, normwise, rounded, small_case, tile_pixels, to_dev
from oracle import ConvolutionSumOracle
from oracle.render import render_rays
from workloads import configs as W
from workloads import inputs as I

pytestmark = pytest.mark.gpu

TDT = {"bf16": "bfloat16", "f16": "float16", "f32": "float32"}


def _tdt(name):
    import torch
    return getattr(torch, TDT[name])


def _oracle_mse(o, coeffs, X, y, dims):
    """The oracle's own MSE step: f*, dL/df = 2 (f* - y) / n, L, and the
    adjoint of dL/df with the two bounds of the per-site tolerance."""
    n = len(X)
    X64 = X.astype(np.float64)
    f, gf = o.eval(coeffs, X64, want_grad=True)
    r = f - y.astype(np.float64)
    g = 2.0 * r / n
    adj = o.adjoint(X64, g, dims)
    b_abs = max(float(np.max(a)) for a in o.adjoint(X64, np.abs(g), dims))
    b_one = max(float(np.max(a)) for a in o.adjoint(X64, np.ones(n), dims))
    return f, gf, r, g, adj, b_abs, b_one


# --------------------------------------------------------------------------- rays (c3)
def _small_ray_case(seed):
    cfg = W.get("c3")
    dims = (16, 16, 16)
    rng = np.random.default_rng(seed)
    coeffs = [rng.uniform(-1, 1, tuple(reversed(dims))) for _ in range(cfg.M)]
    c, A = I.ray_params(cfg)
    return cfg, coeffs, np.full(3, 15.5), A * (11.0 / 187.5)


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_rays_low_precision_per_sample(lsp, dt):
    """c3's sampler (k_rays) with BF16 / FP16 storage: every sample's f and
    grad f against the oracle at the same float32 positions."""
    cfg, coeffs, centre, A = _small_ray_case(51)
    Wd, Hd, S = 16, 8, 37
    ray0, nrays = 3, 101
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    dev = to_dev(coeffs, _tdt(dt))
    vol = sp.bind(dev)
    out, smp = sp.rays(vol, centre.astype(np.float32), A.astype(np.float32), Wd, Hd, S, ray0=ray0, nrays=nrays,
                       samples=True)
    pix = tile_pixels(np.arange(ray0, ray0 + nrays), Wd)
    P = I.ray_samples(cfg, pix[:, None], np.arange(S)[None, :], W=Wd, H=Hd, S=S,
                      params=(centre.astype(np.float32), A.astype(np.float32)))
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    P64 = P.reshape(-1, 3).astype(np.float64)
    fr, gr = o.eval(rounded(dev), P64, want_grad=True)
    fu = o.eval(coeffs, P64)
    smp = smp.cpu().numpy().reshape(-1, 4)
    e_r, e_u, e_g = normwise(smp[:, 0], fr, coeffs), normwise(smp[:, 0], fu, coeffs), normwise(smp[:, 1:], gr, coeffs)
    print(f"c3 {dt} rays: f vs rounded {e_r:.2e}, vs unrounded {e_u:.2e}, grad {e_g:.2e}", flush=True)
    assert e_r <= 1e-5 and e_g <= 1e-4 and e_u <= 2e-3
    out = out.cpu().numpy()
    np.testing.assert_allclose(out[:, 0], fr.reshape(nrays, S).sum(1), rtol=0, atol=S * 1e-5)
    np.testing.assert_allclose(out[:, 1:], gr.reshape(nrays, S, 3).sum(1), rtol=0, atol=S * 1e-4)


def test_render_bf16(lsp):
    """The volume renderer with BF16 storage against the rendering oracle on
    the stored coefficients."""
    import torch
    cfg = W.get("c3")
    dims = (24, 24, 24)
    rng = np.random.default_rng(52)
    coeffs = [rng.uniform(-1, 1, tuple(reversed(dims))) for _ in range(cfg.M)]
    _, A = I.ray_params(cfg)
    A = A * (18.0 / 187.5)
    c = np.full(3, 23.5)
    Wd, Hd, S = 64, 64, 24
    ray0, nrays = 64 * 7, 64
    tf = np.array([[0.1, 0.2, 0.9, 0.00], [0.2, 0.8, 0.3, 0.04], [0.9, 0.7, 0.1, 0.10], [1.0, 0.2, 0.1, 0.30]],
                  dtype=np.float32)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    dev = to_dev(coeffs, torch.bfloat16)
    vol = sp.bind(dev)
    out = sp.render(vol, c.astype(np.float32), A.astype(np.float32), Wd, Hd, S, torch.from_numpy(tf).cuda(), -0.6,
                    0.6, alpha_stop=2.0, ray0=ray0, nrays=nrays).cpu().numpy()
    pix = tile_pixels(np.arange(ray0, ray0 + nrays), Wd)
    P = I.ray_samples(cfg, pix[:, None], np.arange(S)[None, :], W=Wd, H=Hd, S=S,
                      params=(c.astype(np.float32), A.astype(np.float32)))
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    want = render_rays(o, rounded(dev), P.astype(np.float64), A[:, 2], tf.astype(np.float64), -0.6, 0.6,
                       ambient=0.3, diffuse=0.7, grad_eps=1e-6, alpha_stop=2.0)
    err = float(np.max(np.abs(out - want)))
    print("render bf16 max abs err", err, flush=True)
    assert want[:, 3].max() > 0.2 and err <= 1e-4


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_rays_full_size_per_sample_c3(lsp, dt):
    """c3's full launch (2 x 192^3, 1024^2 rays x 512 steps, f and grad f
    summed per ray) in FP32 and BF16 storage: sampled rays are checked sample
    by sample.  The per-ray sums come from the full launch; the samples from
    one-ray launches of the same rays, whose sums must equal the full
    launch's bit for bit (same positions, same arithmetic)."""
    import torch
    cfg = W.get("c3")
    coeffs = I.coefficients(cfg)
    Wd, Hd = cfg.extra["rays"]
    S = cfg.extra["steps"]
    c, A = I.ray_params(cfg)
    c32, A32 = c.astype(np.float32), A.astype(np.float32)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    dev = to_dev(coeffs, _tdt(dt))
    vol = sp.bind(dev)
    out = sp.rays(vol, c32, A32, Wd, Hd, S).cpu().numpy()
    assert out.shape == (Wd * Hd, 4) and np.all(np.isfinite(out))
    rays = np.concatenate([[0, Wd * Hd - 1], np.random.default_rng(44).choice(Wd * Hd, 2, replace=False)])
    stored = rounded(dev)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    for r in rays:
        one, smp = sp.rays(vol, c32, A32, Wd, Hd, S, ray0=int(r), nrays=1, samples=True)
        assert torch.equal(one.cpu(), torch.from_numpy(out[r:r + 1]))
        P = I.ray_samples(cfg, tile_pixels([r], Wd)[:, None], np.arange(S)[None, :], W=Wd, H=Hd, S=S)
        fw, gw = o.eval(stored, P.reshape(-1, 3).astype(np.float64), want_grad=True)
        smp = smp.cpu().numpy().reshape(-1, 4)
        ef, eg = normwise(smp[:, 0], fw, coeffs), normwise(smp[:, 1:], gw, coeffs)
        print(f"c3 {dt} full-size ray {r}: f {ef:.2e}, grad {eg:.2e}", flush=True)
        assert ef <= 1e-5 and eg <= 1e-4
        if dt == "bf16":
            assert normwise(smp[:, 0], o.eval(coeffs, P.reshape(-1, 3).astype(np.float64)), coeffs) <= 2e-3


# --------------------------------------------------------------------------- scheduled adjoint (c5, D4)
@pytest.mark.parametrize("name", ["c5", "d4"])
def test_scheduled_adjoint_every_site(lsp, name):
    """The split (query, coset) scheduled adjoint with a seeded upstream
    gradient: every site of grad_c and every query's grad_x against the
    oracle."""
    import torch
    cfg, coeffs, X = small_case(name, seed=61)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    g = np.random.default_rng(62).normal(size=len(X)).astype(np.float32)
    X64, g64 = X.astype(np.float64), g.astype(np.float64)
    want = o.adjoint(X64, g64, SMALL[name])
    bound = max(float(np.max(a)) for a in o.adjoint(X64, np.abs(g64), SMALL[name]))
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    dev = to_dev(coeffs, torch.float32)
    vol = sp.bind(dev)
    x = torch.from_numpy(X).cuda()
    sch = sp.schedule(vol, x)
    gc, gx = sp.adjoint(vol, x, torch.from_numpy(g).cuda(), grad_x=True, schedule=sch)
    err = max(float(np.max(np.abs(a.cpu().numpy() - b))) for a, b in zip(gc, want)) / bound
    print(f"{name} scheduled adjoint: max site err / bound {err:.2e}", flush=True)
    assert err <= 1e-5
    _, gw = o.eval(rounded(dev), X64, want_grad=True)
    assert normwise(gx.cpu().numpy(), g64[:, None] * gw, coeffs) <= 1e-4 * max(1.0, float(np.max(np.abs(g))))


@pytest.mark.parametrize("name,dt", [("c5", "f32"), ("c5", "bf16"), ("d4", "f32")])
def test_scheduled_mse_step_every_site(lsp, name, dt):
    """The scheduled MSE forward (f, dL/df, L, dL/dx) and the fused backward
    (dL/dc from the dL/df kept in the workspace), in FP32 and BF16 storage,
    against the oracle's own MSE step on the stored coefficients, at every
    query and every site."""
    import torch
    cfg, coeffs, X = small_case(name, seed=63)
    n = len(X)
    y = I.targets(cfg, X)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    dev = to_dev(coeffs, _tdt(dt))
    vol = sp.bind(dev)
    x, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    sch = sp.schedule(vol, x)
    f, dldf, loss, dldx = sp.eval_mse(vol, x, yd, schedule=sch, grad_x=True)
    gc = sp.mse_backward(vol, x, sch)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    stored = rounded(dev)
    fw, gfw, r, g, adj, b_abs, b_one = _oracle_mse(o, stored, X, y, SMALL[name])
    cmax = max(float(np.max(np.abs(c))) for c in coeffs)
    assert normwise(f.cpu().numpy(), fw, coeffs) <= 1e-5
    if dt == "bf16":
        assert normwise(f.cpu().numpy(), o.eval(coeffs, X.astype(np.float64)), coeffs) <= 2e-3
    np.testing.assert_allclose(dldf.cpu().numpy(), g, rtol=0, atol=(2.0 / n) * 1e-5 * cmax)
    assert abs(float(loss.item()) - float(np.mean(r * r))) <= 2 * float(np.mean(np.abs(r))) * 1e-5 * cmax + 1e-12
    np.testing.assert_allclose(dldx.cpu().numpy(), g[:, None] * gfw, rtol=0,
                               atol=(2.0 / n) * 1e-4 * cmax * max(1.0, float(np.max(np.abs(r)))))
    tol = 1e-5 * b_abs + (2.0 / n) * 1e-5 * cmax * b_one
    err = max(float(np.max(np.abs(a.cpu().numpy() - b))) for a, b in zip(gc, adj))
    print(f"{name} {dt} fused MSE backward: max site err {err:.2e} (tol {tol:.2e})", flush=True)
    assert err <= tol


# --------------------------------------------------------------------------- full size, sampled
@pytest.mark.parametrize("name,sites", [("c5", 96), ("d4", 48)])
def test_scheduled_adjoint_full_size_sites(lsp, name, sites):
    """c5 (2 x 48^4) and the D4 spline (8 x 24^4) at full size, 2^22 queries,
    through the schedule the benchmark uses: grad_c of a seeded upstream
    gradient at sampled sites against the oracle's column sums."""
    import torch
    cfg = W.get(name)
    coeffs = I.coefficients(cfg)
    X = I.queries(cfg)
    g = np.random.default_rng(64).normal(size=len(X)).astype(np.float32)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    x = torch.from_numpy(X).cuda()
    sch = sp.schedule(vol, x)
    gc, _ = sp.adjoint(vol, x, torch.from_numpy(g).cuda(), schedule=sch)
    lo = int(np.ceil(cfg.lo / cfg.D)) + 1
    hi = int(np.floor(cfg.hi / cfg.D)) - 1
    pick = interior_sites(cfg, sites, lo, hi, seed=65)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    X64 = X.astype(np.float64)
    want = o.adjoint_at(X64, g.astype(np.float64), pick)
    bound = float(np.max(o.adjoint_at(X64, np.abs(g).astype(np.float64), pick)))
    got = np.array([float(gc[k][tuple(reversed(idx))]) for k, idx in pick])
    err = float(np.max(np.abs(got - want))) / bound
    print(f"{name} full-size scheduled adjoint at {sites} sites: max err / bound {err:.2e}", flush=True)
    assert bound > 0 and err <= 1e-5


def test_mse_step_full_size_bf16_c5(lsp):
    """c5 at full size (2 x 48^4, 2^22 queries) with BF16 storage through the
    benchmark's launch: scheduled MSE forward and fused backward.  Sampled f
    against the oracle on the stored and on the unrounded coefficients, and
    dL/dc at sampled sites against the oracle's dL/df = 2 (f* - y) / n summed
    over the queries in each site's support."""
    import torch
    cfg = W.get("c5")
    coeffs = I.coefficients(cfg)
    X = I.queries(cfg)
    n = len(X)
    y = I.targets(cfg, X)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    dev = to_dev(coeffs, torch.bfloat16)
    vol = sp.bind(dev)
    x, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    sch = sp.schedule(vol, x)
    f, _, loss = sp.eval_mse(vol, x, yd, schedule=sch, want_dldf=False)
    gc = sp.mse_backward(vol, x, sch)
    f = f.cpu().numpy()
    stored = rounded(dev)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    idx = np.random.default_rng(66).choice(n, 192, replace=False)
    X64 = X.astype(np.float64)
    assert normwise(f[idx], o.eval(stored, X64[idx]), coeffs) <= 1e-5
    assert normwise(f[idx], o.eval(coeffs, X64[idx]), coeffs) <= 2e-3
    # sites and the queries in their supports
    lo = int(np.ceil(cfg.lo / cfg.D)) + 1
    hi = int(np.floor(cfg.hi / cfg.D)) - 1
    pick = interior_sites(cfg, 24, lo, hi, seed=67)
    half = 0.5 * np.abs(cfg.Xi).sum(axis=1)
    near = np.zeros(n, dtype=bool)
    for k, ii in pick:
        m = cfg.D * np.asarray(ii, dtype=float) + np.asarray(cfg.shifts[k], dtype=float)
        near |= np.all(np.abs(X64 - m) <= half, axis=1)
    qn = np.nonzero(near)[0]
    fw = o.eval(stored, X64[qn])
    g = np.zeros(n)
    g[qn] = 2.0 * (fw - y[qn].astype(np.float64)) / n
    want = o.adjoint_at(X64, g, pick)
    b_abs = float(np.max(o.adjoint_at(X64, np.abs(g), pick)))
    b_one = float(np.max(o.adjoint_at(X64, np.where(near, 1.0, 0.0), pick)))
    cmax = max(float(np.max(np.abs(c))) for c in coeffs)
    tol = 1e-5 * b_abs + (2.0 / n) * 1e-5 * cmax * b_one
    got = np.array([float(gc[k][tuple(reversed(ii))]) for k, ii in pick])
    err = float(np.max(np.abs(got - want)))
    print(f"c5 bf16 full-size fused backward at {len(pick)} sites ({len(qn)} queries): err {err:.2e} "
          f"(tol {tol:.2e})", flush=True)
    assert err <= tol
    r = f.astype(np.float64) - y.astype(np.float64)
    assert abs(float(loss.item()) - float(np.mean(r * r))) <= 1e-5 * float(np.mean(r * r))
