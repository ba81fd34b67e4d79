"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Sizes span several 256-query blocks with a ragged tail; queries include
interior points, points on lattice sites and mesh planes, and points whose
support leaves the stored arrays (zero extension).  Tolerances (normwise,
relative to max |c|): FP32 1e-5, FP64 accumulation 1e-11, BF16 storage
2e-3 against the unrounded coefficients and 1e-5 against the rounded ones.
"""

import math

import numpy as np
import pytest

from oracle import ConvolutionSumOracle
from workloads import configs as W
from workloads import inputs as I

pytestmark = pytest.mark.gpu

from gpu_cases import NQ, SMALL, normwise, small_case, tile_pixels, to_dev

TABLE1 = ["cc_tp2", "cc_tp3", "cc_tp4", "cc_linear_rd", "bcc_quintic_rd"]
C0_SPLINES = ("c1", "cc_tp2", "cc_linear_rd")   # linear pieces


def _torch():
    import torch
    return torch


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5", "d4"] + TABLE1)
def test_forward_fp32(lsp, name):
    torch = _torch()
    cfg, coeffs, X = small_case(name)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    want = o.eval(coeffs, X.astype(np.float64))
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    c32 = [c.astype(np.float32).astype(np.float64) for c in coeffs]
    want32 = o.eval(c32, X.astype(np.float64))
    f = sp.eval(vol, torch.from_numpy(X).cuda()).cpu().numpy()
    print(name, "fp32 normwise err", normwise(f, want32, coeffs), flush=True)
    assert normwise(f, want32, coeffs) <= 1e-5
    assert normwise(f, want, coeffs) <= 1e-5


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5", "d4"] + TABLE1)
def test_forward_fp64_check(lsp, name):
    torch = _torch()
    cfg, coeffs, X = small_case(name, seed=1)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    want = o.eval(coeffs, X.astype(np.float64))
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float64))
    f = sp.eval(vol, torch.from_numpy(X).cuda())
    assert f.dtype == torch.float64
    err = normwise(f.cpu().numpy(), want, coeffs)
    print(name, "fp64 normwise err", err, flush=True)
    assert err <= 1e-11


def test_c1_full_workload_fp64(lsp):
    """c1 in full (2 x 32^3 FP64 coefficients, 10^5 queries), in given order
    and through the schedule, every query against the oracle."""
    torch = _torch()
    cfg = W.get("c1")
    coeffs = I.coefficients(cfg)
    X = I.queries(cfg)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    want = o.eval([c.astype(np.float64) for c in coeffs], X.astype(np.float64))
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float64))
    x = torch.from_numpy(X).cuda()
    for sch in (None, sp.schedule(vol, x)):
        f = sp.eval(vol, x, schedule=sch)
        assert f.dtype == torch.float64
        assert normwise(f.cpu().numpy(), want, coeffs) <= 1e-11


@pytest.mark.parametrize("name,dt", [("c2", "bf16"), ("c3", "bf16"), ("c5", "bf16"), ("c3", "f16")])
def test_forward_low_precision_storage(lsp, name, dt):
    torch = _torch()
    tdt = {"bf16": torch.bfloat16, "f16": torch.float16}[dt]
    cfg, coeffs, X = small_case(name, seed=2)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    dev = to_dev(coeffs, tdt)              # round-to-nearest-even conversion
    rounded = [d.float().cpu().numpy().astype(np.float64) for d in dev]
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(dev)
    f = sp.eval(vol, torch.from_numpy(X).cuda()).cpu().numpy()
    assert normwise(f, o.eval(coeffs, X.astype(np.float64)), coeffs) <= 2e-3
    assert normwise(f, o.eval(rounded, X.astype(np.float64)), coeffs) <= 1e-5


@pytest.mark.parametrize("name", ["c2", "c3", "c4", "c5", "d4", "cc_tp3", "cc_tp4", "bcc_quintic_rd"])
def test_gradient(lsp, name):
    torch = _torch()
    cfg, coeffs, X = small_case(name, seed=3)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    _, gw = o.eval(coeffs, X.astype(np.float64), want_grad=True)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    f, g = sp.eval(vol, torch.from_numpy(X).cuda(), grad=True)
    err = normwise(g.cpu().numpy(), gw, coeffs)
    print(name, "grad normwise err", err, flush=True)
    assert err <= 1e-4


@pytest.mark.parametrize("name", ["c1", "c2", "c4", "c5", "d4"] + TABLE1)
def test_adjoint(lsp, name):
    torch = _torch()
    cfg, coeffs, X = small_case(name, seed=4)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    rng = np.random.default_rng(5)
    g = rng.normal(size=len(X)).astype(np.float32)
    want = o.adjoint(X.astype(np.float64), g.astype(np.float64), SMALL[name])
    bound = max(float(np.max(a)) for a in o.adjoint(X.astype(np.float64), np.abs(g).astype(np.float64),
                                                      SMALL[name]))
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    gc, gx = sp.adjoint(vol, torch.from_numpy(X).cuda(), torch.from_numpy(g).cuda(), grad_x=True)
    for a, b in zip(gc, want):
        assert float(np.max(np.abs(a.cpu().numpy() - b))) <= 1e-5 * bound
    if name not in C0_SPLINES:   # only C0: the gradient is two-valued on the mesh planes
        _, gw = o.eval(coeffs, X.astype(np.float64), want_grad=True)
        assert normwise(gx.cpu().numpy(), g[:, None] * gw, coeffs) <= 1e-4 * max(1.0, float(np.max(np.abs(g))))


@pytest.mark.parametrize("name", ["c4", "c5", "d4"])
def test_mse_head(lsp, name):
    torch = _torch()
    cfg, coeffs, X = small_case(name, seed=6)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    y = I.targets(cfg, X)
    c32 = [c.astype(np.float32).astype(np.float64) for c in coeffs]
    want = o.eval(c32, X.astype(np.float64))
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    n = len(X)
    r = want - y
    _, gw = o.eval(c32, X.astype(np.float64), want_grad=True)
    for sch in (None, sp.schedule(vol, xd)):
        f, dldf, loss, dldx = sp.eval_mse(vol, xd, yd, schedule=sch, grad_x=True)
        assert normwise(f.cpu().numpy(), want, coeffs) <= 1e-5
        np.testing.assert_allclose(dldf.cpu().numpy(), 2 * r / n, atol=2e-5 / n * 4)
        assert abs(float(loss.item()) - float(np.mean(r * r))) <= 1e-5 * max(1.0, float(np.mean(r * r)))
        # dL/dx = dL/df * grad f
        np.testing.assert_allclose(dldx.cpu().numpy(), (2 * r / n)[:, None] * gw, atol=1e-4 * 2 / n * 4)
        # without storing f: the same loss and gradients
        f2, dldf2, loss2, dldx2 = sp.eval_mse(vol, xd, yd, schedule=sch, grad_x=True, want_f=False)
        assert f2 is None
        assert torch.equal(dldf2, dldf) and torch.equal(dldx2, dldx)
        assert abs(float(loss2.item()) - float(loss.item())) <= 1e-12 * max(1.0, abs(float(loss.item())))


def test_autograd_backward_matches_adjoint(lsp):
    torch = _torch()
    cfg, coeffs, X = small_case("c4", seed=7)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    cs = [t.requires_grad_(True) for t in to_dev(coeffs, torch.float32)]
    x = torch.from_numpy(X).cuda().requires_grad_(True)
    f = lsp.lattice_spline(sp, x, cs)
    y = torch.from_numpy(I.targets(cfg, X)).cuda()
    loss = ((f - y) ** 2).mean()
    loss.backward()
    g = (2.0 * (f.detach() - y) / len(X)).double().cpu().numpy()
    want = o.adjoint(X.astype(np.float64), g, SMALL["c4"])
    bound = max(float(np.max(a)) for a in o.adjoint(X.astype(np.float64), np.abs(g), SMALL["c4"]))
    for c, w in zip(cs, want):
        assert float(np.max(np.abs(c.grad.cpu().numpy() - w))) <= 1e-5 * bound + 1e-9


def test_rays_against_oracle(lsp):
    torch = _torch()
    cfg = W.get("c3")
    dims = (16, 16, 16)
    rng = np.random.default_rng(8)
    coeffs = [rng.uniform(-1, 1, tuple(reversed(dims))) for _ in range(2)]
    centre = np.full(3, 15.5)
    a = 11.0 / np.sqrt(3.0)
    cz, sz = math.cos(math.radians(30.0)), math.sin(math.radians(30.0))
    cx, sx = math.cos(math.radians(20.0)), math.sin(math.radians(20.0))
    R = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]]) @ np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    A = (R * a).astype(np.float32)
    Wd, H, S = 16, 8, 37
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    ray0, nrays = 5, 100
    out, smp = sp.rays(vol, centre.astype(np.float32), A, Wd, H, S, ray0=ray0, nrays=nrays, samples=True)
    rays = np.arange(ray0, ray0 + nrays)
    pix = tile_pixels(rays, Wd)
    # the same float32 sample positions, computed independently on the CPU
    c32, A32 = centre.astype(np.float32), A
    u = (pix % Wd).astype(np.float32)
    v = (pix // Wd).astype(np.float32)
    j = np.arange(S, dtype=np.float32)
    tu = (np.float32(2) * (u + np.float32(0.5))) / np.float32(Wd) - np.float32(1)
    tv = (np.float32(2) * (v + np.float32(0.5))) / np.float32(H) - np.float32(1)
    tj = (np.float32(2) * (j + np.float32(0.5))) / np.float32(S) - np.float32(1)
    P = np.empty((nrays, S, 3), dtype=np.float32)
    for ax in range(3):
        base = (c32[ax] + A32[ax, 0] * tu) + A32[ax, 1] * tv
        P[:, :, ax] = base[:, None] + A32[ax, 2] * tj[None, :]
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    fw, gw = o.eval([c.astype(np.float32).astype(np.float64) for c in coeffs],
                    P.reshape(-1, 3).astype(np.float64), want_grad=True)
    smp = smp.cpu().numpy().reshape(-1, 4)
    assert normwise(smp[:, 0], fw, coeffs) <= 1e-5
    assert normwise(smp[:, 1:], gw, coeffs) <= 1e-4
    out = out.cpu().numpy()
    np.testing.assert_allclose(out[:, 0], fw.reshape(nrays, S).sum(1), atol=S * 1e-5)
    np.testing.assert_allclose(out[:, 1:], gw.reshape(nrays, S, 3).sum(1), atol=S * 1e-4)


def test_rays_full_size_sampled_c3(lsp):
    """c3's full launch (2 x 192^3, 1024 x 1024 rays, 512 steps, forward and
    gradient summed per ray), checked on sampled rays: every sample of those
    rays is evaluated by the oracle at the same float32 positions."""
    torch = _torch()
    cfg = W.get("c3")
    coeffs = I.coefficients(cfg)
    Wd, Hd = cfg.extra["rays"]
    S = cfg.extra["steps"]
    c, A = I.ray_params(cfg)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    out = sp.rays(vol, c.astype(np.float32), A.astype(np.float32), Wd, Hd, S).cpu().numpy()
    assert out.shape == (Wd * Hd, 4) and np.all(np.isfinite(out))
    rays = np.concatenate([[0, Wd * Hd - 1], np.random.default_rng(43).choice(Wd * Hd, 4, replace=False)])
    P = I.ray_samples(cfg, tile_pixels(rays, Wd)[:, None], np.arange(S)[None, :], W=Wd, H=Hd, S=S)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    fw, gw = o.eval([a.astype(np.float32).astype(np.float64) for a in coeffs], P.reshape(-1, 3).astype(np.float64),
                    want_grad=True)
    cmax = max(float(np.abs(a).max()) for a in coeffs)
    np.testing.assert_allclose(out[rays, 0], fw.reshape(len(rays), S).sum(1), rtol=0, atol=S * 1e-5 * cmax)
    np.testing.assert_allclose(out[rays, 1:], gw.reshape(len(rays), S, 3).sum(1), rtol=0, atol=S * 1e-4 * cmax)


def test_edge_cases(lsp):
    torch = _torch()
    cfg, coeffs, X = small_case("c2", n=300, seed=9)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    # empty batch
    f = sp.eval(vol, torch.empty(0, 3, device="cuda"))
    assert f.numel() == 0
    # non-finite queries give NaN and do not fault
    bad = torch.tensor([[float("nan"), 3.0, 3.0], [float("inf"), 3.0, 3.0], [-float("inf"), 1e30, 3.0],
                        [5.0, 5.0, 5.0]], device="cuda")
    fb = sp.eval(vol, bad).cpu().numpy()
    assert np.isnan(fb[0]) and not np.isnan(fb[3])
    # far outside the volume: zero
    far = torch.tensor([[-100.0, -100.0, -100.0], [1e6, 1e6, 1e6]], device="cuda")
    assert np.all(sp.eval(vol, far).cpu().numpy() == 0)
    # constant data reproduces the constant in the interior (partition of unity)
    ones = [torch.ones_like(c) for c in vol.coeffs]
    v1 = sp.bind(ones)
    Xi = torch.from_numpy(np.random.default_rng(1).uniform(4, 15, (777, 3)).astype(np.float32)).cuda()
    assert float((sp.eval(v1, Xi) - 1).abs().max()) < 2e-6


def test_full_size_sampled_c2(lsp):
    """The benchmark's workload (256^3 volume, 2^24 queries, same launch),
    checked on a sample of outputs against the oracle."""
    torch = _torch()
    cfg = W.get("c2")
    coeffs = I.coefficients(cfg)
    X = I.queries(cfg)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    f = sp.eval(vol, torch.from_numpy(X).cuda()).cpu().numpy()
    idx = np.random.default_rng(10).choice(len(X), 2048, replace=False)
    idx = np.concatenate([idx, [0, len(X) - 1]])
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    want = o.eval([c.astype(np.float64) for c in coeffs], X[idx].astype(np.float64))
    assert normwise(f[idx], want, coeffs) <= 1e-5
    assert np.all(np.isfinite(f))
    # the benchmark's sorted launch: same arithmetic per query (one sub-region), so the same bits
    x = torch.from_numpy(X).cuda()
    sch = sp.schedule(vol, x)
    fs = sp.eval(vol, x, schedule=sch).cpu().numpy()
    assert np.array_equal(fs, f)
    # BF16 storage (the benchmark's --dtype bf16 line) against the oracle on the rounded coefficients
    dev = to_dev(coeffs, torch.bfloat16)
    rounded = [d.float().cpu().numpy().astype(np.float64) for d in dev]
    fb = sp.eval(sp.bind(dev), x, schedule=sch).cpu().numpy()
    assert normwise(fb[idx], o.eval(rounded, X[idx].astype(np.float64)), coeffs) <= 1e-5


def test_mse_step_full_size_c4(lsp):
    """The benchmark's c4 training step at full size (4 x 128^3, 2^22 queries):
    scheduled MSE forward storing neither f nor dL/df, then the fused
    backward.  The loss matches the one computed from f in FP64, sampled f
    matches the oracle, dL/dx matches the gradient path, and dL/dc matches
    the given-order adjoint fed dL/df = 2 (f - y) / n."""
    torch = _torch()
    cfg = W.get("c4")
    coeffs = I.coefficients(cfg)
    X = I.queries(cfg)
    n = len(X)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    dev = to_dev(coeffs, torch.float32)
    vol = sp.bind(dev)
    x = torch.from_numpy(X).cuda()
    y = torch.from_numpy(I.targets(cfg, X)).cuda()
    sch = sp.schedule(vol, x)
    f_none, d_none, loss, dldx = sp.eval_mse(vol, x, y, schedule=sch, grad_x=True, want_f=False,
                                             want_dldf=False)
    assert f_none is None and d_none is None
    gc = sp.mse_backward(vol, x, sch)
    f, gf = sp.eval(vol, x, grad=True)
    r = f.double() - y.double()
    want_loss = float((r * r).mean())
    assert abs(float(loss.item()) - want_loss) <= 1e-5 * want_loss
    idx = np.random.default_rng(42).choice(n, 256, replace=False)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    want = o.eval([c.astype(np.float64) for c in coeffs], X[idx].astype(np.float64))
    assert normwise(f.cpu().numpy()[idx], want, coeffs) <= 1e-5
    want_dx = (2.0 / n) * r[:, None] * gf.double()
    assert float((dldx.double() - want_dx).abs().max()) <= 1e-5 * float(want_dx.abs().max())
    g = (2.0 / n * r).float()
    ga, _ = sp.adjoint(vol, x, g)
    for a, b in zip(gc, ga):
        assert float((a - b).abs().max()) <= 1e-5 * float(b.abs().max())


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5", "d4"] + TABLE1)
def test_scheduled_order(lsp, name):
    """The counting-sort schedule changes only the evaluation order: results
    equal the given-order ones (bitwise for one sub-region; up to the order of
    the per-coset float additions otherwise) and the oracle."""
    torch = _torch()
    cfg, coeffs, X = small_case(name, n=2503 if NQ[name] >= 1301 else NQ[name], seed=12)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    x = torch.from_numpy(X).cuda()
    grad = name != "c1"
    r0 = sp.eval(vol, x, grad=grad)
    sch = sp.schedule(vol, x)
    r1 = sp.eval(vol, x, grad=grad, schedule=sch)
    f0, f1 = (r0[0], r1[0]) if grad else (r0, r1)
    split = sp.info["n_subregions"] > 1
    if split:
        assert normwise(f1.cpu().numpy(), f0.cpu().numpy(), coeffs) <= 1e-6
    else:
        assert torch.equal(f0, f1)
    if grad:
        assert normwise(r1[1].cpu().numpy(), r0[1].cpu().numpy(), coeffs) <= 1e-6
    c32 = [c.astype(np.float32).astype(np.float64) for c in coeffs]
    assert normwise(f1.cpu().numpy(), o.eval(c32, X.astype(np.float64)), coeffs) <= 1e-5
    # adjoint through the same schedule
    g = torch.from_numpy(np.random.default_rng(13).normal(size=len(X)).astype(np.float32)).cuda()
    ga, gxa = sp.adjoint(vol, x, g, grad_x=True)
    gb, gxb = sp.adjoint(vol, x, g, grad_x=True, schedule=sch)
    for a, b in zip(ga, gb):
        assert float((a - b).abs().max()) <= 1e-5 * max(1.0, float(a.abs().max()))
    assert float((gxa - gxb).abs().max()) <= 1e-5 * max(1.0, float(gxa.abs().max()))
    # MSE head through the schedule
    if cfg.s == 3 or name == "c5":
        y = torch.from_numpy(I.targets(cfg, X)).cuda()
        fa, da, la = sp.eval_mse(vol, x, y)
        fb, db, lb = sp.eval_mse(vol, x, y, schedule=sch)
        assert float((fa - fb).abs().max()) <= 1e-6
        assert float((da - db).abs().max()) <= 1e-9
        assert abs(float(la) - float(lb)) <= 1e-6 * max(1.0, abs(float(la)))


@pytest.mark.parametrize("name,samples", [("c5", 512), ("d4", 128)])
def test_scheduled_full_size_sampled(lsp, name, samples):
    """c5 (2 x 48^4) and the D4 spline of Sec. 5.2 (8 x 24^4), 2^22 queries
    each, through the schedule (the benchmark's launch), on sampled outputs
    against the oracle; the adjoint's total mass is checked against the
    forward by the adjoint identity <A c, g> = <c, A^T g>."""
    torch = _torch()
    cfg = W.get(name)
    coeffs = I.coefficients(cfg)
    X = I.queries(cfg)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    dev = to_dev(coeffs, torch.float32)
    vol = sp.bind(dev)
    x = torch.from_numpy(X).cuda()
    sch = sp.schedule(vol, x)
    f = sp.eval(vol, x, schedule=sch)
    idx = np.random.default_rng(14).choice(len(X), samples, replace=False)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    want = o.eval([c.astype(np.float64) for c in coeffs], X[idx].astype(np.float64))
    assert normwise(f.cpu().numpy()[idx], want, coeffs) <= 1e-5
    g = torch.from_numpy(np.random.default_rng(15).normal(size=len(X)).astype(np.float32)).cuda()
    gc, _ = sp.adjoint(vol, x, g, schedule=sch)
    lhs = float(torch.dot(f.double(), g.double()))
    rhs = float(sum(torch.sum(c.double() * a.double()) for c, a in zip(dev, gc)))
    assert abs(lhs - rhs) <= 1e-4 * (abs(lhs) + float(g.abs().sum()) * 1e-3)


@pytest.mark.parametrize("name", ["c2", "c4", "c5"])
def test_scheduled_adjoint_fixed_point_scaling(lsp, name):
    """The scheduled adjoint accumulates in 64-bit fixed point with a power-of-
    two scale taken from max |g|: scaling g by a power of two scales the
    result exactly (the same integers are summed), for tiny and huge g; its
    sums do not depend on the order of the additions (two runs agree
    bitwise); a non-finite g turns the result into NaN."""
    torch = _torch()
    n = 1301 if cfg_s(name) == 3 else 601
    cfg, coeffs, X = small_case(name, n=n, seed=21)
    X = np.ascontiguousarray(X[: n // 2])      # interior queries: every item is accumulated in LDS
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    x = torch.from_numpy(X).cuda()
    sch = sp.schedule(vol, x)
    g = torch.from_numpy(np.random.default_rng(22).normal(size=len(X)).astype(np.float32)).cuda()
    base, _ = sp.adjoint(vol, x, g, schedule=sch)
    again, _ = sp.adjoint(vol, x, g, schedule=sch)
    for a, b in zip(base, again):
        assert torch.equal(a, b)
    for e in (-60, 60):
        scaled, _ = sp.adjoint(vol, x, torch.ldexp(g, torch.tensor(e, device="cuda")), schedule=sch)
        for a, b in zip(base, scaled):
            assert torch.equal(torch.ldexp(a, torch.tensor(e, device="cuda")), b)
    gn = g.clone()
    gn[7] = float("nan")
    bad, _ = sp.adjoint(vol, x, gn, schedule=sch)
    assert any(bool(torch.isnan(a).any()) for a in bad)


def cfg_s(name):
    return W.get(name).s


@pytest.mark.parametrize("name,n", [("c4", 200000), ("d4", 70000)])
def test_scheduled_several_groups_per_unit(lsp, name, n):
    """Few units with many items each: the evaluation splits every unit over
    several workgroups; results match the given-order path (and the MSE head
    its loss)."""
    torch = _torch()
    cfg = W.get(name)
    dims = SMALL[name]
    rng = np.random.default_rng(40)
    coeffs = [rng.uniform(-1, 1, tuple(reversed(dims))) for _ in range(cfg.M)]
    ext = cfg.D * (dims[0] - 1) + 1
    X = rng.uniform(2.0, ext - 3.0, (n, cfg.s)).astype(np.float32)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    x = torch.from_numpy(X).cuda()
    f0, g0 = sp.eval(vol, x, grad=True)
    sch = sp.schedule(vol, x)
    f1, g1 = sp.eval(vol, x, grad=True, schedule=sch)
    assert normwise(f1.cpu().numpy(), f0.cpu().numpy(), coeffs) <= 1e-6
    assert normwise(g1.cpu().numpy(), g0.cpu().numpy(), coeffs) <= 1e-5
    y = torch.from_numpy(I.targets(cfg, X)).cuda()
    _, da, la = sp.eval_mse(vol, x, y)
    _, db, lb = sp.eval_mse(vol, x, y, schedule=sch)
    assert float((da - db).abs().max()) <= 1e-9
    assert abs(float(la) - float(lb)) <= 1e-6 * max(1.0, abs(float(la)))


@pytest.mark.parametrize("name", ["c4", "c5"])
def test_scheduled_edge_cases(lsp, name):
    """Empty batches through every scheduled entry point; queries far outside
    the volume or not finite through the schedule give what the given-order
    path gives (zero outside, NaN for NaN, no fault)."""
    torch = _torch()
    cfg, coeffs, X = small_case(name, n=301, seed=30)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    s = cfg.s
    # empty batch
    e = torch.empty(0, s, device="cuda")
    sch0 = sp.schedule(vol, e)
    assert sp.eval(vol, e, schedule=sch0).numel() == 0
    gc, _ = sp.adjoint(vol, e, torch.empty(0, device="cuda"), schedule=sch0)
    assert all(float(a.abs().max()) == 0.0 for a in gc)
    # far outside, non-finite and ordinary queries mixed
    odd = np.array([[-500.0] * s, [1e7] * s, [np.nan] + [5.0] * (s - 1), [np.inf] + [5.0] * (s - 1)],
                   dtype=np.float32)
    Xm = np.concatenate([X, odd]).astype(np.float32)
    x = torch.from_numpy(Xm).cuda()
    f0 = sp.eval(vol, x).cpu().numpy()
    f1 = sp.eval(vol, x, schedule=sp.schedule(vol, x)).cpu().numpy()
    assert np.array_equal(np.isnan(f0), np.isnan(f1))
    ok = ~np.isnan(f0)
    assert np.max(np.abs(f0[ok] - f1[ok])) <= 1e-6
    assert f1[len(X)] == 0.0 and f1[len(X) + 1] == 0.0 and np.isnan(f1[len(X) + 2])
    # the scheduled adjoint ignores the non-finite queries (their grad_x is NaN)
    g = torch.from_numpy(np.random.default_rng(31).normal(size=len(Xm)).astype(np.float32)).cuda()
    gm, gxm = sp.adjoint(vol, x, g, grad_x=True, schedule=sp.schedule(vol, x))
    xf = torch.from_numpy(np.ascontiguousarray(Xm[: len(X) + 2])).cuda()
    gf, gxf = sp.adjoint(vol, xf, g[: len(X) + 2].contiguous(), grad_x=True, schedule=sp.schedule(vol, xf))
    for a, b in zip(gm, gf):
        assert float((a - b).abs().max()) <= 1e-6 * max(1.0, float(b.abs().max()))
    assert bool(torch.isnan(gxm[len(X) + 2:]).all())
    assert float((gxm[: len(X) + 2] - gxf).abs().max()) <= 1e-6 * max(1.0, float(gxf.abs().max()))


@pytest.mark.parametrize("name", ["c2", "c4"])
def test_outlier_key_at_scale(lsp, name):
    """2^20 queries on the full volume, a third of them pushed up to four
    cells past a face (some still reaching it with their stencil, some not):
    those lie outside the brick grid and take the schedule's outlier key and
    kernels.  The scheduled forward matches the given-order one (the same
    arithmetic per query), sampled outliers and interior queries match the
    oracle, and for c4 the scheduled MSE step and fused backward match the
    given-order MSE head and adjoint."""
    torch = _torch()
    cfg = W.get(name)
    coeffs = I.coefficients(cfg)
    rng = np.random.default_rng(77)
    n = 1 << 20
    ext = cfg.D * (cfg.dims[0] - 1) + 1
    X = rng.uniform(0.0, ext, (n, cfg.s))
    out = np.nonzero(rng.random(n) < 1.0 / 3.0)[0]
    ax = rng.integers(0, cfg.s, len(out))
    d = rng.uniform(0.0, 4.0 * cfg.D, len(out))
    X[out, ax] = np.where(rng.random(len(out)) < 0.5, -d, ext + d)
    X = X.astype(np.float32)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    x = torch.from_numpy(X).cuda()
    sch = sp.schedule(vol, x)
    f0 = sp.eval(vol, x).cpu().numpy()
    f1 = sp.eval(vol, x, schedule=sch).cpu().numpy()
    assert np.all(np.isfinite(f1))
    print(name, "scheduled vs given order", float(np.max(np.abs(f1 - f0))), flush=True)
    assert normwise(f1, f0.astype(np.float64), coeffs) <= 1e-6
    idx = np.concatenate([rng.choice(out, 64, replace=False), rng.choice(n, 64, replace=False)])
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    want = o.eval([c.astype(np.float64) for c in coeffs], X[idx].astype(np.float64))
    assert normwise(f1[idx], want, coeffs) <= 1e-5
    if name != "c4":
        return
    y = torch.from_numpy(I.targets(cfg, X)).cuda()
    _, dl0, l0, dx0 = sp.eval_mse(vol, x, y, grad_x=True)
    _, dl1, l1, dx1 = sp.eval_mse(vol, x, y, schedule=sch, grad_x=True)
    assert abs(float(l1) - float(l0)) <= 1e-6 * abs(float(l0))
    assert float((dl1 - dl0).abs().max()) <= 1e-6 * float(dl0.abs().max())
    assert float((dx1 - dx0).abs().max()) <= 1e-5 * float(dx0.abs().max())
    gc = sp.mse_backward(vol, x, sch)
    ga, _ = sp.adjoint(vol, x, dl0)
    for a, b in zip(gc, ga):
        assert float((a - b).abs().max()) <= 1e-5 * float(b.abs().max())


@pytest.mark.parametrize("name", ["c4", "c5", "d4"])
def test_mse_backward_fused(lsp, name):
    """The fused MSE backward (dL/df kept in the workspace by the scheduled
    forward) equals the scheduled adjoint fed the returned dL/df, also when
    the forward stores neither f nor dL/df."""
    torch = _torch()
    cfg, coeffs, X = small_case(name, seed=41)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    x = torch.from_numpy(X).cuda()
    y = torch.from_numpy(I.targets(cfg, X)).cuda()
    sch = sp.schedule(vol, x)
    _, dldf, loss = sp.eval_mse(vol, x, y, schedule=sch)
    want, _ = sp.adjoint(vol, x, dldf, schedule=sch)
    got = sp.mse_backward(vol, x, sch)
    for a, b in zip(got, want):
        assert float((a - b).abs().max()) <= 1e-6 * max(1e-12, float(b.abs().max()))
    f2, d2, loss2, dx2 = sp.eval_mse(vol, x, y, schedule=sch, grad_x=True, want_f=False, want_dldf=False)
    assert f2 is None and d2 is None
    assert abs(float(loss2.item()) - float(loss.item())) <= 1e-12 * max(1.0, abs(float(loss.item())))
    got2 = sp.mse_backward(vol, x, sch)
    for a, b in zip(got2, want):
        assert float((a - b).abs().max()) <= 1e-6 * max(1e-12, float(b.abs().max()))
