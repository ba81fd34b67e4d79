"""The allocation-free entry point (lsp_eval_scheduled_static) against the
workspace path (lsp_schedule + lsp_eval_scheduled) it shares its kernels
with, through the C ABI: two calls in a row, the second with fewer queries
(the static scratch keeps the first call's schedule), with and without the
gradient, and the size limit."""

import ctypes

import numpy as np
import pytest
import torch

from gpu_cases import normwise, to_dev
from oracle import ConvolutionSumOracle
from workloads import configs as W
from workloads import inputs as I

pytestmark = pytest.mark.gpu


def _static(L, sp, vol, x, grad):
    n = x.shape[0]
    f = torch.empty(n, device="cuda", dtype=torch.float32)
    g = torch.empty(n, 3, device="cuda", dtype=torch.float32) if grad else None
    L.lsp_eval_scheduled_static(sp.plan, vol.handle, x.data_ptr(), n, f.data_ptr(),
                                g.data_ptr() if grad else None, torch.cuda.current_stream().cuda_stream)
    return f, g


@pytest.mark.parametrize("name,sizes", [("c4", (300_000, 77_777)), ("c2", (200_003, 4_097))])
def test_static_scratch_matches_workspace_path(lsp, name, sizes):
    from paper_2102_08514_amd import _lib as L
    cfg = W.get(name)
    coeffs = I.coefficients(cfg)
    X = I.queries(cfg)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev(coeffs, torch.float32))
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    for n in sizes:
        for grad in (False, True):
            x = torch.from_numpy(np.ascontiguousarray(X[:n])).cuda()
            print(f"{name}: n={n} grad={grad}", flush=True)
            f, g = _static(L, sp, vol, x, grad)
            sch = sp.schedule(vol, x)
            ref = sp.eval(vol, x, grad=grad, schedule=sch)
            torch.cuda.synchronize()
            if grad:
                ref_f, ref_g = ref
                assert torch.equal(g, ref_g)
            else:
                ref_f = ref
            assert torch.equal(f, ref_f)
            k = 256
            want = o.eval([c.astype(np.float32).astype(np.float64) for c in coeffs], X[:k].astype(np.float64))
            assert normwise(f[:k].cpu().numpy(), want, coeffs) <= 1e-5


def test_static_scratch_size_limit(lsp):
    from paper_2102_08514_amd import _lib as L
    cfg = W.get("c4")
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    vol = sp.bind(to_dev([np.zeros(tuple(reversed(cfg.dims)), dtype=np.float32)] * cfg.M, torch.float32))
    n = 5_000_000          # its 16-byte records alone need 80 MB
    x = torch.zeros(n, 3, device="cuda", dtype=torch.float32)
    f = torch.zeros(n, device="cuda", dtype=torch.float32)
    with pytest.raises(L.LspError) as e:
        L.lsp_eval_scheduled_static(sp.plan, vol.handle, x.data_ptr(), n, f.data_ptr(), None,
                                    torch.cuda.current_stream().cuda_stream)
    assert e.value.status == -8
    assert int(torch.count_nonzero(f)) == 0
