"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every symbol the header declares, matches plans and rejects bad arguments."""

import ctypes
import os
import re

import pytest

from workloads import configs as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2102_08514_amd import _lib as L
    return L


def header_functions():
    txt = open(os.path.join(ROOT, "include", "lsp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:lsp_status|const char\*)\s+(lsp_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = L.lib()
    names = header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
def test_plan_matches_configs(name):
    L = _lib()
    cfg = W.get(name)
    p = L.lsp_plan_create(cfg.L, cfg.Xi)
    info = L.lsp_plan_info(p)
    assert info["lookups"] == cfg.lookups
    assert info["n_cosets"] == cfg.M and info["D"] == cfg.D
    assert [tuple(v) for v in info["shifts"]] == [tuple(v) for v in cfg.shifts]
    L.lsp_plan_destroy(p)


def test_plan_accepts_equivalent_inputs():
    L = _lib()
    # another basis of the BCC lattice and a permuted, sign-flipped Xi
    Lb = [[2, 0, 1], [0, 2, 1], [0, 0, 1]]
    Xi = (-W.XI_BCC_QUARTIC[:, ::-1]).tolist()
    p = L.lsp_plan_create(Lb, Xi)
    assert L.lsp_plan_info(p)["name"] == "bcc_quartic"
    L.lsp_plan_destroy(p)


def test_plan_errors():
    L = _lib()
    with pytest.raises(L.LspError) as e:
        L.lsp_plan_create(W.L_CC, [[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 1]])   # valid but no tables
    assert e.value.status == -3
    with pytest.raises(L.LspError) as e:
        L.lsp_plan_create(W.L_FCC, W.XI_ZP)                  # e1 is not an FCC vector
    assert e.value.status == -7
    with pytest.raises(L.LspError) as e:
        L.lsp_plan_create([[1, 0, 0], [0, 1, 0], [0, 0, 0]], W.XI_ZP)   # singular lattice
    assert e.value.status == -2
    with pytest.raises(L.LspError) as e:
        L.lsp_plan_create(W.L_CC, [[1, 0], [0, 1], [0, 0]])             # n < s
    assert e.value.status == -2
    with pytest.raises(L.LspError) as e:
        L.lsp_plan_create(W.L_CC, [[1, 1, 0, 0], [0, 0, 1, 1], [0, 0, 0, 0]])   # rank 2
    assert e.value.status == -2
    lib = L.lib()
    assert lib.lsp_plan_create(3, None, 4, None, 0, None) == -1
    assert lib.lsp_plan_destroy(None) == -1
    assert L.status_string(-3).startswith("no generated tables")


def test_bind_and_eval_argument_errors():
    L = _lib()
    cfg = W.get("c4")
    p = L.lsp_plan_create(cfg.L, cfg.Xi)
    fake = [0x1000 * (k + 1) for k in range(4)]   # never dereferenced by these calls
    with pytest.raises(L.LspError) as e:
        L.lsp_vol_bind(p, 9, fake, (8, 8, 8))
    assert e.value.status == -4
    with pytest.raises(L.LspError) as e:
        L.lsp_vol_bind(p, 0, fake, (8, 0, 8))
    assert e.value.status == -5
    with pytest.raises(L.LspError) as e:
        L.lsp_vol_bind(p, 0, fake, (2048, 2048, 1024))
    assert e.value.status == -5
    with pytest.raises(L.LspError) as e:
        L.lsp_vol_bind(p, 0, fake[:3] + [0], (8, 8, 8))
    assert e.value.status == -1
    v = L.lsp_vol_bind(p, 0, fake, (8, 8, 8))
    lib = L.lib()
    # empty batches succeed without touching the GPU; bad pointers and sizes fail
    assert lib.lsp_eval(p, v, None, 0, None, None, None) == 0
    assert lib.lsp_eval(p, v, None, 5, None, None, None) == -1
    assert lib.lsp_eval(p, v, 0x1000, -1, 0x1000, None, None) == -2
    assert lib.lsp_eval_adjoint(p, v, None, None, 0, None, None, None) == 0
    assert lib.lsp_eval_adjoint(p, v, 0x1000, 0x1000, 4, None, None, None) == -1
    cc = (ctypes.c_float * 3)(0, 0, 0)
    AA = (ctypes.c_float * 9)(*([0.0] * 9))
    assert lib.lsp_eval_rays(p, v, cc, AA, 12, 8, 4, 0, 1, 0x1000, None, None) == -2   # W not a multiple of 8
    # plan / volume mismatch
    q = L.lsp_plan_create(W.get("c2").L, W.get("c2").Xi)
    assert lib.lsp_eval(q, v, 0x1000, 4, 0x1000, None, None) == -2
    L.lsp_vol_release(v)
    L.lsp_plan_destroy(p)
    L.lsp_plan_destroy(q)


def test_schedule_workspace_checks():
    L = _lib()
    cfg = W.get("c5")
    p = L.lsp_plan_create(cfg.L, cfg.Xi)
    v = L.lsp_vol_bind(p, 0, [0x1000, 0x2000], (48, 48, 48, 48))
    need = L.lsp_schedule_size(p, v, 1 << 22)
    # items = queries x cosets for a spline with several sub-regions: 3 x 4 B each at least
    assert need >= 12 * 2 * (1 << 22)
    lib = L.lib()
    assert lib.lsp_schedule(p, v, 0x1000, 1 << 22, 0x100000, need - 1, None) == -2      # too small
    assert lib.lsp_schedule(p, v, 0x1000, 1 << 22, 0x100010, need, None) == -2          # misaligned
    assert lib.lsp_schedule(p, v, 0x1000, 1 << 22, None, need, None) == -1
    assert lib.lsp_eval_scheduled(p, v, 0x1000, 1 << 22, 0x100000, need - 1, 0x1000, None, None) == -2
    assert lib.lsp_schedule(p, v, None, 0, 0x100000, L.lsp_schedule_size(p, v, 0), None) == 0   # empty batch
    with pytest.raises(L.LspError):
        L.lsp_schedule_size(p, v, 1 << 31)          # items would overflow 32 bits
    L.lsp_vol_release(v)
    L.lsp_plan_destroy(p)


def test_no_fallback_without_the_library(monkeypatch, tmp_path):
    """The product path raises when the HIP library is absent; nothing falls
    back to a CPU evaluation."""
    L = _lib()
    from paper_2102_08514_amd import api
    cfg = W.get("c2")
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "liblsp.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        api.LatticeSpline(cfg.L, cfg.Xi)


def test_host_tensors_are_rejected():
    """Coefficients and queries must be device tensors: the API never
    evaluates host memory."""
    import torch
    from paper_2102_08514_amd import api
    cfg = W.get("c2")
    sp = api.LatticeSpline(cfg.L, cfg.Xi)
    with pytest.raises(ValueError, match="GPU"):
        sp.bind([torch.zeros(8, 8, 8)])
