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


@pytest.mark.parametrize("name", ["vor_bcc1", "vor_fcc1", "vor_cc_bcc1", "vor_cc_fcc1", "vor_fcc2", "vor_cc_fcc2"])
def test_voronoi_plan_matches_configs(name):
    L = _lib()
    cfg = W.get(name)
    p = L.lsp_plan_create_voronoi(cfg.L, cfg.Lv, cfg.voronoi[1])
    info = L.lsp_plan_info(p)
    assert info["kind"] == "voronoi" and info["voronoi_n"] == cfg.voronoi[1]
    assert info["lookups"] == cfg.lookups
    assert info["n_cosets"] == cfg.M and info["D"] == cfg.D
    L.lsp_plan_destroy(p)


def test_voronoi_plan_errors_and_equivalent_bases():
    L = _lib()
    # another basis of the BCC lattice, for both L and the cell's lattice
    Lb = [[2, 0, 1], [0, 2, 1], [0, 0, 1]]
    p = L.lsp_plan_create_voronoi(Lb, Lb, 1)
    assert L.lsp_plan_info(p)["name"] == "bcc_voronoi1"
    L.lsp_plan_destroy(p)
    with pytest.raises(L.LspError) as e:
        L.lsp_plan_create_voronoi(W.L_BCC, W.L_CC, 1)        # Z^3 is not inside BCC
    assert e.value.status == -7
    with pytest.raises(L.LspError) as e:
        L.lsp_plan_create_voronoi(W.L_BCC, W.L_BCC, 2)       # BCC V_2: no tables
    assert e.value.status == -3
    with pytest.raises(L.LspError) as e:
        L.lsp_plan_create_voronoi(W.L_CC, [[1, 0, 0], [0, 1, 0], [0, 0, 0]], 1)
    assert e.value.status == -2
    with pytest.raises(L.LspError) as e:
        L.lsp_plan_create_voronoi(W.L_CC, W.L_BCC, 0)
    assert e.value.status == -2
    lib = L.lib()
    assert lib.lsp_plan_create_voronoi(3, None, None, 1, 0, None) == -1
    # the cell's zonotope generators are not a box spline the library ships
    gen2 = [[2 * v for v in col] for col in zip(*W.VORONOI_GEN["BCC"])]
    with pytest.raises(L.LspError) as e:
        L.lsp_plan_create(W.L_BCC, gen2)
    assert e.value.status == -3


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


def test_schedule_is_tied_to_its_volume_and_queries():
    """A workspace serves only the plan, volume dims, dtype class, queries and
    n that lsp_schedule filled it for; the scheduled calls refuse anything
    else (their workspace layout depends on all of these)."""
    L = _lib()
    lib = L.lib()
    cfg = W.get("c4")
    p = L.lsp_plan_create(cfg.L, cfg.Xi)
    fake = [0x1000 * (k + 1) for k in range(4)]
    v = L.lsp_vol_bind(p, 0, fake, (16, 16, 16))
    v_small = L.lsp_vol_bind(p, 0, fake, (8, 8, 8))
    v_wide = L.lsp_vol_bind(p, 3, fake, (16, 16, 16))
    ws = 0x200000
    need = max(L.lsp_schedule_size(p, w, 0) for w in (v, v_small, v_wide))
    # never scheduled: refused
    assert lib.lsp_eval_scheduled(p, v, None, 0, ws + 256, need, 0x1000, None, None) == -2
    # an empty batch is scheduled without touching the GPU
    assert lib.lsp_schedule(p, v, None, 0, ws, need, None) == 0
    assert lib.lsp_eval_scheduled(p, v, None, 0, ws, need, 0x1000, None, None) == 0
    assert lib.lsp_eval_adjoint_scheduled(p, v, None, None, 0, ws, need, None, None, None) == 0
    # other dims, other dtype class, other queries: refused
    assert lib.lsp_eval_scheduled(p, v_small, None, 0, ws, need, 0x1000, None, None) == -2
    assert lib.lsp_eval_scheduled(p, v_wide, None, 0, ws, need, 0x1000, None, None) == -2
    assert lib.lsp_eval_scheduled(p, v, 0x4000, 0, ws, need, 0x1000, None, None) == -2
    # the same dims in another binding of the same plan and dtype class is fine
    v2 = L.lsp_vol_bind(p, 1, fake, (16, 16, 16))
    assert lib.lsp_eval_scheduled(p, v2, None, 0, ws, need, 0x1000, None, None) == 0
    for h in (v, v_small, v_wide, v2):
        L.lsp_vol_release(h)
    L.lsp_plan_destroy(p)


def test_query_count_limit():
    """Given-order launches are 1-D grids of one query per lane: more than
    2^31 queries (or rays) are refused before any launch."""
    L = _lib()
    lib = L.lib()
    cfg = W.get("c2")
    p = L.lsp_plan_create(cfg.L, cfg.Xi)
    v = L.lsp_vol_bind(p, 0, [0x1000], (8, 8, 8))
    big = (1 << 31) + 1
    assert lib.lsp_eval(p, v, 0x1000, big, 0x1000, None, None) == -2
    assert lib.lsp_eval_mse(p, v, 0x1000, 0x1000, big, None, None, None, 0x1000, None) == -2
    assert lib.lsp_eval_adjoint(p, v, 0x1000, 0x1000, big, (ctypes.c_void_p * 1)(0x1000), None, None) == -2
    L.lsp_vol_release(v)
    L.lsp_plan_destroy(p)


def test_api_argument_validation():
    """The Python layer checks dtype, rank and length of every per-query
    argument before anything reaches the library (a float64 target or a
    short gradient would otherwise be read as float32 or past its end)."""
    import torch
    from paper_2102_08514_amd import api
    cfg = W.get("c4")
    sp = api.LatticeSpline(cfg.L, cfg.Xi)
    x64 = torch.zeros(10, 3, dtype=torch.float64)
    x2 = torch.zeros(10, 2)
    x = torch.zeros(10, 3)
    for bad in (x64, x2, torch.zeros(10)):
        with pytest.raises(ValueError, match="x must be"):
            sp.eval(None, bad)
        with pytest.raises(ValueError, match="x must be"):
            sp.eval_mse(None, bad, torch.zeros(10))
        with pytest.raises(ValueError, match="x must be"):
            sp.adjoint(None, bad, torch.zeros(10))
    for bad in (torch.zeros(10, dtype=torch.float64), torch.zeros(9), torch.zeros(10, 1)):
        with pytest.raises(ValueError, match="y must be"):
            sp.eval_mse(None, x, bad)
        with pytest.raises(ValueError, match="g must be"):
            sp.adjoint(None, x, bad)
    # correct shapes and dtypes, but host memory: refused as well
    with pytest.raises(ValueError, match="GPU"):
        sp.eval(None, x)
    with pytest.raises(ValueError, match="GPU"):
        sp.eval_mse(None, x, torch.zeros(10))


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
