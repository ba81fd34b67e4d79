"""ctypes binding of the C ABI (include/lsp.h): argument marshalling only.

Every step of the computation runs in the HIP library; if it cannot be
loaded, using the binding raises.
"""

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# LSP_LIBRARY selects another build of the same library (the host-sanitizer
# build of the CPU tests); by default the in-tree one
LIB_PATH = os.environ.get("LSP_LIBRARY") or os.path.join(_PKG, "lib", "liblsp.so")

LSP_F32, LSP_BF16, LSP_F16, LSP_F64 = 0, 1, 2, 3

# every symbol declared in include/lsp.h
EXPORTS = (
    "lsp_plan_create", "lsp_plan_create_voronoi", "lsp_plan_info", "lsp_plan_destroy", "lsp_vol_bind", "lsp_vol_release",
    "lsp_eval", "lsp_eval_mse", "lsp_eval_adjoint", "lsp_eval_rays", "lsp_status_string",
    "lsp_schedule_size", "lsp_schedule", "lsp_eval_scheduled", "lsp_eval_mse_scheduled",
    "lsp_eval_adjoint_scheduled", "lsp_render", "lsp_mse_backward_scheduled", "lsp_eval_scheduled_static",
)
LSP_STATIC_SCRATCH_BYTES = 64 << 20


class LspInfo(ctypes.Structure):
    _fields_ = [
        ("s", ctypes.c_int32), ("n_dirs", ctypes.c_int32), ("det_l", ctypes.c_int32), ("D", ctypes.c_int32),
        ("n_cosets", ctypes.c_int32), ("shifts", (ctypes.c_int32 * 4) * 8), ("degree", ctypes.c_int32),
        ("n_subregions", ctypes.c_int32), ("n_planes", ctypes.c_int32), ("fold_even", ctypes.c_int32),
        ("stencil", ctypes.c_int32 * 16), ("lookups", ctypes.c_int32), ("n_monomials", ctypes.c_int32),
        ("nnz", ctypes.c_int32 * 16), ("offset_min", ctypes.c_int32), ("offset_max", ctypes.c_int32),
        ("name", ctypes.c_char * 32), ("fma_b", ctypes.c_int32 * 16), ("fma_w", ctypes.c_int32 * 16),
        ("grad_terms", ctypes.c_int32), ("kind", ctypes.c_int32), ("voronoi_n", ctypes.c_int32),
    ]


class LspRenderParams(ctypes.Structure):
    _fields_ = [
        ("f0", ctypes.c_float), ("f1", ctypes.c_float), ("ambient", ctypes.c_float), ("diffuse", ctypes.c_float),
        ("grad_eps", ctypes.c_float), ("alpha_stop", ctypes.c_float), ("tf_len", ctypes.c_int32),
    ]


class LspError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        P = ctypes.POINTER
        L.lsp_plan_create.argtypes = [i32, P(i32), i32, P(i32), u32, P(vp)]
        L.lsp_plan_create_voronoi.argtypes = [i32, P(i32), P(i32), i32, u32, P(vp)]
        L.lsp_plan_info.argtypes = [vp, P(LspInfo)]
        L.lsp_plan_destroy.argtypes = [vp]
        L.lsp_vol_bind.argtypes = [vp, i32, P(vp), P(i64), P(vp)]
        L.lsp_vol_release.argtypes = [vp]
        L.lsp_eval.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.lsp_eval_mse.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, vp, vp]
        L.lsp_eval_adjoint.argtypes = [vp, vp, vp, vp, i64, P(vp), vp, vp]
        L.lsp_eval_rays.argtypes = [vp, vp, P(ctypes.c_float), P(ctypes.c_float), i32, i32, i32, i64, i64, vp, vp,
                                    vp]
        sz = ctypes.c_size_t
        L.lsp_schedule_size.argtypes = [vp, vp, i64, P(sz)]
        L.lsp_schedule.argtypes = [vp, vp, vp, i64, vp, sz, vp]
        L.lsp_eval_scheduled.argtypes = [vp, vp, vp, i64, vp, sz, vp, vp, vp]
        L.lsp_eval_mse_scheduled.argtypes = [vp, vp, vp, vp, i64, vp, sz, vp, vp, vp, vp, vp]
        L.lsp_eval_adjoint_scheduled.argtypes = [vp, vp, vp, vp, i64, vp, sz, P(vp), vp, vp]
        L.lsp_render.argtypes = [vp, vp, P(ctypes.c_float), P(ctypes.c_float), i32, i32, i32, i64, i64, vp,
                                 P(LspRenderParams), vp, vp]
        L.lsp_mse_backward_scheduled.argtypes = [vp, vp, vp, i64, vp, sz, P(vp), vp]
        L.lsp_eval_scheduled_static.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.lsp_status_string.argtypes = [i32]
        L.lsp_status_string.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != "lsp_status_string":
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def status_string(status):
    return lib().lsp_status_string(int(status)).decode()


def check(status, where):
    if status != 0:
        raise LspError(status, where)


def _i32_array(vals):
    vals = [int(v) for v in vals]
    return (ctypes.c_int32 * len(vals))(*vals)


def lsp_plan_create(L, Xi, flags=0):
    """L: s x s, Xi: s x n integer matrices (nested sequences or arrays)."""
    L = [[int(v) for v in row] for row in L]
    Xi = [[int(v) for v in row] for row in Xi]
    s, n = len(L), len(Xi[0])
    out = ctypes.c_void_p()
    check(lib().lsp_plan_create(s, _i32_array(sum(L, [])), n, _i32_array(sum(Xi, [])), flags, ctypes.byref(out)),
          "lsp_plan_create")
    return out


def lsp_plan_create_voronoi(L, Lv, n, flags=0):
    """L, Lv: s x s integer matrices; n: the Voronoi spline's index (V_n)."""
    L = [[int(v) for v in row] for row in L]
    Lv = [[int(v) for v in row] for row in Lv]
    out = ctypes.c_void_p()
    check(lib().lsp_plan_create_voronoi(len(L), _i32_array(sum(L, [])), _i32_array(sum(Lv, [])), int(n), flags,
                                        ctypes.byref(out)), "lsp_plan_create_voronoi")
    return out


def lsp_plan_info(plan):
    info = LspInfo()
    check(lib().lsp_plan_info(plan, ctypes.byref(info)), "lsp_plan_info")
    M, s, K = info.n_cosets, info.s, info.n_subregions
    return {
        "name": info.name.decode(), "s": s, "n_dirs": info.n_dirs, "det_l": info.det_l, "D": info.D,
        "n_cosets": M, "shifts": [tuple(info.shifts[k][a] for a in range(s)) for k in range(M)],
        "degree": info.degree, "n_subregions": K, "n_planes": info.n_planes, "fold_even": bool(info.fold_even),
        "stencil": [info.stencil[k] for k in range(K)], "lookups": info.lookups,
        "n_monomials": info.n_monomials, "nnz": [info.nnz[k] for k in range(K)],
        "offset_min": info.offset_min, "offset_max": info.offset_max,
        "fma_b": [info.fma_b[k] for k in range(K)], "fma_w": [info.fma_w[k] for k in range(K)],
        "grad_terms": info.grad_terms, "kind": "voronoi" if info.kind == 1 else "box",
        "voronoi_n": info.voronoi_n,
    }


def lsp_plan_destroy(plan):
    check(lib().lsp_plan_destroy(plan), "lsp_plan_destroy")


def lsp_vol_bind(plan, dtype, coset_ptrs, dims):
    ptrs = (ctypes.c_void_p * len(coset_ptrs))(*[int(p) for p in coset_ptrs])
    d = (ctypes.c_int64 * len(dims))(*[int(v) for v in dims])
    out = ctypes.c_void_p()
    check(lib().lsp_vol_bind(plan, int(dtype), ptrs, d, ctypes.byref(out)), "lsp_vol_bind")
    return out


def lsp_vol_release(vol):
    check(lib().lsp_vol_release(vol), "lsp_vol_release")


def lsp_eval(plan, vol, x_ptr, n, f_ptr, grad_ptr, stream):
    check(lib().lsp_eval(plan, vol, x_ptr, int(n), f_ptr, grad_ptr, stream), "lsp_eval")


def lsp_eval_scheduled_static(plan, vol, x_ptr, n, f_ptr, grad_ptr, stream):
    check(lib().lsp_eval_scheduled_static(plan, vol, x_ptr, int(n), f_ptr, grad_ptr, stream),
          "lsp_eval_scheduled_static")


def lsp_eval_mse(plan, vol, x_ptr, y_ptr, n, f_ptr, dldf_ptr, dldx_ptr, loss_ptr, stream):
    check(lib().lsp_eval_mse(plan, vol, x_ptr, y_ptr, int(n), f_ptr, dldf_ptr, dldx_ptr, loss_ptr, stream),
          "lsp_eval_mse")


def lsp_eval_adjoint(plan, vol, x_ptr, g_ptr, n, grad_c_ptrs, grad_x_ptr, stream):
    arr = (ctypes.c_void_p * len(grad_c_ptrs))(*[int(p) for p in grad_c_ptrs])
    check(lib().lsp_eval_adjoint(plan, vol, x_ptr, g_ptr, int(n), arr, grad_x_ptr, stream), "lsp_eval_adjoint")


def lsp_eval_rays(plan, vol, c, A, W, H, steps, ray0, nrays, out_ptr, samples_ptr, stream):
    cc = (ctypes.c_float * 3)(*[float(v) for v in c])
    AA = (ctypes.c_float * 9)(*[float(v) for v in A])
    check(lib().lsp_eval_rays(plan, vol, cc, AA, int(W), int(H), int(steps), int(ray0), int(nrays), out_ptr,
                              samples_ptr, stream), "lsp_eval_rays")


def lsp_schedule_size(plan, vol, n):
    out = ctypes.c_size_t()
    check(lib().lsp_schedule_size(plan, vol, int(n), ctypes.byref(out)), "lsp_schedule_size")
    return out.value


def lsp_schedule(plan, vol, x_ptr, n, ws_ptr, ws_bytes, stream):
    check(lib().lsp_schedule(plan, vol, x_ptr, int(n), ws_ptr, int(ws_bytes), stream), "lsp_schedule")


def lsp_eval_scheduled(plan, vol, x_ptr, n, ws_ptr, ws_bytes, f_ptr, grad_ptr, stream):
    check(lib().lsp_eval_scheduled(plan, vol, x_ptr, int(n), ws_ptr, int(ws_bytes), f_ptr, grad_ptr, stream),
          "lsp_eval_scheduled")


def lsp_eval_mse_scheduled(plan, vol, x_ptr, y_ptr, n, ws_ptr, ws_bytes, f_ptr, dldf_ptr, dldx_ptr, loss_ptr,
                           stream):
    check(lib().lsp_eval_mse_scheduled(plan, vol, x_ptr, y_ptr, int(n), ws_ptr, int(ws_bytes), f_ptr, dldf_ptr,
                                       dldx_ptr, loss_ptr, stream), "lsp_eval_mse_scheduled")


def lsp_eval_adjoint_scheduled(plan, vol, x_ptr, g_ptr, n, ws_ptr, ws_bytes, grad_c_ptrs, grad_x_ptr, stream):
    arr = (ctypes.c_void_p * len(grad_c_ptrs))(*[int(p) for p in grad_c_ptrs])
    check(lib().lsp_eval_adjoint_scheduled(plan, vol, x_ptr, g_ptr, int(n), ws_ptr, int(ws_bytes), arr, grad_x_ptr,
                                           stream), "lsp_eval_adjoint_scheduled")


def lsp_render(plan, vol, c, A, W, H, steps, ray0, nrays, tf_ptr, params, rgba_ptr, stream):
    """params: dict with f0, f1, ambient, diffuse, grad_eps, alpha_stop, tf_len."""
    cc = (ctypes.c_float * 3)(*[float(v) for v in c])
    AA = (ctypes.c_float * 9)(*[float(v) for v in A])
    p = LspRenderParams(**{k: params[k] for k in ("f0", "f1", "ambient", "diffuse", "grad_eps", "alpha_stop",
                                                  "tf_len")})
    check(lib().lsp_render(plan, vol, cc, AA, int(W), int(H), int(steps), int(ray0), int(nrays), tf_ptr,
                           ctypes.byref(p), rgba_ptr, stream), "lsp_render")


def lsp_mse_backward_scheduled(plan, vol, x_ptr, n, ws_ptr, ws_bytes, grad_c_ptrs, stream):
    arr = (ctypes.c_void_p * len(grad_c_ptrs))(*[int(p) for p in grad_c_ptrs])
    check(lib().lsp_mse_backward_scheduled(plan, vol, x_ptr, int(n), ws_ptr, int(ws_bytes), arr, stream),
          "lsp_mse_backward_scheduled")
