"""Object layer over the C ABI for torch device tensors."""

import torch

from . import _lib as L

_DTYPES = {torch.float32: L.LSP_F32, torch.bfloat16: L.LSP_BF16, torch.float16: L.LSP_F16,
           torch.float64: L.LSP_F64}


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def _require_device(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("tensors must live on the GPU")
        if t is not None and not t.is_contiguous():
            raise ValueError("tensors must be contiguous")


def _check_queries(x, s):
    """x must be an N x s float32 tensor (row-major; the device is checked
    after every shape and dtype check of a call)."""
    if not isinstance(x, torch.Tensor) or x.dtype != torch.float32 or x.dim() != 2 or x.shape[1] != s:
        raise ValueError(f"x must be an N x {s} float32 tensor")


def _zero_grad_c(vol, device):
    """Zeroed float32 arrays shaped like the coset arrays, as views of one
    buffer (one fill instead of one per coset)."""
    sizes = [c.numel() for c in vol.coeffs]
    flat = torch.zeros(sum(sizes), device=device, dtype=torch.float32)
    return [t.view(c.shape) for t, c in zip(torch.split(flat, sizes), vol.coeffs)]


def _check_grad_c(grad_c, vol):
    """grad_c: one float32 array per coset, shaped like the coefficient arrays."""
    if len(grad_c) != len(vol.coeffs):
        raise ValueError(f"grad_c must hold {len(vol.coeffs)} arrays (one per coset)")
    for t, c in zip(grad_c, vol.coeffs):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.shape != c.shape:
            raise ValueError("grad_c arrays must be float32 and shaped like the coefficient arrays")
    _require_device(*grad_c)


def _check_per_query(v, n, name):
    """v must be a float32 vector of one value per query."""
    if not isinstance(v, torch.Tensor) or v.dtype != torch.float32 or v.dim() != 1 or v.shape[0] != n:
        raise ValueError(f"{name} must be a float32 vector of length {n} (one value per query)")


class Volume:
    """Coefficient arrays bound to a plan: M device tensors of shape
    (n_{s-1}, ..., n_0) (x fastest), one per coset, same dtype."""

    def __init__(self, spline, coeffs):
        coeffs = list(coeffs)
        if len(coeffs) != spline.info["n_cosets"]:
            raise ValueError(f"expected {spline.info['n_cosets']} coset arrays")
        _require_device(*coeffs)
        dt = coeffs[0].dtype
        if dt not in _DTYPES or any(c.dtype != dt or c.shape != coeffs[0].shape for c in coeffs):
            raise ValueError("coset arrays must share shape and a supported dtype")
        if coeffs[0].dim() != spline.s:
            raise ValueError("coset arrays must be s-dimensional")
        self.spline = spline
        self.coeffs = coeffs              # keeps the memory alive
        self.dtype = dt
        self.dims = tuple(reversed(coeffs[0].shape))
        self.handle = L.lsp_vol_bind(spline.plan, _DTYPES[dt], [c.data_ptr() for c in coeffs], self.dims)

    @property
    def out_dtype(self):
        return torch.float64 if self.dtype == torch.float64 else torch.float32

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                L.lsp_vol_release(h)
            except Exception:
                pass
            self.handle = None


class Schedule:
    """Evaluation order for one batch of queries (device workspace).  It is
    valid only for the same queries x and a volume of the same dims and
    dtype class as the one it was built with."""

    def __init__(self, spline, vol, x):
        _check_queries(x, spline.s)
        _require_device(x)
        self.n = x.shape[0]
        self.dims = vol.dims
        self.wide = vol.dtype == torch.float64
        self.bytes = L.lsp_schedule_size(spline.plan, vol.handle, self.n)
        # 256-byte aligned: torch's caching allocator returns 512-byte aligned blocks
        self.ws = torch.empty(max(self.bytes, 1), dtype=torch.uint8, device=x.device)
        self.x = x
        L.lsp_schedule(spline.plan, vol.handle, x.data_ptr(), self.n, self.ws.data_ptr(), self.bytes, _stream())


class LatticeSpline:
    """A plan for lattice L and direction matrix Xi, or, with voronoi=(Lv, n),
    for the Voronoi spline V_n of the lattice Lv on L (generated tables must
    exist)."""

    def __init__(self, L_matrix, Xi=None, voronoi=None):
        if (Xi is None) == (voronoi is None):
            raise ValueError("give either a direction matrix Xi or voronoi=(Lv, n)")
        if voronoi is not None:
            self.plan = L.lsp_plan_create_voronoi(L_matrix, voronoi[0], voronoi[1])
        else:
            self.plan = L.lsp_plan_create(L_matrix, Xi)
        self.info = L.lsp_plan_info(self.plan)
        self.s = self.info["s"]

    def __del__(self):
        p = getattr(self, "plan", None)
        if p is not None and p.value:
            try:
                L.lsp_plan_destroy(p)
            except Exception:
                pass
            self.plan = None

    def bind(self, coeffs):
        return Volume(self, coeffs)

    def schedule(self, vol, x):
        """Sort the queries x into cache-friendly evaluation order (see lsp_schedule)."""
        return Schedule(self, vol, x)

    # ------------------------------------------------------------- forward
    def eval(self, vol, x, grad=False, out=None, grad_out=None, schedule=None):
        _check_queries(x, self.s)
        _require_device(x)
        n = x.shape[0]
        f = out if out is not None else torch.empty(n, device=x.device, dtype=vol.out_dtype)
        g = None
        if grad:
            g = grad_out if grad_out is not None else torch.empty(n, self.s, device=x.device, dtype=vol.out_dtype)
        if schedule is None:
            L.lsp_eval(self.plan, vol.handle, x.data_ptr(), n, f.data_ptr(), _ptr(g), _stream())
        else:
            self._check_sched(schedule, x, vol)
            L.lsp_eval_scheduled(self.plan, vol.handle, x.data_ptr(), n, schedule.ws.data_ptr(), schedule.bytes,
                                 f.data_ptr(), _ptr(g), _stream())
        return (f, g) if grad else f

    @staticmethod
    def _check_sched(schedule, x, vol):
        if schedule.n != x.shape[0] or schedule.x.data_ptr() != x.data_ptr():
            raise ValueError("the schedule was built for other queries")
        if schedule.dims != vol.dims or schedule.wide != (vol.dtype == torch.float64):
            raise ValueError("the schedule was built for a volume of other dims or dtype class")

    def eval_mse(self, vol, x, y, schedule=None, grad_x=False, want_f=True, want_dldf=True):
        """f, dL/df, L (and dL/dx if grad_x) for L = mean (f - y)^2; f (dL/df)
        is None when want_f (want_dldf) is False.  With a schedule, dL/df also
        stays in the schedule's workspace for mse_backward."""
        _check_queries(x, self.s)
        n = x.shape[0]
        _check_per_query(y, n, "y")
        _require_device(x, y)
        f = torch.empty(n, device=x.device, dtype=torch.float32) if want_f else None
        dldf = torch.empty(n, device=x.device, dtype=torch.float32) if want_dldf else None
        dldx = torch.empty(n, self.s, device=x.device, dtype=torch.float32) if grad_x else None
        loss = torch.zeros(1, device=x.device, dtype=torch.float64)
        if schedule is None:
            L.lsp_eval_mse(self.plan, vol.handle, x.data_ptr(), y.data_ptr(), n, _ptr(f), _ptr(dldf),
                           _ptr(dldx), loss.data_ptr(), _stream())
        else:
            self._check_sched(schedule, x, vol)
            L.lsp_eval_mse_scheduled(self.plan, vol.handle, x.data_ptr(), y.data_ptr(), n, schedule.ws.data_ptr(),
                                     schedule.bytes, _ptr(f), _ptr(dldf), _ptr(dldx), loss.data_ptr(),
                                     _stream())
        return (f, dldf, loss, dldx) if grad_x else (f, dldf, loss)

    def mse_backward(self, vol, x, schedule, grad_c=None):
        """grad_c (zero-initialised here unless given) += A^T dL/df, with the
        dL/df that the preceding eval_mse(schedule=schedule) left in the
        schedule's workspace."""
        _check_queries(x, self.s)
        _require_device(x)
        self._check_sched(schedule, x, vol)
        if grad_c is None:
            grad_c = _zero_grad_c(vol, x.device)
        _check_grad_c(grad_c, vol)
        L.lsp_mse_backward_scheduled(self.plan, vol.handle, x.data_ptr(), x.shape[0], schedule.ws.data_ptr(),
                                     schedule.bytes, [t.data_ptr() for t in grad_c], _stream())
        return grad_c

    def adjoint(self, vol, x, g, grad_x=False, grad_c=None, schedule=None):
        """grad_c (zero-initialised here unless given) += A^T g; grad_x = g * grad f."""
        _check_queries(x, self.s)
        n = x.shape[0]
        _check_per_query(g, n, "g")
        _require_device(x, g)
        if grad_c is None:
            grad_c = _zero_grad_c(vol, x.device)
        _check_grad_c(grad_c, vol)
        gx = torch.empty(n, self.s, device=x.device, dtype=torch.float32) if grad_x else None
        if schedule is None:
            L.lsp_eval_adjoint(self.plan, vol.handle, x.data_ptr(), g.data_ptr(), n, [t.data_ptr() for t in grad_c],
                               _ptr(gx), _stream())
        else:
            self._check_sched(schedule, x, vol)
            L.lsp_eval_adjoint_scheduled(self.plan, vol.handle, x.data_ptr(), g.data_ptr(), n,
                                         schedule.ws.data_ptr(), schedule.bytes, [t.data_ptr() for t in grad_c],
                                         _ptr(gx), _stream())
        return grad_c, gx

    def rays(self, vol, centre, A, W, H, steps, ray0=0, nrays=None, samples=False):
        nrays = W * H - ray0 if nrays is None else nrays
        dev = vol.coeffs[0].device
        out = torch.empty(nrays, 4, device=dev, dtype=torch.float32)
        smp = torch.empty(nrays, steps, 4, device=dev, dtype=torch.float32) if samples else None
        L.lsp_eval_rays(self.plan, vol.handle, list(centre), [float(v) for row in A for v in row], W, H, steps,
                        ray0, nrays, out.data_ptr(), _ptr(smp), _stream())
        return (out, smp) if samples else out

    def render(self, vol, centre, A, W, H, steps, tf, f0, f1, ambient=0.3, diffuse=0.7, grad_eps=1e-6,
               alpha_stop=2.0, ray0=0, nrays=None):
        """Volume rendering of rays [ray0, ray0 + nrays) (see lsp_render): tf is a
        (T, 4) float32 RGBA tensor on the GPU spanning f in [f0, f1]; returns
        (nrays, 4) float32 (premultiplied colour, opacity)."""
        _require_device(tf)
        if tf.dtype != torch.float32 or tf.dim() != 2 or tf.shape[1] != 4:
            raise ValueError("tf must be a T x 4 float32 tensor")
        nrays = W * H - ray0 if nrays is None else nrays
        out = torch.empty(nrays, 4, device=tf.device, dtype=torch.float32)
        params = {"f0": float(f0), "f1": float(f1), "ambient": float(ambient), "diffuse": float(diffuse),
                  "grad_eps": float(grad_eps), "alpha_stop": float(alpha_stop), "tf_len": int(tf.shape[0])}
        L.lsp_render(self.plan, vol.handle, list(centre), [float(v) for row in A for v in row], W, H, steps, ray0,
                     nrays, tf.data_ptr(), params, out.data_ptr(), _stream())
        return out
