"""Throughput benchmark: lattice box-spline evaluation on one MI355X.

Headline (`value`): the 7-direction ZP box spline on Z^3 (c2), a 256^3 FP32
coefficient volume (smooth random field + noise) and 2^24 uniform random
FP32 queries, forward.  One step = the schedule (counting sort of the
queries by brick) plus one evaluation of all queries, inputs resident in HBM.

The same run also times, as sub-records of the one JSON line, the rest of
the metric: c2 with BF16 storage; c3 (BCC quartic, 1024^2 rays x 512 steps,
f and grad f) in FP32 and BF16; c4 (FCC 6-direction) and c5 (D4* 8-direction)
MSE training steps, forward + backward, in FP32 (and c5 in BF16), each with
its fwd+bwd / fwd ratio and its max / RMS error against the FP64 oracle on a
prefix; and the BF16 / FP32 speedups.

    python bench.py [--steps K] [--warmup W] [--config c1|c2|c3|c4|c5|d4] [--dtype f32|bf16|f16]
                    [--no-cpu] [--no-extra] [--no-sub] [--order sorted|given] [--render] [--gpus 1]

With --config only that workload is timed (no sub-records), as the
profiling runs do.
"""

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed instructions: 256 CUs x 4 SIMDs x 16 lanes
# x 2 flops (one FMA) x 2.4 GHz.  The published 157.3 TFLOP/s counts packed
# FP32 FMAs, which this library is built without.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
VALU_PEAK_PUBLISHED_TFLOPS = 157.3
WORKLOADS = {
    "c1": "BCC 2x32^3 FP64 coefficients, linear rhombic dodecahedron (4 dir.), 1e5 queries, forward",
    "c2": "Z^3 256^3, 7-direction ZP box spline, 2^24 random queries, forward",
    "c3": "BCC 2x192^3, quartic 7-direction box spline, 1024x1024 rays x 512 steps, forward + grad",
    "c4": "FCC 4x128^3, 6-direction box spline, 2^22 queries, MSE forward + backward",
    "c5": "D4* 2x48^4, 8-direction box spline, 2^22 queries, MSE forward + backward",
    "d4": "D4 8x24^4, the 8-direction box spline of Sec. 5.2 (240 lookups), 2^22 queries, forward",
    "vor_rays": "BCC 2x192^3, BCC Voronoi spline 1, 1024x1024 rays x 512 steps, forward + grad",
    "vor_fcc": "FCC 4x128^3, FCC Voronoi spline 1, 2^22 random queries, forward",
}
SUB_RECORDS = (("c2", "bf16"), ("c3", "f32"), ("c3", "bf16"), ("c4", "f32"), ("c5", "f32"), ("c5", "bf16"),
               ("vor_rays", "f32"), ("vor_fcc", "f32"))
ACC_PREFIX = {"c2": 4096, "c4": 4096, "c5": 2048, "d4": 512, "c1": 100000}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ CPU oracle
def make_oracle(cfg):
    from oracle import ConvolutionSumOracle, VoronoiSumOracle
    from workloads import configs as W
    if cfg.voronoi:
        return VoronoiSumOracle(cfg.L, cfg.Lv, cfg.voronoi[1], W=cfg.voronoi_gen, sigma=W.VORONOI_SIGMA,
                                method="boxsum")
    return ConvolutionSumOracle(cfg.L, cfg.Xi)


def _oracle_chunk(args):
    name, coeffs, X, chunk, grad = args
    from workloads import configs as W
    return make_oracle(W.get(name)).eval(coeffs, X, chunk=chunk, want_grad=grad)


def host_cores():
    return min(os.cpu_count() or 1, 16)


def oracle_values(name, coeffs, X, grad=False, chunk=256):
    """The FP64 oracle at the rows of X on the host's cores."""
    coeffs64 = [np.asarray(c, dtype=np.float64) for c in coeffs]
    X = np.asarray(X, dtype=np.float64)
    parts = [(name, coeffs64, X[i:i + chunk], chunk, grad) for i in range(0, len(X), chunk)]
    with mp.get_context("fork").Pool(host_cores()) as pool:
        res = pool.map(_oracle_chunk, parts)
    if grad:
        return np.concatenate([r[0] for r in res]), np.concatenate([r[1] for r in res])
    return np.concatenate(res)


def cpu_baseline(name, coeffs, X, target_s=8.0):
    """Time the FP64 oracle on a bounded prefix of the same queries using the
    host's cores; returns (record, indices, values)."""
    cores = host_cores()
    coeffs64 = [np.asarray(c, dtype=np.float64) for c in coeffs]
    chunk = 256
    # calibrate on one core with one chunk (also the single-core rate)
    t0 = time.perf_counter()
    _oracle_chunk((name, coeffs64, X[:chunk].astype(np.float64), chunk, False))
    per_q = (time.perf_counter() - t0) / chunk
    n = int(min(len(X), max(256, target_s * cores / per_q)))
    n = (n // 256) * 256 or 256
    t0 = time.perf_counter()
    vals = oracle_values(name, coeffs64, X[:n], chunk=chunk)
    dt = time.perf_counter() - t0
    rec = {"value": n / dt / 1e9, "unit": "Gsamples/s", "cores": cores, "kind": "oracle",
           "sample": f"first {n} queries of the same workload, FP64 oracle, {dt:.1f} s",
           "single_core_value": 1.0 / per_q / 1e9}
    return rec, np.arange(n), vals


def error_record(got, want, coeffs, what):
    scale = max(float(np.abs(c).max()) for c in coeffs)
    err = np.abs(np.asarray(got, dtype=np.float64) - np.asarray(want, dtype=np.float64)) / scale
    return {"max_err": float(err.max()), "rms_err": float(np.sqrt(np.mean(err ** 2))),
            "norm": "|f - f_oracle| / max|c|", "n": int(err.shape[0]), "against": what}


# ------------------------------------------------------------------ timing
def time_phases(fn, steps, warmup, torch, nmarks=1, flush=None):
    """Run fn() `warmup` times, then time `steps` calls.  fn(marks) records
    the events in `marks` at its phase boundaries (nmarks of them), so every
    step yields nmarks + 1 phase durations, measured with HIP events on the
    stream the library launches on (torch's current stream).  With `flush`,
    flush() runs before every step, outside the timed events and the wall
    clock (cold-cache timing).  Returns (wall seconds over the timed steps,
    per-phase mean seconds, per-phase median seconds)."""
    for _ in range(warmup):
        fn(None)
    torch.cuda.synchronize()
    E = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    ev = [[E() for _ in range(nmarks + 2)] for _ in range(steps)]
    wall = 0.0
    t0 = time.perf_counter()
    for row in ev:
        if flush is not None:
            torch.cuda.synchronize()
            flush()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        row[0].record()
        fn(row[1:-1])
        row[-1].record()
        if flush is not None:
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
    torch.cuda.synchronize()
    if flush is None:
        wall = time.perf_counter() - t0
    per = np.array([[row[i].elapsed_time(row[i + 1]) / 1e3 for i in range(nmarks + 1)] for row in ev])
    return wall, per.mean(axis=0), np.median(per, axis=0)


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy of 1 GiB: read + write bandwidth in GB/s.  Its
    kernel also calibrates the traffic counters, since it reads and writes
    exactly nbytes per dispatch."""
    a = torch.ones(nbytes // 4, device="cuda")
    b = torch.empty_like(a)
    _, mean, _ = time_phases(lambda marks: b.copy_(a), reps, 3, torch, nmarks=0)
    del a, b
    return 2 * nbytes / float(mean[0]) / 1e9


# ------------------------------------------------------------------ committed counter summaries
_CSRC = "paper_2102_08514_amd/csrc"
_SHARED_SRC = ("lsp_kernels.hip", "lsp_binned.hip", "lsp_launch.hip", "lsp_internal.h", "lsp_api.hip")
SPLINE_OF = {"c1": "bcc_linear", "c2": "cc_zp", "c3": "bcc_quartic", "c4": "fcc_6dir", "c5": "d4s_8dir",
             "d4": "d4_8dir", "vor_rays": "bcc_voronoi1", "vor_fcc": "fcc_voronoi1"}


def kernel_source_digest(config=None):
    """sha256 over the shared HIP sources and the generated table of the
    workload's spline (every table when config is None)."""
    import hashlib
    h = hashlib.sha256()
    names = list(_SHARED_SRC)
    gen = os.path.join(ROOT, _CSRC, "generated")
    if config is None:
        names += [os.path.join("generated", n) for n in sorted(os.listdir(gen)) if n.endswith(".inc")]
    else:
        names.append(os.path.join("generated", SPLINE_OF[config] + ".inc"))
    for name in names:
        h.update(os.path.basename(name).encode())
        with open(os.path.join(ROOT, _CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_counters(config, dtype):
    """Per-launch counter values of this workload's kernels from the committed
    summaries under profiles/: rows `| counter | <config> | <dtype> |
    <kernel> | <name> | <value> | <digest> |`, kept only when taken with the
    current kernel sources.  Returns {kernel: {name: value}, '_source': [...]}."""
    pdir = os.path.join(ROOT, "profiles")
    out, srcs = {}, set()
    if not os.path.isdir(pdir):
        return out
    digest = kernel_source_digest(config)
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(pdir, name)) as fh:
            for line in fh:
                cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
                if len(cells) == 7 and cells[0] == "counter" and cells[1] == config and cells[2] == dtype \
                        and cells[6] == digest:
                    try:
                        out.setdefault(cells[3], {})[cells[4]] = float(cells[5])
                    except ValueError:
                        continue
                    srcs.add(f"profiles/{name}")
    if out:
        out["_source"] = sorted(srcs)
    return out


# ------------------------------------------------------------------ per-sample work of the generated code
def flops_per_sample(info, grad, adjoint=False):
    """Algorithmic FP32 operations per query (or ray sample) of the generated
    polynomial code, counting each emitted multiply-add as 2 flops: per coset
    b = A c (fma_b, averaged over sub-regions), the monomials (n_mono - 1
    products) and psi = b . mono (n_mono), plus the gradient (grad_terms);
    the adjoint adds the stencil weights w = A^T mono (fma_w)."""
    nm = info["n_monomials"]
    fb = float(np.mean(info["fma_b"]))
    fw = float(np.mean(info["fma_w"]))
    fwd = fb + (nm - 1) + nm + (info["grad_terms"] if grad else 0)
    adj = fw + (nm - 1)
    return 2.0 * info["n_cosets"] * (fwd + (adj if adjoint else 0.0))


def roofline(kernel, n, seconds, bytes_per, flops_per, counters):
    """The dominant kernel against its bound: VALU for the polynomial work
    (the staged, LDS-fed kernels move far fewer HBM bytes than the gather
    formulation counts), with the algorithmic-byte view kept as
    `effective_hbm` (it may exceed 1: LDS staging serves most gathers) and
    the measured counters when a summary for the current sources exists."""
    tflops = flops_per * n / seconds / 1e12
    gbs = bytes_per * n / seconds / 1e9
    rec = {"bound": "alu", "achieved": round(tflops, 3), "peak": round(VALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
           "frac": round(tflops / VALU_PEAK_TFLOPS, 4), "traffic": None, "kernel": kernel,
           "flops_per_sample": round(flops_per, 1), "samples_per_launch": int(n),
           "launch_ms_mean": round(seconds * 1e3, 4), "peak_published_packed": VALU_PEAK_PUBLISHED_TFLOPS,
           "effective_hbm": {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_sample": round(bytes_per, 3)}}
    c = counters.get(kernel)
    if c and "read_bytes" in c and "write_bytes" in c:
        # bytes between L2 and the memory fabric per launch (size-class request
        # counters; Infinity-Cache hits included, so an upper bound on HBM bytes)
        traffic = c["read_bytes"] + c["write_bytes"]
        rec["traffic"] = int(traffic)
        rec["dram"] = {"achieved": round(traffic / seconds / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(traffic / seconds / 1e9 / HBM_PEAK_GBS, 4),
                       "read_bytes": int(c["read_bytes"]), "write_bytes": int(c["write_bytes"])}
        if "valu_insts" in c:
            # wave-level VALU instructions, 4 cycles each on a 16-lane SIMD, 4 SIMDs per CU
            rec["valu_issue_frac"] = round(c["valu_insts"] / (256 * 2.4e9 * seconds), 4)
        for key in ("valu_busy_pct", "l2_hit_pct", "lds_bank_conflict_pct", "dur_us"):
            if key in c:
                rec["profiled_" + key if key == "dur_us" else key] = round(c[key], 2)
        rec["counter_source"] = counters.get("_source")
    return rec


def binned_kernel(w):
    """Name of the scheduled forward kernel: 4-D units run the variant held to
    128 VGPRs."""
    return "k_eval_binned_w4" if w.s == 4 else "k_eval_binned"


# ------------------------------------------------------------------ workloads
class Workload:
    def __init__(self, name, dtype, torch, lsp, W, I):
        self.name, self.torch = name, torch
        self.cfg = cfg = W.get(name)
        tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[dtype]
        if name == "c1":
            tdt = torch.float64
        self.tdt = tdt
        self.dname = {torch.float32: "f32", torch.bfloat16: "bf16", torch.float16: "f16", torch.float64: "f64"}[tdt]
        self.bytes_c = {torch.float32: 4, torch.bfloat16: 2, torch.float16: 2, torch.float64: 8}[tdt]
        log(f"[bench] generating {name} inputs ({self.dname})")
        self.coeffs = I.coefficients(cfg)
        self.sp = (lsp.LatticeSpline(cfg.L, voronoi=(cfg.Lv, cfg.voronoi[1])) if cfg.voronoi else
                   lsp.LatticeSpline(cfg.L, cfg.Xi))
        self.info = self.sp.info
        self.dev = [torch.from_numpy(np.ascontiguousarray(c)).to(tdt).cuda() for c in self.coeffs]
        self.vol = self.sp.bind(self.dev)
        self.strm = torch.cuda.current_stream().cuda_stream
        self.s = cfg.s
        self.rays = "rays" in cfg.extra
        self.X = None if self.rays else I.queries(cfg)
        self.I = I

    def stored(self):
        """The coefficients as stored on the device (after rounding), FP64."""
        return [d.double().cpu().numpy() for d in self.dev]

    def release(self):
        self.torch.cuda.synchronize()
        for k in list(vars(self)):
            if k not in ("torch", "name"):
                setattr(self, k, None)
        self.torch.cuda.empty_cache()


def mark(marks, k):
    if marks:
        marks[k].record()


def bench_forward(w, steps, warmup, order="sorted", extra=False):
    """Schedule + forward (f only) of all queries."""
    torch = w.torch
    from paper_2102_08514_amd import _lib as Lb
    n = len(w.X)
    x = torch.from_numpy(w.X).cuda()
    f = torch.empty(n, device="cuda", dtype=w.vol.out_dtype)
    ws_bytes = Lb.lsp_schedule_size(w.sp.plan, w.vol.handle, n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")

    def step(marks, sched=(order == "sorted")):
        if sched:
            Lb.lsp_schedule(w.sp.plan, w.vol.handle, x.data_ptr(), n, ws.data_ptr(), ws_bytes, w.strm)
        mark(marks, 0)
        if sched:
            Lb.lsp_eval_scheduled(w.sp.plan, w.vol.handle, x.data_ptr(), n, ws.data_ptr(), ws_bytes, f.data_ptr(),
                                  None, w.strm)
        else:
            Lb.lsp_eval(w.sp.plan, w.vol.handle, x.data_ptr(), n, f.data_ptr(), None, w.strm)

    wall, pmean, pmed = time_phases(step, steps, warmup, torch, nmarks=1)
    out_b = 8 if w.tdt == torch.float64 else 4
    rec = {"value": round(n / (wall / steps) / 1e9, 4), "unit": "Gsamples/s", "ms_per_step": round(wall / steps * 1e3, 4),
           "n_samples": n, "phases_ms_mean": {"schedule": round(float(pmean[0]) * 1e3, 4),
                                              "forward": round(float(pmean[1]) * 1e3, 4)}}
    rec["_eval_s"] = float(pmean[1])
    rec["_bytes_per"] = 4 * w.s + w.info["lookups"] * w.bytes_c + out_b
    rec["_flops_per"] = flops_per_sample(w.info, grad=False)
    rec["_kernel"] = binned_kernel(w) if order == "sorted" else "k_eval"
    if extra and order == "sorted":
        k = max(3, steps // 4)
        gw, _, _ = time_phases(lambda marks: step(marks, sched=False), k, 1, torch, nmarks=1)
        rec["given_order"] = {"ms_per_step": round(gw / k * 1e3, 4), "value": round(n / (gw / k) / 1e9, 4)}
        junk = torch.empty(1 << 28, device="cuda")
        cw, _, _ = time_phases(step, k, 1, torch, nmarks=1, flush=lambda: junk.fill_(1.0))
        rec["cold_cache"] = {"ms_per_step": round(cw / k * 1e3, 4), "value": round(n / (cw / k) / 1e9, 4),
                             "note": "a 1 GiB write evicts the MALL and every L2 before each step"}
        del junk
    step(None)
    torch.cuda.synchronize()
    rec["_f"] = f
    return rec


def bench_mse(w, steps, warmup, order="sorted"):
    """One MSE training step: schedule, forward (loss, dL/dx; dL/df kept in
    the workspace), backward (dL/dc)."""
    torch = w.torch
    from paper_2102_08514_amd import _lib as Lb
    n = len(w.X)
    x = torch.from_numpy(w.X).cuda()
    y = torch.from_numpy(w.I.targets(w.cfg, w.X)).cuda()
    loss = torch.zeros(1, device="cuda", dtype=torch.float64)
    f = torch.empty(n, device="cuda")
    dldf = torch.empty(n, device="cuda")
    # one buffer for every coset's dL/dc, so clearing it is one fill
    gflat = torch.zeros(sum(c.numel() for c in w.dev), device="cuda")
    gradc = list(torch.split(gflat, [c.numel() for c in w.dev]))
    gradc = [g.view(c.shape) for g, c in zip(gradc, w.dev)]
    gx = torch.empty(n, w.s, device="cuda")
    ws_bytes = Lb.lsp_schedule_size(w.sp.plan, w.vol.handle, n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    sched = order == "sorted"

    def step(marks, want_f=False):
        if sched:
            Lb.lsp_schedule(w.sp.plan, w.vol.handle, x.data_ptr(), n, ws.data_ptr(), ws_bytes, w.strm)
        mark(marks, 0)
        loss.zero_()
        fo = f.data_ptr() if want_f else None
        if sched:
            Lb.lsp_eval_mse_scheduled(w.sp.plan, w.vol.handle, x.data_ptr(), y.data_ptr(), n, ws.data_ptr(), ws_bytes,
                                      fo, None, gx.data_ptr(), loss.data_ptr(), w.strm)
        else:
            Lb.lsp_eval_mse(w.sp.plan, w.vol.handle, x.data_ptr(), y.data_ptr(), n, fo, dldf.data_ptr(),
                            gx.data_ptr(), loss.data_ptr(), w.strm)
        mark(marks, 1)
        gflat.zero_()
        if sched:
            Lb.lsp_mse_backward_scheduled(w.sp.plan, w.vol.handle, x.data_ptr(), n, ws.data_ptr(), ws_bytes,
                                          [g.data_ptr() for g in gradc], w.strm)
        else:
            Lb.lsp_eval_adjoint(w.sp.plan, w.vol.handle, x.data_ptr(), dldf.data_ptr(), n,
                                [g.data_ptr() for g in gradc], None, w.strm)

    wall, pmean, _ = time_phases(step, steps, warmup, torch, nmarks=2)
    t_s, t_f, t_b = (float(v) for v in pmean)
    Lq = w.info["lookups"]
    rec = {"value": round(n / (wall / steps) / 1e9, 4), "unit": "Gsamples/s",
           "ms_per_step": round(wall / steps * 1e3, 4), "n_samples": n,
           "phases_ms_mean": {"schedule": round(t_s * 1e3, 4), "forward": round(t_f * 1e3, 4),
                              "backward": round(t_b * 1e3, 4)},
           "forward_only": {"value": round(n / (t_s + t_f) / 1e9, 4), "unit": "Gsamples/s",
                            "note": "schedule + forward phases of the same timed steps"},
           "fwd_bwd_over_fwd": round((t_s + t_f + t_b) / (t_s + t_f), 3)}
    # forward: x + y + coefficients + dL/df + dL/dx; backward: x + dL/df + one 4-byte scatter per site
    rec["_phases"] = {
        "forward": (t_f, 4 * w.s + 4 + Lq * w.bytes_c + 4 + 4 * w.s, flops_per_sample(w.info, grad=True)),
        "backward": (t_b, 4 * w.s + 4 + Lq * 4, flops_per_sample(w.info, grad=False, adjoint=True)
                     - flops_per_sample(w.info, grad=False))}
    step(None, want_f=True)        # untimed: store f for the accuracy check
    torch.cuda.synchronize()
    rec["_f"] = f
    return rec


def bench_rays(w, steps, warmup, render=False):
    torch = w.torch
    cfg = w.cfg
    W_, H_ = cfg.extra["rays"]
    S_ = cfg.extra["steps"]
    c, A = w.I.ray_params(cfg)
    cf, Af = c.astype(np.float32), A.astype(np.float32)
    n = W_ * H_ * S_
    if render:
        tfv = torch.tensor([[0.1, 0.2, 0.9, 0.0], [0.2, 0.8, 0.3, 0.004], [0.9, 0.7, 0.1, 0.008],
                            [1.0, 0.2, 0.1, 0.012]], device="cuda")

        def step(marks):
            w.sp.render(w.vol, cf, Af, W_, H_, S_, tfv, -0.5, 0.5, alpha_stop=2.0)
    else:
        def step(marks):
            w.sp.rays(w.vol, cf, Af, W_, H_, S_)
    wall, pmean, _ = time_phases(step, steps, warmup, torch, nmarks=0)
    rec = {"value": round(n / (wall / steps) / 1e9, 4), "unit": "Gsamples/s",
           "ms_per_step": round(wall / steps * 1e3, 4), "n_samples": n, "rays": W_ * H_, "steps_per_ray": S_,
           "phases_ms_mean": {"render" if render else "rays": round(float(pmean[0]) * 1e3, 4)}}
    rec["_eval_s"] = float(pmean[0])
    rec["_bytes_per"] = w.info["lookups"] * w.bytes_c + 16.0 / S_
    rec["_flops_per"] = flops_per_sample(w.info, grad=True)
    rec["_kernel"] = "k_render" if render else "k_rays"
    return rec


def rays_accuracy(w, rays=(0, 524_287, 1_048_575)):
    """Every sample of a few rays (one-ray launches with per-sample output)
    against the oracle at the same float32 positions."""
    cfg = w.cfg
    W_, H_ = cfg.extra["rays"]
    S_ = cfg.extra["steps"]
    c, A = w.I.ray_params(cfg)
    got, P = [], []
    for r in rays:
        _, smp = w.sp.rays(w.vol, c.astype(np.float32), A.astype(np.float32), W_, H_, S_, ray0=int(r), nrays=1,
                           samples=True)
        got.append(smp.cpu().numpy().reshape(-1, 4))
        tile, within = r >> 6, r & 63
        u = (tile % (W_ // 8)) * 8 + (within & 7)
        v = (tile // (W_ // 8)) * 8 + (within >> 3)
        P.append(w.I.ray_samples(cfg, np.array([u + W_ * v])[:, None], np.arange(S_)[None, :]).reshape(-1, 3))
    got = np.concatenate(got)
    P = np.concatenate(P)
    return got, P


# ------------------------------------------------------------------ one workload -> record
def run_workload(name, dtype, args, torch, lsp, W, I, headline=False):
    w = Workload(name, dtype, torch, lsp, W, I)
    counters = profile_counters(name, w.dname)
    rec = {"workload": f"{name}: {WORKLOADS[name]}", "dtype": w.dname, "spline": w.info["name"],
           "lookups_per_sample": w.info["lookups"], "volume_dims": list(w.cfg.dims), "n_cosets": w.cfg.M,
           "passes": w.cfg.passes}
    t0 = time.perf_counter()
    if w.rays:
        r = bench_rays(w, args.steps, args.warmup, render=args.render)
    elif w.cfg.passes == "mse":
        r = bench_mse(w, args.steps, args.warmup, order=args.order)
    else:
        r = bench_forward(w, args.steps, args.warmup, order=args.order, extra=headline and not args.no_extra)
    f = r.pop("_f", None)
    if "_phases" in r:
        ph = r.pop("_phases")
        n = r["n_samples"]
        r["roofline"] = {p: roofline({"forward": binned_kernel(w), "backward": "k_adjoint_binned"}[p]
                                     if args.order == "sorted" else {"forward": "k_eval_mse",
                                                                     "backward": "k_adjoint"}[p],
                                     n, t, b, fl, counters) for p, (t, b, fl) in ph.items()}
    else:
        r["roofline"] = roofline(r.pop("_kernel"), r["n_samples"], r.pop("_eval_s"), r.pop("_bytes_per"),
                                 r.pop("_flops_per"), counters)
    rec.update(r)
    # accuracy against the FP64 oracle
    if not args.no_acc:
        if w.rays:
            got, P = rays_accuracy(w)
            fw, gw = oracle_values(name, w.stored(), P, grad=True)
            rec["accuracy"] = error_record(got[:, 0], fw, w.coeffs, "stored coefficients, every sample of 3 rays")
            rec["accuracy"]["grad_max_err"] = error_record(got[:, 1:], gw, w.coeffs, "")["max_err"]
            if w.dname != "f32":
                fu = oracle_values(name, w.coeffs, P)
                rec["accuracy_unrounded"] = error_record(got[:, 0], fu, w.coeffs, "unrounded coefficients")
        elif f is not None and not headline:
            k = min(ACC_PREFIX.get(name, 2048), len(w.X))
            got = f[:k].double().cpu().numpy()
            rec["accuracy"] = error_record(got, oracle_values(name, w.stored(), w.X[:k]), w.coeffs,
                                           f"stored coefficients, first {k} queries")
            if w.dname != "f32":
                rec["accuracy_unrounded"] = error_record(got, oracle_values(name, w.coeffs, w.X[:k]), w.coeffs,
                                                         "unrounded coefficients")
    if headline and not args.no_cpu and w.X is not None:
        log("[bench] CPU oracle leg")
        cb, idx, want = cpu_baseline(name, w.stored(), w.X)
        rec["cpu_baseline"] = cb
        rec["accuracy"] = error_record(f[:len(idx)].double().cpu().numpy(), want, w.coeffs,
                                       f"stored coefficients, first {len(idx)} queries")
    rec["kernel_source_digest"] = kernel_source_digest(name)
    rec["wall_s"] = round(time.perf_counter() - t0, 1)
    w.release()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default=None, choices=sorted(WORKLOADS))
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-acc", action="store_true", help="skip the accuracy checks of the sub-records")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the context legs (given order, cold cache, copy bandwidth)")
    ap.add_argument("--no-sub", action="store_true", help="time the headline workload only")
    ap.add_argument("--render", action="store_true",
                    help="c3: time the volume renderer (transfer function, shading, compositing) instead of the "
                         "plain ray sums")
    ap.add_argument("--order", default="sorted", choices=["sorted", "given"],
                    help="evaluate in the library's scheduled order (timed) or in the given order")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the evaluation shards over queries with no exchange in the forward "
              "pass, and only the single-GPU kernel is timed. Run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2102_08514_amd as lsp
    from workloads import configs as W
    from workloads import inputs as I

    name = args.config or "c2"
    log(f"[bench] headline {name} {args.dtype}: {args.steps} steps after {args.warmup} warm-up")
    head = run_workload(name, args.dtype, args, torch, lsp, W, I, headline=True)
    rec = {
        "metric": "Gsamples/s fwd and fwd+bwd at stated max err vs FP64 oracle; % HBM roofline",
        "value": head["value"], "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "bf16 storage, f32 math", "f16": "f16 storage, f32 math",
                  "f64": "f64"}[head["dtype"]],
        "data": "synthetic",
        "config": {"workload": head["workload"], "spline": head["spline"], "n_samples": head["n_samples"],
                   "lookups_per_sample": head["lookups_per_sample"], "volume_dims": head["volume_dims"],
                   "n_cosets": head["n_cosets"], "passes": head["passes"],
                   "order": ("render" if args.render else "rays") if "rays" in W.get(name).extra else args.order},
    }
    ph = head.pop("roofline")
    rec["roofline"] = ph["forward"] if isinstance(ph, dict) and "forward" in ph else ph
    if isinstance(ph, dict) and "backward" in ph:
        rec["roofline_backward"] = ph["backward"]
    for key in ("phases_ms_mean", "given_order", "cold_cache", "forward_only", "fwd_bwd_over_fwd", "cpu_baseline",
                "accuracy", "kernel_source_digest"):
        if key in head:
            rec[key] = head[key]
    if not args.no_extra:
        rec["roofline"]["copy_gbs"] = round(copy_bandwidth(torch), 1)
    if args.config is None and not args.no_sub:
        subs = {}
        for cname, dt in SUB_RECORDS:
            key = f"{cname}_{dt}"
            log(f"[bench] sub-record {key}")
            sub_args = argparse.Namespace(**vars(args))
            sub_args.render = False
            try:
                subs[key] = run_workload(cname, dt, sub_args, torch, lsp, W, I)
            except Exception as e:          # a failing sub-record must not hide the headline
                subs[key] = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] {key}: {subs[key].get('value')} Gsamples/s")
        rec["sub_records"] = subs
        speed = {}
        for cname in ("c2", "c3", "c5"):
            a = head if cname == name and args.dtype == "f32" else subs.get(f"{cname}_f32")
            b = subs.get(f"{cname}_bf16")
            if a and b and "ms_per_step" in a and "ms_per_step" in b:
                speed[cname] = round(a["ms_per_step"] / b["ms_per_step"], 3)
        rec["bf16_over_f32_speedup"] = speed
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
