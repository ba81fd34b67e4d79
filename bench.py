"""Throughput benchmark: lattice box-spline evaluation on one MI355X.

Default workload (c2): the 7-direction ZP box spline on Z^3, a 256^3 FP32
coefficient volume (smooth random field + noise) and 2^24 uniform random
FP32 queries, forward.  One step = one evaluation of all queries with the
inputs resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--config c2|c3|c4|c5|c1|d4] [--dtype f32|bf16|f16]
                    [--no-cpu] [--no-extra] [--order sorted|given] [--gpus 1]

Besides the timed steps it reports the same step in the given query order,
with a cold cache, a plain-copy bandwidth (whose kernel also calibrates the
traffic counters), the CPU oracle on a bounded prefix and the accuracy there.
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
WORKLOADS = {
    "c1": "BCC 2x32^3 FP64 coefficients, linear rhombic dodecahedron (4 dir.), 1e5 queries, forward",
    "c2": "Z^3 256^3 FP32, 7-direction ZP box spline, 2^24 random queries, forward",
    "c3": "BCC 2x192^3, quartic 7-direction box spline, 1024x1024 rays x 512 steps, forward + grad",
    "c4": "FCC 4x128^3 FP32, 6-direction box spline, 2^22 queries, MSE forward + backward",
    "c5": "D4* 2x48^4 FP32, 8-direction box spline, 2^22 queries, MSE forward + backward",
    "d4": "D4 8x24^4 FP32, the 8-direction box spline of Sec. 5.2 (240 lookups), 2^22 queries, forward",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ CPU oracle leg
def _oracle_chunk(args):
    name, coeffs, X, chunk = args
    from oracle import ConvolutionSumOracle
    from workloads import configs as W
    cfg = W.get(name)
    o = ConvolutionSumOracle(cfg.L, cfg.Xi)
    return o.eval(coeffs, X, chunk=chunk)


def cpu_baseline(name, coeffs, X, target_s=8.0):
    """Time the FP64 oracle on a bounded prefix of the same queries using the
    host's cores; returns (record, indices, values)."""
    cores = min(os.cpu_count() or 1, 16)
    coeffs64 = [np.asarray(c, dtype=np.float64) for c in coeffs]
    chunk = 256
    # calibrate on one core with one chunk (also the single-core rate)
    t0 = time.perf_counter()
    _oracle_chunk((name, coeffs64, X[:chunk].astype(np.float64), chunk))
    per_q = (time.perf_counter() - t0) / chunk
    n = int(min(len(X), max(256, target_s * cores / per_q)))
    n = (n // 256) * 256 or 256
    Xs = X[:n].astype(np.float64)
    parts = [(name, coeffs64, Xs[i:i + chunk], chunk) for i in range(0, n, chunk)]
    t0 = time.perf_counter()
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        vals = np.concatenate(pool.map(_oracle_chunk, parts))
    dt = time.perf_counter() - t0
    rec = {"value": n / dt / 1e9, "unit": "Gsamples/s", "cores": cores, "kind": "oracle",
           "sample": f"first {n} queries of the same workload, FP64 oracle, {dt:.1f} s",
           "single_core_value": 1.0 / per_q / 1e9}
    return rec, np.arange(n), vals


# ------------------------------------------------------------------ GPU legs
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
    kernel also calibrates the FETCH_SIZE / WRITE_SIZE counters, since it
    reads and writes exactly nbytes per dispatch."""
    a = torch.ones(nbytes // 4, device="cuda")
    b = torch.empty_like(a)
    _, mean, _ = time_phases(lambda marks: b.copy_(a), reps, 3, torch, nmarks=0)
    del a, b
    return 2 * nbytes / float(mean[0]) / 1e9


_SRC_DIRS = ("paper_2102_08514_amd/csrc", "paper_2102_08514_amd/csrc/generated")


def kernel_source_digest():
    """sha256 over the HIP sources and generated tables the library is built from."""
    import hashlib
    h = hashlib.sha256()
    for d in _SRC_DIRS:
        full = os.path.join(ROOT, d)
        for name in sorted(os.listdir(full)):
            if name.endswith((".hip", ".h", ".inc")):
                h.update(name.encode())
                with open(os.path.join(full, name), "rb") as fh:
                    h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(config, dtype):
    """HBM bytes per launch of the dominant kernel from a committed counter
    summary (a row `| traffic | <config> | <dtype> | <kernel> | <bytes> |
    <digest> |`), or None when none exists for the current kernel sources."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    digest = kernel_source_digest()
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(pdir, name)) as fh:
            for line in fh:
                cells = [c.strip() for c in line.strip().strip("|").split("|")]
                if len(cells) == 6 and cells[0] == "traffic" and cells[1] == config and cells[2] == dtype:
                    if cells[5].strip("`") == digest:
                        return {"bytes_per_launch": float(cells[4]), "kernel": cells[3].strip("`"),
                                "source": f"profiles/{name}"}
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the context legs (given order, cold cache, copy bandwidth)")
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

    cfg = W.get(args.config)
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[args.dtype]
    if args.config == "c1":
        tdt = torch.float64
    dname = {torch.float32: "f32", torch.bfloat16: "bf16", torch.float16: "f16", torch.float64: "f64"}[tdt]
    bytes_c = {torch.float32: 4, torch.bfloat16: 2, torch.float16: 2, torch.float64: 8}[tdt]
    log(f"[bench] generating {args.config} inputs")
    coeffs = I.coefficients(cfg)
    sp = lsp.LatticeSpline(cfg.L, cfg.Xi)
    info = sp.info
    dev = [torch.from_numpy(np.ascontiguousarray(c)).to(tdt).cuda() for c in coeffs]
    vol = sp.bind(dev)
    Lq = info["lookups"]
    s = cfg.s
    out_b = 8 if tdt == torch.float64 else 4

    strm = torch.cuda.current_stream().cuda_stream
    from paper_2102_08514_amd import _lib as Lb
    given = None
    X = None
    mark = lambda marks, k: marks[k].record() if marks else None  # noqa: E731
    if args.config == "c3":
        W_, H_ = cfg.extra["rays"]
        S_ = cfg.extra["steps"]
        c, A = I.ray_params(cfg)
        n = W_ * H_ * S_
        cf, Af = c.astype(np.float32), A.astype(np.float32)
        phases = ["rays"]

        if args.render:
            # mostly transparent transfer function: every ray crosses the whole volume
            tfv = torch.tensor([[0.1, 0.2, 0.9, 0.0], [0.2, 0.8, 0.3, 0.004], [0.9, 0.7, 0.1, 0.008],
                                [1.0, 0.2, 0.1, 0.012]], device="cuda")
            phases = ["render"]

            def step(marks, sched=None):
                sp.render(vol, cf, Af, W_, H_, S_, tfv, -0.5, 0.5, alpha_stop=2.0)
            kernels = "k_render"
        else:
            def step(marks, sched=None):
                sp.rays(vol, cf, Af, W_, H_, S_)
            kernels = "k_rays"
        bytes_per = Lq * bytes_c + 16.0 / S_                     # coefficients + per-ray output
    else:
        X = I.queries(cfg)
        n = len(X)
        x = torch.from_numpy(X).cuda()
        f = torch.empty(n, device="cuda", dtype=vol.out_dtype)
        ws_bytes = Lb.lsp_schedule_size(sp.plan, vol.handle, n)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        use_sched = args.order == "sorted"
        if cfg.passes == "mse":
            y = torch.from_numpy(I.targets(cfg, X)).cuda()
            loss = torch.zeros(1, device="cuda", dtype=torch.float64)
            dldf = torch.empty(n, device="cuda")
            gradc = [torch.zeros(c.shape, device="cuda") for c in dev]
            gx = torch.empty(n, s, device="cuda")
            phases = ["schedule", "forward", "backward"]

            def step(marks, sched=use_sched, want_f=False):
                if sched:
                    Lb.lsp_schedule(sp.plan, vol.handle, x.data_ptr(), n, ws.data_ptr(), ws_bytes, strm)
                mark(marks, 0)
                loss.zero_()
                # forward: L, dL/df and dL/dx (f itself is not stored: the step needs only the loss and
                # the gradients); backward: dL/dc (scatter-add into zeroed arrays)
                fo = f.data_ptr() if want_f else None
                if sched:
                    # dL/df stays in the workspace, in schedule order, for the fused backward
                    Lb.lsp_eval_mse_scheduled(sp.plan, vol.handle, x.data_ptr(), y.data_ptr(), n, ws.data_ptr(),
                                              ws_bytes, fo, None, gx.data_ptr(), loss.data_ptr(), strm)
                else:
                    Lb.lsp_eval_mse(sp.plan, vol.handle, x.data_ptr(), y.data_ptr(), n, fo, dldf.data_ptr(),
                                    gx.data_ptr(), loss.data_ptr(), strm)
                mark(marks, 1)
                for g in gradc:
                    g.zero_()
                if sched:
                    Lb.lsp_mse_backward_scheduled(sp.plan, vol.handle, x.data_ptr(), n, ws.data_ptr(), ws_bytes,
                                                  [g.data_ptr() for g in gradc], strm)
                else:
                    Lb.lsp_eval_adjoint(sp.plan, vol.handle, x.data_ptr(), dldf.data_ptr(), n,
                                        [g.data_ptr() for g in gradc], None, strm)
            # fwd: x + y + coefficients + dL/df + dL/dx; bwd: x + dL/df + scatter (4 B per site)
            bytes_fwd = 4 * s + 4 + Lq * bytes_c + 4 + 4 * s
            bytes_bwd = 4 * s + 4 + Lq * 4
            bytes_per = bytes_fwd + bytes_bwd
            kernels = "forward + backward kernels (MSE forward with dL/dx, adjoint scatter)"
        else:
            phases = ["schedule", "forward"]

            def step(marks, sched=use_sched):
                if sched:
                    Lb.lsp_schedule(sp.plan, vol.handle, x.data_ptr(), n, ws.data_ptr(), ws_bytes, strm)
                mark(marks, 0)
                if sched:
                    Lb.lsp_eval_scheduled(sp.plan, vol.handle, x.data_ptr(), n, ws.data_ptr(), ws_bytes,
                                          f.data_ptr(), None, strm)
                else:
                    Lb.lsp_eval(sp.plan, vol.handle, x.data_ptr(), n, f.data_ptr(), None, strm)
            bytes_per = 4 * s + Lq * bytes_c + out_b
            kernels = "k_eval_binned" if use_sched else "k_eval"
        if use_sched and not args.no_extra:
            # context: the same step on the queries in their given order
            k = max(3, args.steps // 4)
            gw, _, _ = time_phases(lambda marks: step(marks, sched=False), k, 1, torch, nmarks=len(phases) - 1)
            given = {"ms_per_step": round(gw / k * 1e3, 4), "value": round(n / (gw / k) / 1e9, 4)}
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps after {args.warmup} warm-up")
    nm = len(phases) - 1
    wall, pmean, pmed = time_phases(step, args.steps, args.warmup, torch, nmarks=nm)
    ms_per_step = wall / args.steps * 1e3
    value = n / (wall / args.steps) / 1e9
    # the roofline covers everything after the schedule: the evaluation kernels
    ev_mean = float(pmean[1:].sum()) if nm else float(pmean[0])
    ev_med = float(pmed[1:].sum()) if nm else float(pmed[0])
    achieved = bytes_per * n / ev_mean / 1e9
    traffic = measured_traffic(args.config, dname)
    # compulsory floor: the coefficient volume once, the queries once, the outputs once
    vol_bytes = sum(int(np.prod(c.shape)) for c in dev) * bytes_c
    if X is None:
        compulsory = vol_bytes + (W_ * H_) * 16
    elif cfg.passes == "mse":
        compulsory = vol_bytes + n * (4 * s + 4 + 4 + 4 * s) + sum(int(np.prod(c.shape)) for c in dev) * 4
    else:
        compulsory = vol_bytes + n * (4 * s + out_b)
    rec = {
        "metric": "Gsamples/s fwd and fwd+bwd at stated max err vs FP64 oracle; % HBM roofline",
        "value": round(value, 4),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "bf16 storage, f32 math", "f16": "f16 storage, f32 math",
                  "f64": "f64"}[dname],
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "spline": info["name"],
                   "n_samples": n, "lookups_per_sample": Lq, "volume_dims": list(cfg.dims),
                   "n_cosets": cfg.M, "passes": cfg.passes,
                   "order": ("render" if args.render else "rays") if X is None else args.order},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else traffic["bytes_per_launch"],
                     "kernel": kernels, "algorithmic_bytes_per_sample": round(bytes_per, 3),
                     "samples_per_launch": n, "compulsory_bytes": int(compulsory),
                     "compulsory_floor_ms": round(compulsory / (HBM_PEAK_GBS * 1e9) * 1e3, 4),
                     "eval_ms_mean": round(ev_mean * 1e3, 4), "eval_ms_median": round(ev_med * 1e3, 4)},
        "phases_ms_mean": {p: round(float(v) * 1e3, 4) for p, v in zip(phases, pmean)},
        "kernel_source_digest": kernel_source_digest(),
    }
    if traffic is not None:
        rec["roofline"]["traffic_source"] = traffic["source"]
        rec["roofline"]["traffic_kernel"] = traffic["kernel"]
    if cfg.passes == "mse":
        t_sched, t_fwd, t_bwd = (float(v) for v in pmean)
        rec["forward_only"] = {"value": round(n / (t_sched + t_fwd) / 1e9, 4), "unit": "Gsamples/s",
                               "note": "schedule + forward phases of the same timed steps"}
        rec["fwd_bwd_over_fwd"] = round((t_sched + t_fwd + t_bwd) / (t_sched + t_fwd), 3)
    if given is not None:
        rec["given_order"] = given
    if not args.no_extra:
        # cold cache: a 1 GiB write evicts the 256 MB MALL and every L2 before each step
        junk = torch.empty(1 << 28, device="cuda")
        k = max(3, args.steps // 4)
        cw, cmean, _ = time_phases(step, k, 1, torch, nmarks=nm, flush=lambda: junk.fill_(1.0))
        rec["cold_cache"] = {"ms_per_step": round(cw / k * 1e3, 4), "value": round(n / (cw / k) / 1e9, 4)}
        del junk
        rec["roofline"]["copy_gbs"] = round(copy_bandwidth(torch), 1)
    if not args.no_cpu and X is not None:
        if cfg.passes == "mse":
            step(None, want_f=True)        # untimed: store f for the accuracy check
            torch.cuda.synchronize()
        log("[bench] CPU oracle leg")
        cb, idx, want = cpu_baseline(args.config, coeffs if tdt != torch.float32 else
                                     [c.astype(np.float32) for c in coeffs], X)
        rec["cpu_baseline"] = cb
        got = f[:len(idx)].double().cpu().numpy()
        scale = max(float(np.abs(c).max()) for c in coeffs)
        err = np.abs(got - want) / scale
        rec["accuracy"] = {"max_err": float(err.max()), "rms_err": float(np.sqrt(np.mean(err ** 2))),
                           "norm": "|f - f_oracle| / max|c|", "n": int(len(idx))}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
