"""Write tests/golden/voronoi_expected.npz: FP64 oracle values for the GPU
parity tests of the Voronoi splines.

Inputs are regenerated from seeds by `tests/gpu_cases.small_case` (the same
builder the GPU tests call); every stored value comes from `oracle/` alone:

    f, grad         the oracle at the float32 queries, unrounded coefficients
    f_bf16          the oracle on the coefficients rounded to bfloat16
                    (round to nearest even, as the device conversion does)
    adj             the adjoint sum_q g_q phi(x_q - m) for seeded g
    adj_abs         the same for |g| (the tolerance scale of the adjoint)

    python tests/golden/make_voronoi_expected.py      (minutes, all cores)
"""

import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

NAMES = ["vor_bcc1", "vor_fcc1", "vor_cc_bcc1", "vor_cc_fcc1", "vor_fcc2", "vor_cc_fcc2"]
OUT = os.path.join(HERE, "voronoi_expected.npz")


def job(args):
    name, part = args
    from gpu_cases import SMALL, bf16_round, small_case, voronoi_oracle
    from workloads import configs as W
    cfg, coeffs, X = small_case(name)
    o = voronoi_oracle(cfg)
    X64 = X.astype(np.float64)
    if part == "f":
        f, g = o.eval(coeffs, X64, want_grad=True)
        return {"f": f, "grad": g}
    if part == "bf16":
        return {"f_bf16": o.eval([bf16_round(c) for c in coeffs], X64)}
    g = np.random.default_rng(5).normal(size=len(X))
    dims = SMALL[name]
    return {"adj": np.stack(o.adjoint(X64, g, dims)), "adj_abs": np.stack(o.adjoint(X64, np.abs(g), dims))}


def main(names=None):
    """Regenerate the given workloads (all by default), keeping the others'
    stored values."""
    names = names or NAMES
    jobs = [(n, p) for n in names for p in ("f", "bf16", "adj")]
    with Pool(min(len(jobs), os.cpu_count() or 1)) as pool:
        res = pool.map(job, jobs)
    out = {}
    if os.path.exists(OUT):
        with np.load(OUT, allow_pickle=False) as z:
            out = {k: z[k] for k in z.files if k.split("/")[0] not in names}
    for (name, _), r in zip(jobs, res):
        for k, v in r.items():
            out[f"{name}/{k}"] = np.asarray(v, dtype=np.float64)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT, sorted(out))


if __name__ == "__main__":
    main(sys.argv[1:])
