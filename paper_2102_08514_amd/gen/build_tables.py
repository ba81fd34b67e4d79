"""Regenerate the committed tables under csrc/generated/ (offline, exact).

    python -m paper_2102_08514_amd.gen.build_tables [name ...]

Each spline takes seconds to minutes (the 4-D one about four minutes).
"""

import os
import sys
import time

from .emit import write
from .specs import SPECS, make_tables

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "csrc", "generated")


def reemit(names):
    """Rewrite the headers from the committed exact JSON records (no analysis)."""
    from .emit import emit_header
    from .tables import load
    import hashlib
    for name in names or list(SPECS):
        t = load(name, OUT)
        with open(os.path.join(OUT, f"{name}.json")) as fh:
            blob = fh.read()
        digest = hashlib.sha256(blob.encode()).hexdigest()[:16]
        with open(os.path.join(OUT, f"{name}.inc"), "w") as fh:
            fh.write(f"// table digest {digest}\n" + emit_header(t, SPECS[name][0]))
        print(f"{name}: header rewritten", flush=True)


def main(names):
    if names and names[0] == "--reemit":
        return reemit(names[1:])
    for name in names or list(SPECS):
        struct = SPECS[name][0]
        t0 = time.time()
        t = make_tables(name)
        t.verify()
        write(t, OUT, struct)
        print(f"{name}: K={t.K} Q={len(t.planes)} stencils={t.lookups_per_coset()} ({time.time() - t0:.1f} s)",
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
