"""Load generated tables back from their exact JSON record.

`LoadedTables` exposes the same attributes as the analysis object that
produced the record, so the interpreter and the header emitter work on
either.
"""

import json
import os
from fractions import Fraction

from .poly import Poly

GENERATED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "csrc", "generated")


class _Lat:
    def __init__(self, L, shifts, det, D):
        self.L = L
        self.shifts = [tuple(v) for v in shifts]
        self.det = det
        self.M = len(shifts)
        self.D = D


class LoadedTables:
    def __init__(self, record):
        r = record
        self.name = r["name"]
        self.s = r["s"]
        self.Xi_rows = r["Xi"]
        self.n = len(r["Xi"][0])
        self.cols = [tuple(r["Xi"][a][j] for a in range(self.s)) for j in range(self.n)]
        self.D = r["D"]
        self.lat = _Lat(r["L"], r["shifts"], r["det"], r["D"])
        self.fold = r["fold"]
        self.degree = r["degree"]
        self.order = r["order"]
        self.planes = [(tuple(nu), Fraction(off)) for nu, off in r["planes"]]
        self.orbit_table = list(r["orbit_table"])
        self.sigma = r.get("sigma")
        self.voronoi = r.get("voronoi")
        self._mons = [tuple(e) for e in r["monomials"]]
        self._A = [[[Fraction(v) for v in row] for row in o["A"]] for o in r["orbits"]]
        self.orbits = []
        for o, A in zip(r["orbits"], self._A):
            polys = []
            for row in A:
                polys.append(Poly(self.s, {e: v for e, v in zip(self._mons, row) if v != 0}))
            self.orbits.append({"stencil": [tuple(j) for j in o["stencil"]], "polys": polys})
        self.K = len(self.orbits)

    def monomials(self):
        return list(self._mons)

    def coefficient_matrix(self, k):
        return [list(row) for row in self._A[k]]

    def lookups_per_coset(self):
        return [len(o["stencil"]) for o in self.orbits]


def load(name, directory=GENERATED):
    with open(os.path.join(directory, f"{name}.json")) as fh:
        return LoadedTables(json.load(fh))
