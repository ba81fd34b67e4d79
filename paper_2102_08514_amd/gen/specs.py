"""The splines the library ships tables for.

Box splines: (struct name, lattice matrix L, direction matrix Xi).
Voronoi splines (Sec. 3): (struct name, L, VoronoiSpec(L_v, generators W,
sigma, n)) for phi = |det L| V_n of the Voronoi cell of L_v, a zonotope
sum_j [-1/2, 1/2] W_j / sigma (checked when the tables are built).
"""

from collections import namedtuple

VoronoiSpec = namedtuple("VoronoiSpec", "Lv W sigma n")

I3 = [[1, 0, 0], [0, 1, 0], [0, 0, 1]]
BCC_DIAG = [[-1, 1, 1, -1], [1, -1, 1, -1], [1, 1, -1, -1]]
HAD4 = [[1, 1, 1, 1], [1, 1, -1, -1], [1, -1, 1, -1], [1, -1, -1, 1]]


def _hcat(*ms):
    return [sum((list(m[r]) for m in ms), []) for r in range(len(ms[0]))]


def _scale(m, k):
    return [[k * v for v in row] for row in m]


L_CC = I3
L_BCC = [[-1, 1, 1], [1, -1, 1], [1, 1, -1]]
L_FCC = [[0, 1, 1], [1, 0, 1], [1, 1, 0]]
L_D4S = [[2, 0, 0, 1], [0, 2, 0, 1], [0, 0, 2, 1], [0, 0, 0, 1]]
# the D4 lattice and its 8-direction spline of Sec. 5.2 (columns (+-1, +-1, +-1, 1))
L_D4 = [[-1, 0, 0, 0], [1, 0, -1, -1], [0, -1, 0, 1], [0, -1, 1, 0]]
XI_D4 = [[1, 1, 1, 1, -1, -1, -1, -1], [1, 1, -1, -1, 1, 1, -1, -1], [1, -1, 1, -1, 1, -1, 1, -1],
         [1, 1, 1, 1, 1, 1, 1, 1]]
I4 = [[int(a == b) for b in range(4)] for a in range(4)]
HAD4_COLS = [list(r) for r in zip(*HAD4)]  # columns of the Hadamard matrix as rows

# Voronoi cells: the truncated octahedron of BCC and the rhombic dodecahedron of FCC
W_BCC_CELL = [(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)]
W_FCC_CELL = [(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]

SPECS = {
    # name: (struct name, L, Xi)
    "bcc_linear": ("SplineBccLinear", L_BCC, BCC_DIAG),
    "cc_zp": ("SplineCcZp", L_CC, _hcat(I3, BCC_DIAG)),
    "bcc_quartic": ("SplineBccQuartic", L_BCC, _hcat(_scale(I3, 2), BCC_DIAG)),
    "fcc_6dir": ("SplineFcc6", L_FCC, [[1, -1, 1, 1, 0, 0], [1, 1, 0, 0, 1, -1], [0, 0, 1, -1, 1, 1]]),
    "d4s_8dir": ("SplineD4s8", L_D4S, _hcat(_scale(I4, 2), [list(r) for r in zip(*HAD4_COLS)])),
    "d4_8dir": ("SplineD48", L_D4, XI_D4),
    # the remaining box-spline rows of Table 1
    "cc_tp2": ("SplineCcTp2", L_CC, _hcat(I3, I3)),
    "cc_tp3": ("SplineCcTp3", L_CC, _hcat(I3, I3, I3)),
    "cc_tp4": ("SplineCcTp4", L_CC, _hcat(I3, I3, I3, I3)),
    "cc_linear_rd": ("SplineCcLinearRd", L_CC, BCC_DIAG),
    "bcc_quintic_rd": ("SplineBccQuinticRd", L_BCC, _hcat(BCC_DIAG, BCC_DIAG)),
    # Voronoi splines (Table 1 Voronoi rows)
    "bcc_voronoi1": ("SplineBccVoronoi1", L_BCC, VoronoiSpec(L_BCC, W_BCC_CELL, 2, 1)),
    "fcc_voronoi1": ("SplineFccVoronoi1", L_FCC, VoronoiSpec(L_FCC, W_FCC_CELL, 2, 1)),
    "cc_bcc_voronoi1": ("SplineCcBccVoronoi1", L_CC, VoronoiSpec(L_BCC, W_BCC_CELL, 2, 1)),
    "cc_fcc_voronoi1": ("SplineCcFccVoronoi1", L_CC, VoronoiSpec(L_FCC, W_FCC_CELL, 2, 1)),
    "fcc_voronoi2": ("SplineFccVoronoi2", L_FCC, VoronoiSpec(L_FCC, W_FCC_CELL, 2, 2)),
    "cc_fcc_voronoi2": ("SplineCcFccVoronoi2", L_CC, VoronoiSpec(L_FCC, W_FCC_CELL, 2, 2)),
}


def make_tables(name):
    """Run the analysis for a shipped spline."""
    from .analysis import SplineTables
    from .phi import VoronoiPhi
    _, L, what = SPECS[name]
    if isinstance(what, VoronoiSpec):
        return SplineTables(name, L, phi=VoronoiPhi(L, what.Lv, what.W, what.sigma, what.n))
    return SplineTables(name, L, what)
