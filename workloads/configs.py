"""The five workloads (lattice, direction matrix, sizes) the project is built around.

Lattices and splines are the ones of the paper's Table 1 (BCC linear rhombic
dodecahedron, the Cartesian truncated rhombic dodecahedron / ZP element, the
BCC quartic truncated rhombic dodecahedron, the FCC 6-direction truncated
octahedron) plus a 4-D spline on the D4* lattice in the spirit of Sec. 5.2.

Coefficient storage: coset k is an s-D array indexed by i (x fastest) holding
the value at lattice site D i + l_k; shifts are ordered by sum_a l_a D^a.
``lo``/``hi`` bound the queries so that every query's full support lies in
the stored arrays (the largest first stored coordinate over the cosets plus
the support half-width, and symmetrically at the top).
"""

from dataclasses import dataclass, field

import numpy as np

I3 = np.eye(3, dtype=np.int64)
BCC_DIAG = np.array([[-1, 1, 1, -1],
                     [1, -1, 1, -1],
                     [1, 1, -1, -1]], dtype=np.int64)          # the four BCC diagonals
HAD4 = np.array([[1, 1, 1, 1],
                 [1, 1, -1, -1],
                 [1, -1, 1, -1],
                 [1, -1, -1, 1]], dtype=np.int64).T            # Hadamard directions

L_CC = I3
L_BCC = np.array([[-1, 1, 1], [1, -1, 1], [1, 1, -1]], dtype=np.int64)
L_FCC = np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=np.int64)
# D4* realised as 2Z^4 u (2Z^4 + (1,1,1,1)): columns 2e_1, 2e_2, 2e_3, (1,1,1,1)
L_D4S = np.array([[2, 0, 0, 1], [0, 2, 0, 1], [0, 0, 2, 1], [0, 0, 0, 1]], dtype=np.int64)
# the paper's D4 generating matrix (Sec. 5.2)
L_D4 = np.array([[-1, 0, 0, 0], [1, 0, -1, -1], [0, -1, 0, 1], [0, -1, 1, 0]], dtype=np.int64)

XI_BCC_LINEAR = BCC_DIAG
XI_ZP = np.hstack([I3, BCC_DIAG])
XI_BCC_QUARTIC = np.hstack([2 * I3, BCC_DIAG])
XI_FCC6 = np.array([[1, -1, 1, 1, 0, 0],
                    [1, 1, 0, 0, 1, -1],
                    [0, 0, 1, -1, 1, 1]], dtype=np.int64)
XI_D4S8 = np.hstack([2 * np.eye(4, dtype=np.int64), HAD4])
# the paper's D4 spline (Sec. 5.2): the 8 directions (+-1, +-1, +-1, 1)
XI_D4 = np.array([[1, 1, 1, 1, -1, -1, -1, -1],
                  [1, 1, -1, -1, 1, 1, -1, -1],
                  [1, -1, 1, -1, 1, -1, 1, -1],
                  [1, 1, 1, 1, 1, 1, 1, 1]], dtype=np.int64)
# D4 = 2 Z^4 + the 8 shifts with an even coordinate sum, ordered by sum l_a 2^a
D4_SHIFTS = ((0, 0, 0, 0), (1, 1, 0, 0), (1, 0, 1, 0), (0, 1, 1, 0), (1, 0, 0, 1), (0, 1, 0, 1), (0, 0, 1, 1),
             (1, 1, 1, 1))


# Voronoi cells of the BCC and FCC lattices as zonotopes sum_j [-1/2, 1/2] g_j
# with g_j = w_j / 2 (truncated octahedron: 6 generators; rhombic
# dodecahedron: 4).  The oracle checks that each spans its lattice's cell.
VORONOI_SIGMA = 2
VORONOI_GEN = {
    "BCC": ((1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)),
    "FCC": ((1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)),
}
LATTICES = {"CC": L_CC, "BCC": L_BCC, "FCC": L_FCC}


@dataclass(frozen=True)
class Config:
    name: str
    title: str
    L: np.ndarray
    Xi: np.ndarray
    D: int
    shifts: tuple          # coset shifts l_k
    dims: tuple            # per-coset array dims (n_0, ..., n_{s-1})
    n_queries: int
    lo: float
    hi: float
    coeff_kind: str        # 'uniform' or 'field'
    noise: float = 0.0
    passes: str = "fwd"    # 'fwd', 'fwd+grad', 'mse'
    lookups: int = 0       # sites with nonzero weight per query (Table 1 column)
    extra: dict = field(default_factory=dict)
    voronoi: tuple = None  # (lattice of the Voronoi cell, n) for phi = |det L| V_n; Xi is None then

    @property
    def s(self):
        return self.L.shape[0]

    @property
    def Lv(self):
        return LATTICES[self.voronoi[0]] if self.voronoi else None

    @property
    def voronoi_gen(self):
        return VORONOI_GEN[self.voronoi[0]] if self.voronoi else None

    @property
    def M(self):
        return len(self.shifts)


def _z(s):
    return (0,) * s


CONFIGS = {
    "c1": Config("c1", "BCC 2x32^3, linear rhombic dodecahedron (4 dir.), FP64 coefficients, 1e5 queries, forward",
                 L_BCC, XI_BCC_LINEAR, 2, (_z(3), (1, 1, 1)), (32, 32, 32), 100000, 3.0, 60.0,
                 "uniform", lookups=4, extra={"coeff_dtype": "f64"}),
    "c2": Config("c2", "Z^3 256^3, 7-direction ZP box spline, FP32, 2^24 random queries, forward",
                 L_CC, XI_ZP, 1, (_z(3),), (256, 256, 256), 1 << 24, 2.5, 252.5,
                 "field", noise=0.01, lookups=53),
    "c3": Config("c3", "BCC 2x192^3, quartic 7-direction box spline, 1024^2 rays x 512 steps, forward + grad",
                 L_BCC, XI_BCC_QUARTIC, 2, (_z(3), (1, 1, 1)), (192, 192, 192), 1 << 29, 4.0, 379.0,
                 "field", noise=0.01, passes="fwd+grad", lookups=30,
                 extra={"rays": (1024, 1024), "steps": 512}),
    "c4": Config("c4", "FCC 4x128^3, 6-direction box spline, 2^22 queries, MSE forward + backward",
                 L_FCC, XI_FCC6, 2, (_z(3), (1, 1, 0), (1, 0, 1), (0, 1, 1)), (128, 128, 128), 1 << 22,
                 3.0, 252.0, "field", passes="mse", lookups=16),
    "c5": Config("c5", "D4* 2x48^4, 8-direction box spline, 2^22 queries, forward + backward",
                 L_D4S, XI_D4S8, 2, (_z(4), (1, 1, 1, 1)), (48, 48, 48, 48), 1 << 22, 4.0, 91.0,
                 "field", passes="mse", lookups=60),
    # the paper's own 4-D experiment (Sec. 5.2): 8 cosets, 240 lookups per query
    "d4": Config("d4", "D4 8x24^4, 8-direction box spline of Sec. 5.2, FP32, 2^22 queries, forward",
                 L_D4, XI_D4, 2, D4_SHIFTS, (24, 24, 24, 24), 1 << 22, 5.0, 42.0,
                 "field", lookups=240),
    # the remaining box-spline rows of Table 1 (parity cases)
    "cc_tp2": Config("cc_tp2", "Z^3 64^3, [I3 I3] (trilinear; Table 1 CC Voronoi 1)", L_CC, np.hstack([I3] * 2), 1,
                     (_z(3),), (64, 64, 64), 1 << 20, 1.0, 62.0, "uniform", lookups=8),
    "cc_tp3": Config("cc_tp3", "Z^3 64^3, [I3 I3 I3] (triquadratic; Table 1 CC Voronoi 2)", L_CC,
                     np.hstack([I3] * 3), 1, (_z(3),), (64, 64, 64), 1 << 20, 1.5, 61.5, "uniform", lookups=27),
    "cc_tp4": Config("cc_tp4", "Z^3 64^3, [I3 I3 I3 I3] (tricubic; Table 1 CC Voronoi 3)", L_CC,
                     np.hstack([I3] * 4), 1, (_z(3),), (64, 64, 64), 1 << 20, 2.0, 61.0, "uniform", lookups=64),
    "cc_linear_rd": Config("cc_linear_rd", "Z^3 64^3, the 4 BCC diagonals (Table 1 CC linear rhombic dodecahedron)",
                           L_CC, BCC_DIAG, 1, (_z(3),), (64, 64, 64), 1 << 20, 2.0, 61.0, "uniform", lookups=16),
    "bcc_quintic_rd": Config("bcc_quintic_rd", "BCC 2x32^3, the BCC diagonals twice (Table 1 quintic rhombic "
                             "dodecahedron)", L_BCC, np.hstack([BCC_DIAG] * 2), 2, (_z(3), (1, 1, 1)), (32, 32, 32),
                             1 << 20, 5.0, 58.0, "uniform", lookups=32),
    # Voronoi splines (Sec. 3; Table 1 Voronoi rows): phi = |det L| V_n of the BCC / FCC Voronoi cell
    "vor_bcc1": Config("vor_bcc1", "BCC 2x32^3, BCC Voronoi spline 1", L_BCC, None, 2, (_z(3), (1, 1, 1)),
                       (32, 32, 32), 1 << 20, 3.0, 60.0, "uniform", lookups=8, voronoi=("BCC", 1)),
    "vor_fcc1": Config("vor_fcc1", "FCC 4x32^3, FCC Voronoi spline 1", L_FCC, None, 2,
                       (_z(3), (1, 1, 0), (1, 0, 1), (0, 1, 1)), (32, 32, 32), 1 << 20, 3.0, 60.0, "uniform",
                       lookups=8, voronoi=("FCC", 1)),
    "vor_cc_bcc1": Config("vor_cc_bcc1", "Z^3 64^3, BCC Voronoi spline 1 on the Cartesian lattice", L_CC, None, 1,
                          (_z(3),), (64, 64, 64), 1 << 20, 2.0, 61.0, "uniform", lookups=32, voronoi=("BCC", 1)),
    "vor_cc_fcc1": Config("vor_cc_fcc1", "Z^3 64^3, FCC Voronoi spline 1 on the Cartesian lattice", L_CC, None, 1,
                          (_z(3),), (64, 64, 64), 1 << 20, 2.0, 61.0, "uniform", lookups=16, voronoi=("FCC", 1)),
    "vor_fcc2": Config("vor_fcc2", "FCC 4x32^3, FCC Voronoi spline 2", L_FCC, None, 2,
                       (_z(3), (1, 1, 0), (1, 0, 1), (0, 1, 1)), (32, 32, 32), 1 << 20, 4.0, 59.0, "uniform",
                       lookups=27, voronoi=("FCC", 2)),
    "vor_cc_fcc2": Config("vor_cc_fcc2", "Z^3 32^3, FCC Voronoi spline 2 on the Cartesian lattice", L_CC, None, 1,
                          (_z(3),), (32, 32, 32), 1 << 20, 3.0, 28.0, "uniform", lookups=54, voronoi=("FCC", 2)),
    # Voronoi splines at benchmark size: the c3 ray grid on a BCC volume, and
    # c4's FCC volume under random queries
    "vor_rays": Config("vor_rays", "BCC 2x192^3, BCC Voronoi spline 1, 1024x1024 rays x 512 steps, forward + grad",
                       L_BCC, None, 2, (_z(3), (1, 1, 1)), (192, 192, 192), 1 << 29, 4.0, 379.0,
                       "field", noise=0.01, passes="fwd+grad", lookups=8, extra={"rays": (1024, 1024), "steps": 512},
                       voronoi=("BCC", 1)),
    "vor_fcc": Config("vor_fcc", "FCC 4x128^3, FCC Voronoi spline 1, 2^22 random queries, forward",
                      L_FCC, None, 2, (_z(3), (1, 1, 0), (1, 0, 1), (0, 1, 1)), (128, 128, 128), 1 << 22,
                      3.0, 252.0, "field", lookups=8, voronoi=("FCC", 1)),
}


def get(name):
    return CONFIGS[name]
