"""Reference oracle for the lattice convolution sum with box-spline bases.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the GPU path.

What it computes (Horacsek & Alim, "Automatic Generation of Interpolants for
Lattice Samplings: Part I"):

* the box spline M_Xi of a direction matrix Xi (Sec. 3, box-spline
  definition), evaluated by the de Boor--Hoellig recurrence with a single
  global symbolic perturbation that decides every point lying on a mesh
  plane consistently (Sec. 2 notes that decisions on separating planes must
  be consistent);
* the convolution sum f(x) = sum_n c_n phi(x - n) over every lattice site
  n in the support (Eq. conv_sum and its per-coset form, Eq. coset_form),
  with phi = |det L| M_Xi(. + c0) centred at the origin (c0 = half the sum
  of the directions) so that phi has partition of unity on the lattice
  (the requirement stated in Sec. 4.1);
* its spatial gradient and the adjoint (transpose) of the map c -> f;
* Voronoi splines V_n (Sec. 3): V_1 from its definition as the overlap
  volume of the Voronoi cell with its translate, and any V_n through the
  paper's expansion into shifted box splines (``voronoi.py``).

Everything is FP64 (numpy); an exact mode in ``fractions.Fraction`` exists
for single points.
"""

from .boxspline import BoxSplineOracle  # noqa: F401
from .lattice import CosetLattice  # noqa: F401
from .convsum import ConvolutionSumOracle  # noqa: F401
from .voronoi import VoronoiSumOracle  # noqa: F401
