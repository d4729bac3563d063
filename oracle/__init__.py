"""FP64 CPU oracle of the axisymmetric charge-conserving EM-PIC step.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or calls
this package; only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark may.  It shares no code with the GPU library: the setup
(incidence, Hodge matrices, SPAI, stability limit) is plain numpy/scipy and
the per-step loop is plain C (``pic_step.c``, built by ``build_oracle``).

Every function cites the part of the paper it follows: Na, Omelchenko, Moon,
Borges, Teixeira, "Axisymmetric charge-conservative electromagnetic particle
simulation algorithm on unstructured grids" (arXiv:1701.03784).

Readings of the paper where it is silent, ambiguous or garbled:
  * meridian frame (x, y) := (z, rho); faces counter-clockwise there, so a
    face value is the flux of B_phi (Sec. 2.2, eq. for B as B_phi dz^drho);
  * edge current is (q/dt) * line integral of the Whitney 1-form along the
    path, i.e. (q/dt)(lam_t^n lam_h^{n+1} - lam_h^n lam_t^{n+1}) with
    t < h; the printed eq. (current) has the opposite sign of its own
    DCE derivation (Sec. 3.5.1), and only this sign satisfies the DCE with
    the divergence incidence of App. D;
  * ring sources carry charge and current per radian (q / 2 pi);
  * the App. B local entry T22 is garbled; Hodge entries are computed by
    exact barycentric quadrature of their defining integral instead;
  * SPAI pattern, drop rule and symmetrisation are not given (Sec. 3.1);
    level-L pattern of the Jacobi-scaled matrix, relative drop tolerance,
    symmetric average;
  * the corrected Boris algorithm of Sec. 3.3 is the relativistic Boris rotation
    with gamma taken from the half-accelerated momentum; the axisymmetric
    position update pushes in the local Cartesian frame and rotates back.
"""

from .topology import Topology, build_topology  # noqa: F401
from .hodge import hodge_eps, hodge_mu_inv, whitney2_value  # noqa: F401
from .spai import spai, spai_pattern, spai_residuals  # noqa: F401
from .cfl import cfl_dt, curl_curl  # noqa: F401
