"""Oracle: plain, slow, FP64 CPU implementation of the method.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product library
(``paper_1810_03358_amd``) never imports it, links it or calls it, and it
shares no code with the HIP path.

* ``energy`` (C, ``ff_oracle.c``): the section-2 energy and its analytic
  gradient, term by term in double precision.
* ``minimize`` (Python): the line searches LS_H and LS_PAR (section 5.2,
  Algorithms 5 and 6) and the methods GD (steepest descent with a line search,
  eq. 4), FGM (Algorithm 1), CG (Algorithm 2, Polak-Ribiere-Polyak beta of
  section 4) and L-BFGS (Algorithms 3 and 4), heavy ball (eq. HB) and the
  optimized gradient method (eq. optim), in the paper's order and notation.
* ``learn`` (numpy): the learned warm start, which is not in the paper: BF16
  rounding, 16-nearest-neighbour features, the 3-layer network, its loss
  gradient and Adam, by their definitions.
"""
from . import learn  # noqa: F401
from .energy import (System, energy_grad, energy_terms, atom_gradients, num_threads, build,  # noqa: F401
                     energy_profile, abs_pair_force, set_num_threads)
from .minimize import (  # noqa: F401
    MinParams, MinResult, minimize, ls_par, ls_h, lbfgs_direction, fgm_coefficients, ogm_t_next,
    GD, FGM, CG, LBFGS, HB, OGM, LS_PAR, LS_H, cg_beta,
    CG_PRP, CG_FR, CG_HS, CG_PRP_PLUS, CG_CD, CG_LS, CG_DY,
    CONVERGED, MAX_ITER, LS_FAILED, NONFINITE_START, DIVERGED,
)
