"""Plain FP64 CPU oracle for the explicit phase-field fracture step.

TEST INFRASTRUCTURE ONLY.  This package is imported by the test-suite, by the
package's smoke check and by the benchmark's CPU-baseline leg, and by nothing
else: the product path (the HIP library and its Python binding) never calls
it and shares no code with it.

It computes, slowly and in the order the paper states them (Sec. 2.1-2.4,
Sec. 4.2), one staggered step of explicit phase-field fracture on a P1
triangle mesh:

* P1 geometry and lumped mass (eq. grad_phi; Sec. 2.3, velocity-Verlet paragraph),
* small strain, the energy splits (eq. spectral_split, eq. amor_split, the
  star-convex variant), degradation g(d) and stress (Sec. 2.1-2.2),
* element forces scattered into the internal force, velocity-Verlet
  predictor/corrector (eq. vv_u, vv_a, vv_v) and the history maximum,
* the damage update as the exact minimiser of the quadratic programme of
  the AT1/AT2 weak form (eq. damage_pde_at2, eq. damage_pde_at1,
  consistent mass of Sec. 2.4) over d_n <= d <= 1, solved by a primal-dual
  active-set method with sparse LU,
* energies and, by forward-mode differentiation of the whole trajectory, the
  derivative of the final-damage loss (eq. inversion_loss) with respect to
  G_c, using the implicit rule of Sec. 4.2 for the damage solve.

Every function is FP64.  Pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py``.
"""
from .constitutive import elastic_constants, split_energy
from .fem import (Mesh, cfl_dt, element_strain, internal_force, lumped_mass, make_mesh)
from .damage import (DamageQP, assemble_damage, energies, kkt_residuals, solve_bound_qp, solve_box_qp,
                     stiffness_matrix, mass_matrix)
from .step import Material, State, explicit_step, initial_state, run, staggered_step, loss_and_grad

__all__ = ["elastic_constants", "split_energy", "Mesh", "cfl_dt", "element_strain", "internal_force",
           "lumped_mass", "make_mesh", "DamageQP", "assemble_damage", "energies", "kkt_residuals",
           "solve_bound_qp", "solve_box_qp", "stiffness_matrix", "mass_matrix", "Material", "State", "explicit_step",
           "initial_state", "run", "staggered_step", "loss_and_grad"]
