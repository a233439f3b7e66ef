"""Plain FP64 CPU oracle of the MLVS-DUGKS hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
CPU-baseline leg of the benchmark may import or call anything in this
package; the product path (the HIP library and its Python binding) never
does.  It shares no code with the GPU path: its quadrature, equilibria,
moments, corrections, criterion, clustering, projection and DUGKS step are
written here from the paper's definitions, step by step, with numpy arrays
over the velocity axis and Python loops over cells and faces.

Modules and what they follow (sections / equations of the paper):
  quadrature  discrete velocity sets (Sec. 2.3: Newton-Cotes on a uniform
              Cartesian grid; Gauss-Hermite as an alternative rule)
  kinetic     BGK-Shakhov reduced equilibria (Eq. g_h_eq_Pr), discrete
              moments (Eqs. discrete_W, discrete_q), the linear
              moment-constrained compatibility correction (Sec. 3.3.1,
              Eqs. gh_model_correction ... eq_four_moment_constraint, and the
              eight-moment variant, Eq. eq_eight_moment_constraint)
  mesh        structured finite-volume geometry
  levels      quadtree blocks and representative levels (Sec. 3.2),
              hierarchical projection (Sec. 3.3.2, Eqs. mapping_g_projection
              .. mapping_h_projection), mapping corrections (Eqs.
              mapping_four_targets .. raw_four_gh_coupling, nine-moment
              Eqs. mapping_nine_targets .. mapping_h_residual_correction),
              criterion (Eqs. M2, block-contribution-indicator,
              block-hysteresis-rule, merge-transport-error,
              combined-merge-condition), clustering (graded distance,
              leader clustering, enclosing mask)
  solver      the DUGKS step (Sec. 2.2, Eqs. phi_update .. recover_phi) on
              uniform and multi-level velocity spaces with the inter-level
              coupling of Sec. 3.4 (Eqs. level_switch_conservation,
              interface_state_moment_matching, interface_reduced_fluxes,
              native_flux_moment_matching)
  mlp         the learned level selector's network (plain loops)
"""
