"""FP64 CPU oracle for the exact two-electron split-step Fourier propagation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the HIP path: the two see the
same inputs (from the ``workloads`` generator) and nothing else.

It is deliberately plain and slow: numpy/scipy in float64/complex128, full 4D
arrays, the paper's 2D transforms over particle-coordinate pairs, and the
factors applied literally one after the other (no merging of half steps).

Source: L. Bellentani, P. Bordone, X. Oriols, A. Bertoni, arXiv 1903.02581,
Sec. II.C Eq. (evoloperat) and Appendix A (split-step Fourier method for two
particles), Sec. III Eq. (p_bunching) (bunching probability), Sec. II.A Eq. (H_effective)
and Sec. II.B Eq. (singlepwp) (edge states and edge-state wave packets), Sec. III.B
Eq. (coulomb) and Eq. (screenedCoulomb), Sec. III.C Eq. (reduced_density)
(spatial entanglement).

Pins: every function here is checked in tests/test_oracle_pins.py (the edge
states in tests/test_oracle_edge.py) against closed forms, invariants, dense
matrix exponentials or finite differences.
Parity status per function is listed in each module docstring.
"""
from .splitstep import (Grid, make_grid, theta_x, theta_y, theta_v, apply_x, apply_y,  # noqa
                        apply_v, strang_step, propagate, init_state, propagate_2d,
                        strang_step_2d)
from .observables import (observables, entanglement, region_weights_4d, marginal, conditional,  # noqa
                          orbital_observables)
from .adjoint import loss_and_grad_stored, grad_fd  # noqa
from .edge_states import lowest_edge_states, edge_packet  # noqa
