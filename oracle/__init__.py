"""Plain FP64 CPU oracle for the Sternheimer chi0 apply.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it. It shares no code, tables or helpers with the GPU
library; it reads the same seeded inputs (atoms, fields, occupied states) and
maps plane-wave coefficients by their Miller indices, so it depends on no
ordering chosen elsewhere.

What it computes (the paper, Sec. II.A, only says that the density response
chi0 dV is obtained by solving the Sternheimer equation within DFPT; the
definitions below are the standard DFPT ones):

  for every occupied band v and field dV_i,
      P_c (H - eps_v) P_c x_{v,i} = -P_c dV_i psi_v,  x in range(P_c),
      P_c = 1 - sum_v |psi_v><psi_v|,
  solved by preconditioned CG (Teter-Payne-Allan diagonal, zero start), then
      dn_i(r) = 4 Re sum_v conj(psi_v(r)) x_{v,i}(r).

Modules:
  model        basis, local potential, KB projectors, H apply and dense H
  sternheimer  RHS, projected PCG, density response
  closed_form  sum over all empty states, finite field, free-electron Lindhard sum
  net          one training step of the learned-start net (forward, loss, gradients, Adam)
               in float64 over BF16-rounded values, for checking the net's kernels
  pdep         dense symmetrised response chi-bar0 in the real potential basis (PDEP)
  frequency    the response at imaginary frequency i u: sum over states, dense shifted
               solve, free-electron Lindhard sum at i u, residual of the shifted system
  liouville    TDDFT Liouville superoperator in the Tamm-Dancoff approximation (Hartree
               kernel, bare-exchange and screened direct terms): grid route, transition-basis
               matrix, free-electron matrix by hand, residual of the Z-vector system, Lanczos
               chain and spectra
  deflation    the Sternheimer solve with known lowest empty states taken out in closed form

Pins (tests/test_oracle_*.py) tie each function to something other than
itself: a brute-force lattice count, the real-space Gaussian sum, the dense
matrix, the sum over states from full diagonalisation, the finite-field
derivative of the density, the discrete Lindhard sum, and the Hermiticity,
negative semidefiniteness and charge conservation of chi0.
"""
from .model import OracleCell, fft_grid, sphere_miller
from .sternheimer import apply_chi0, project, rhs, teter, pcg_solve, delta_n, band_kinetic
from .closed_form import sum_over_states, finite_field_dn, lindhard_dn
