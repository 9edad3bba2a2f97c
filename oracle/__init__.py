"""CPU oracle for the exponential-midpoint / Krylov time evolution of the
Peierls-driven Hubbard model (arXiv:2005.13498).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It is a plain, slow, obviously-correct FP64
implementation written from the paper, sharing no code, tables or helpers
with the HIP library.

Conventions (each follows the passage cited in the module that implements it):
  * modes are ordered as in Eq. (statedef): (site 0, up), (site 0, down),
    (site 1, up), ...; bit 2*i of a basis-state integer is n_{i,up} and bit
    2*i+1 is n_{i,down};
  * ladder operators act as in Eq. (creation-annihilation), with the sign
    exponent counting the occupied modes strictly before the acted-on mode;
  * the Hamiltonian is Eq. (hubbardhamiltonian) with the Peierls phase of
    Eq. (peierls): each directed hop j -> i carries -t_ij exp(i A(t) dx_ij),
    dx_ij = (R_i - R_j) projected on the field;
  * the stepper is Eq. (time-stepping), each exponential evaluated to machine
    precision; the literal Krylov step of Alg. 6 is in `krylov`.
"""
from .fock import (mode_index, sector_states, apply_ladder, ladder_matrix,
                   popcount, docc_weights)
from .hamiltonian import HubbardOracle, pulse_A
from .stepper import (midpoint_step_exact, propagate_exact, ground_state,
                      observables)
from .krylov import krylov_step_alg6, tridiag_expm_e1
from .canonical import canonical_map, to_canonical, from_canonical

__all__ = [
    "mode_index", "sector_states", "apply_ladder", "ladder_matrix", "popcount",
    "docc_weights", "HubbardOracle", "pulse_A", "midpoint_step_exact",
    "propagate_exact", "ground_state", "observables", "krylov_step_alg6",
    "tridiag_expm_e1", "canonical_map", "to_canonical", "from_canonical",
]
