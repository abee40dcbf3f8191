"""CPU FP64 oracle for the lattice strong-coupling Dyson solve (arXiv:1309.5994).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library (no kernels, headers, helpers or tables); the two meet only
through the seeded inputs that ``paper_1309_5994_amd.workloads`` generates,
and that module holds none of the method's arithmetic.

What it computes (plain, slow, obviously correct, complex128 throughout):

* ``contour``     -- the discretised Kadanoff-Baym-Keldysh contour (Sec. IV.A,
                     Fig. 1) with the quadrature weights +dt, -dt, -i dtau.
* ``atomic``      -- the on-site no-hopping contour Green's function of each
                     site (Sec. III, the number-basis evaluation with the
                     tabulated phases zeta_nu), in closed form and by a
                     brute-force 4x4 Fock-space trace.
* ``lattice``     -- nearest-neighbour table and the hopping operator
                     (Sec. IV.D, eq. Ginvblockstruct: contour-delta in time,
                     tight-binding in space).
* ``dyson``       -- G = (I - S D)^-1 S by dense LU (eq. Glatt with the
                     block-diagonal B = S^-1 of eq. blockdiagdysonelement at
                     lowest order), selected columns by exact block-tridiagonal
                     elimination in lattice rows, and Neumann partial sums
                     (App. C, the Dyson-series view).
* ``gmres``       -- preconditioned restarted GMRES per unit-vector column
                     (App. C), the paper's own solver for the same system.
* ``selfenergy``  -- the second-order strong-coupling self-energy (Sec. III):
                     Fock-space two-particle propagator, cumulant, Sigma~,
                     dressed blocks and the mixed self-consistency loop.
* ``observables`` -- occupancy, kinetic energy and double occupancy (Sec. III.A,
                     eq. docc with the derivative of App. B), the doubly
                     occupied fraction (Sec. V.B) and dt -> 0 extrapolation.
* ``gradients``   -- dense adjoint formulas for d(sum_i w_i n_i(t_end)).

Pins (tests/test_oracle_*.py, run with ``-m "not gpu"``) tie every function to
something other than itself: the Fock-space trace, contour normalisation and
KMS identities, the J=0 and two-site closed forms, the per-momentum solution of
translation-invariant lattices, the U=0 free-fermion propagator (which fixes
the contour conventions), C4v symmetry and the Dyson-series light cone.
Where the paper is silent, each module states the reading it takes.
"""
from .contour import Contour, make_contour
from .atomic import atomic_gf, atomic_gf_fock, boltzmann_weights, level_phases
from .lattice import neighbours, hopping_on_contour, hopping_operator_dense
from .dyson import (blockdiag, dyson_dense, dyson_columns_blocktri,
                    neumann_partial_sums, dense_system_matrix, dyson_columns_truncated,
                    lattice_distance)
from .gmres import gmres_column, gmres_dense
from . import selfenergy
from .observables import (occupancy, kinetic_energy, double_occupancy,
                          doubly_occupied_fraction, extrapolate_dt)
from .gradients import (loss_and_grad_dense, loss_dense, site_levels,
                        atomic_gf_derivatives)
from .observables import local_blocks_from_dense, neighbour_blocks_from_dense

__all__ = [
    "Contour", "make_contour",
    "atomic_gf", "atomic_gf_fock", "boltzmann_weights", "level_phases",
    "neighbours", "hopping_on_contour", "hopping_operator_dense",
    "blockdiag", "dyson_dense", "dyson_columns_blocktri",
    "neumann_partial_sums", "dense_system_matrix", "gmres_column", "gmres_dense",
    "dyson_columns_truncated", "lattice_distance",
    "occupancy", "kinetic_energy", "double_occupancy", "doubly_occupied_fraction",
    "extrapolate_dt", "loss_and_grad_dense", "loss_dense",
    "site_levels", "atomic_gf_derivatives",
    "local_blocks_from_dense", "neighbour_blocks_from_dense",
]
