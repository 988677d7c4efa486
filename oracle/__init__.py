"""FP64 CPU oracle for the R-matrix outer-region energy sweep.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, the package's
``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may import,
call or execute anything in this directory.  The HIP library never links it and
the Python binding never falls back to it.

The oracle is a plain, slow, double-precision restatement of what the method
computes at each scattering energy E (McLaughlin & Ballance, "Petascale
computations for large-scale atomic and molecular collisions", Sec. 6, Eq. 1-2,
plus the standard R-matrix matching of Burke, "R-Matrix Theory of Atomic
Collisions", 2011, Ch. 2-3, for the steps the paper leaves implicit):

* ``rmatrix.r_matrix``            boundary R-matrix from poles (Eq. 1, as the
                                   product X*Y of Eq. 2)
* ``coulomb.open_channel_functions``  Coulomb F, G and derivatives at r = a
* ``coulomb.closed_channel_logderiv``  log-derivative of the decaying
                                   Whittaker function at r = a
* ``rmatrix.k_matrix``            matching of R to the asymptotic functions
* ``rmatrix.t_matrix``            T = 2iK (1 - iK)^-1
* ``rmatrix.collision_strengths`` Omega = sum (g/2) |T|^2 per target pair
* ``rmatrix.sweep``               all of the above over an energy mesh
* ``postproc.gaussian_convolve``  Omega(E) convolved with a Gaussian of given
                                   FWHM on the mesh (Sec. 4-5 figures)
* ``postproc.effective_collision_strengths``  Maxwellian averages Upsilon(kT)
* ``postproc.group_collision_strengths``  Omega summed over the level pairs of
                                   level groups (statistical averaging)
* ``photo.photoionization``       photoionization cross sections from the
                                   same solve and bound-free dipole vectors
* ``photo.photoionization_damped`` the same with radiatively damped poles
* ``outer.sweep_propagated``      Omega with the R-matrix propagated beyond
                                   r = a through long-range multipole coupling
* ``outer.gailitis``              coupled asymptotic solutions beyond the
                                   propagation radius (the multipole tail)
* ``resonance.measure_resonance`` position and width of a resonance from the
                                   slope of the eigenphase sum
* ``inner.inner_region``          poles and surface amplitudes from the full
                                   eigen-solve of a model inner-region
                                   Hamiltonian

It shares no code with the HIP path (``paper_1403_5524_amd``) and imports
nothing from it; both sides receive the same seeded arrays from
``paper_1403_5524_amd.workloads``, which holds no arithmetic of the method.
"""
from .coulomb import (coulomb_fg, open_channel_functions,
                      closed_channel_logderiv)
from .rmatrix import (r_matrix, channel_data, k_matrix, k_matrix_elimination,
                      k_matrix_lambda, t_matrix, s_matrix, eigenphases, collision_strengths,
                      omega_pair_index, sweep)
from .postproc import (gaussian_convolve, effective_collision_strengths,
                       trapezoid_weights, group_collision_strengths)
from .photo import (dipole_pole_sum, matching_solution, dipole_strength,
                    photoionization, photoionization_damped, SIGMA_CONST)
from . import outer
from . import inner
from . import resonance

__all__ = [
    "coulomb_fg", "open_channel_functions", "closed_channel_logderiv",
    "r_matrix", "channel_data", "k_matrix", "k_matrix_elimination",
    "k_matrix_lambda",
    "t_matrix", "s_matrix", "eigenphases", "collision_strengths",
    "omega_pair_index", "sweep",
    "gaussian_convolve", "effective_collision_strengths", "trapezoid_weights",
    "group_collision_strengths",
    "dipole_pole_sum", "matching_solution", "dipole_strength",
    "photoionization", "photoionization_damped", "SIGMA_CONST", "outer",
    "inner", "resonance",
]
