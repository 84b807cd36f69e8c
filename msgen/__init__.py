"""Seeded synthetic inputs for the plane-wave multiple-scattering transport path.

This package builds the *inputs* of the method only: the transverse cell, the
plane-wave basis (which reciprocal vectors are kept), the difference-vector
index map, the slice potentials' Fourier coefficients of a set of Gaussian
wells, slice thicknesses and the (E, k_par) grids.  It holds none of the
method's arithmetic (no Hamiltonians, eigenproblems, scattering matrices or
transmissions); both the CPU oracle and the HIP library consume what it
produces.

Units: Rydberg atomic units with the kinetic operator written as -nabla^2
(hbar^2/2m = 1), energies in Ry, lengths in bohr.
"""
from .lattice import Cell, plane_wave_basis, difference_set
from .potential import Wells, slice_edges, vq_gaussian_wells
from .configs import (Junction, junction_inputs, config1, config2, config3,
                      config3_electrode,
                      config4_instances, config5, CONFIGS)

__all__ = [
    "Cell", "plane_wave_basis", "difference_set", "Wells", "slice_edges",
    "vq_gaussian_wells", "Junction", "junction_inputs", "config1", "config2",
    "config3", "config3_electrode", "config4_instances", "config5", "CONFIGS",
]
