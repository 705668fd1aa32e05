"""Seeded synthetic inputs for the many-variable VMC hot path.

This package only *describes* workloads: lattices and bond lists, the index
maps that tie pair amplitudes f_ij, Gutzwiller g_i and Jastrow v_ij to
variational-parameter slots, the initial parameter vectors, and uniformly
drawn electron configurations.  It holds none of the method's arithmetic
(no Pfaffians, ratios, energies or derivatives), so both the CPU oracle and
the GPU library can consume it without sharing any computation.

Every generator takes an explicit seed; the same seed gives the same arrays
on every machine (numpy's PCG64 bit generator).
"""
from .lattice import Lattice, chain, square
from .instance import Instance, make_instance, n_params_of
from .configs import WORKLOADS, workload, random_configs

__all__ = [
    "Lattice", "chain", "square", "Instance", "make_instance", "n_params_of",
    "WORKLOADS", "workload", "random_configs",
]
