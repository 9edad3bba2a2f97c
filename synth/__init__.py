"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package describes *inputs* only: lattice geometries as bond lists, pulse
parameter sets, workload presets and seeded random vectors.  It contains none
of the method's arithmetic (no Hamiltonian, no basis, no pulse evaluation, no
time stepping), so the CPU oracle and the HIP path can both draw from it
without sharing any computation.
"""
from .lattices import Lattice, ring, chain, cluster_2d, two_site, ring_nnn, random_graph
from .workloads import (PulseParams, Workload, workloads, random_state, draw_amplitudes, controller_draws,
                        controller_groups)

__all__ = [
    "Lattice", "ring", "chain", "cluster_2d", "two_site", "ring_nnn", "random_graph",
    "PulseParams", "Workload", "workloads", "random_state", "draw_amplitudes", "controller_draws",
    "controller_groups",
]
