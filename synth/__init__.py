"""Seeded synthetic inputs: counter-based RNG, parameter grids, flip-angle
trains, Bloch/EPG fingerprint simulation, phantoms, sampling patterns and
simulated k-space.  Shared by the tests, the oracle and the benchmark; it
holds none of the reconstruction's arithmetic (no matched filter, no
projected gradient, no search)."""
from . import bloch, grids, rng, sequences, workloads  # noqa: F401
