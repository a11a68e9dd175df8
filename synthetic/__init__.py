"""Seeded synthetic inputs for the ladder: counter-based random draws only.

This package holds no arithmetic of the ladder itself.  It draws the raw random
quantities of the input recipe (Cholesky-vector entries, orbital energies, the
multiplier noise) from a counter-based generator, so that any single element can
be regenerated from (seed, stream, index) alone.  The amplitudes built from these
draws are formed by each side on its own (the CPU oracle, or the HIP library).
"""
from .generate import *  # noqa: F401,F403
