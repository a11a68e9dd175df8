"""MI355X-native particle-particle ladder of CD-CCSD (forward, energy, adjoint).

The compute path is libladder.so (hand-written HIP kernels for gfx950 behind a C
ABI, include/ladder.h).  This package is the thin ctypes binding: it checks
tensors, passes device pointers and the current HIP stream, and raises on error.
There is no CPU fallback: without the built library every call raises.
"""
from .ladder import (  # noqa: F401
    FP64, SPLIT_BF16, SPLIT_INT8, FLAG_GENERAL, FLAG_DENSE, DO_FORWARD, DO_ADJOINT, U_TABLE, U_APPENDIX, LadderError, Options,
    workspace_size, forward, adjoint, tau_gradient_workspace_size, tau_gradient, autotune, autotune_load,
    autotune_reset, w_intermediate, metric_contraction,
    back_transform_workspace_size, back_transform, excited_amplitudes, ov3_abci_workspace_size, ov3_abci,
    ov3_abic_workspace_size, ov3_abic, metric_contraction_pairs, mfma_probe, PROBE_BF16, PROBE_FP64, PROBE_INT8, mp2_amplitudes, amplitude_update, batched,
    batched_workspace_size, LadderEnergy, ladder_energy, library_path, exported_symbols, profile_start, profile_stop, gemm, gemm_workspace_size,
    forward_noalloc,
)
