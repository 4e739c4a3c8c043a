"""Chebyshev expansion of sparse matrix functions on AMD Instinct MI355X.

The method is that of "Efficient computation of sparse matrix functions for
large scale electronic structure calculations: The CheSS library": density
kernels by Fermi-operator expansion, matrix powers S^a and eigenvalues in an
interval, all from the truncated Chebyshev recursion on a fixed block sparsity
pattern.  The computation lives in libchess.so (hand-written HIP kernels for
gfx950 plus the host pipeline); this package is its Python binding.
"""
from .api import (BlockPattern, ChessError, Context, chess_chebyshev, chess_degree, chess_eigs_in_interval,
                  chess_features, chess_fermi_operator, chess_fermi_operator_batched,
                  chess_masked_product, chess_matrix_power,
                  chess_mlp_adam, chess_mlp_forward, chess_mlp_grad, chess_mlp_grad_noalloc,
                  chess_model_load,
                  chess_model_save, chess_bcsr_to_ssf, chess_ssf_to_bcsr, default_opts)
from .build import build_library, library_path

__all__ = ["BlockPattern", "ChessError", "Context", "chess_chebyshev", "chess_degree", "chess_eigs_in_interval",
           "chess_features", "chess_fermi_operator", "chess_fermi_operator_batched",
           "chess_masked_product", "chess_matrix_power",
           "chess_mlp_adam", "chess_mlp_forward", "chess_mlp_grad", "chess_mlp_grad_noalloc",
           "chess_model_load",
           "chess_model_save", "chess_bcsr_to_ssf", "chess_ssf_to_bcsr", "default_opts",
           "build_library", "library_path"]
