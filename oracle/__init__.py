"""CPU FP64 oracle for the Bloch-CAP transmission path.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path (the HIP library and its Python
binding) never imports, calls or links anything here, and nothing here imports
the product path.  Inputs come from the seeded generators, which hold none of
the method's arithmetic.

Pins (tests/test_oracle_*.py) tie each function to the paper and to
mathematics independent of this code: FD weights exact on polynomials and the
textbook 4th-order values; the lateral Laplacian spectrum in closed form; the
free-electron separable identity against an independent 1D solve; the
open-channel count for long CAPs; Bloch-mode counting in a periodic chain;
supercell folding; T_LR = T_RL, T(k) = T(-k), T(k+G) = T(k), the CAP sum rule
and T >= 0; a one-point projector reducing to a local potential.  The eigen
route (oracle.eigen) is pinned by the LU route: with all eigenpairs both give
the same T; by the +-k relation of left and right eigenvectors; by Im(lam) <= 0
and by the complex-orthogonality of the eigenvectors where K is complex symmetric.
"""
from . import eigen
from .transport import (fd_second_derivative, fd_dispersion, hamiltonian_dense,
                        hamiltonian_sparse, bloch_projectors, system_matrix,
                        apply_system, transmission, green_columns, trace_forms,
                        residual_norms)

__all__ = ["fd_second_derivative", "fd_dispersion", "hamiltonian_dense",
           "hamiltonian_sparse", "bloch_projectors", "system_matrix", "apply_system",
           "transmission", "green_columns", "trace_forms", "residual_norms", "eigen"]
