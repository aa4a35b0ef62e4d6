"""FP64 CPU oracle for the DG-CheFSI hot path.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path (the HIP
library and its Python binding) never does, and shares no code with it.

Everything here is float64 NumPy, written from the paper:
  * Algorithm 1 (the CheFSI cycle): bounds, Chebyshev filter, Cholesky-QR,
    Rayleigh-Ritz, subspace rotation;
  * eqs. matvec_1-matvec_3 (block-sparse H^DG times a block of vectors);
  * Sec. II B 2 (Cholesky factorisation instead of QR/DGKS for the
    orthonormalisation).
After the cycle: Fermi-Dirac occupations and the diagonal density-matrix
blocks (eq. densitymatrix, :mod:`oracle.density`), and the re-alignment of
the coefficients to a new ALB basis (eqs. basis_rotation_1-3,
:mod:`oracle.realign`).
The adjoint (reverse-mode gradient) of one filter + Cholesky-QR +
Rayleigh-Ritz pass is not in the paper; it follows the textbook reverse-mode
rules stated in :mod:`oracle.adjoint`.

Two operator modes: dense (H assembled as an N x N array; the parity
authority) and block-sparse (stored blocks applied element by element,
eq. matvec_3; used where the dense matrix does not fit and for the CPU
baseline timing).  The block-sparse mode is checked against the dense mode
in the test suite.
"""
from .core import (  # noqa: F401
    slot_neighbour, assemble_dense, DenseOperator, BlockOperator,
    chebyshev_coefficients, chebyshev_filter, lanczos, lanczos_upper_bound,
    bounds_cold, bounds_warm, cholesky_upper, solve_right_upper, cholesky_qr,
    rayleigh_ritz, sign_normalize, sweep, chebyshev_T, cholqr_condition_bound,
    auto_passes,
)
from .jacobi import jacobi_eigh  # noqa: F401
from .adjoint import (  # noqa: F401
    filter_backward, cholesky_qr_backward, rayleigh_ritz_backward,
    loss_forward, loss_backward, restrict_to_pattern,
)
from .density import (  # noqa: F401
    fermi_dirac, fermi_level, occupations, density_diag_blocks, density_dense, pack_blocks,
)
from .realign import (  # noqa: F401
    overlap_blocks, realign, realign_dense, assemble_samples, element_samples,
)
