"""MI355X (gfx950) DG-CheFSI: Chebyshev-filtered subspace iteration on a
block-sparse DG Hamiltonian, as a C-ABI HIP library with a thin Python binding.

The binding only marshals arguments: torch tensors provide device memory and
the current stream, every step of the method runs in libchefsi.so.  Importing
this package loads the library and fails loudly if it is missing.

    import paper_1606_03416_amd as chefsi
    plan = chefsi.Plan((12, 12, 12), 7, J)            # element grid, stencil, ALB counts
    Y = plan.filter(H, X, m, a, b, a0)                 # Algorithm 1 step 2
    U = chefsi.orthonormalize(Y, passes=2)             # step 3 (in place)
    Xn, ritz, resid, Q = plan.rayleigh_ritz(H, Y)      # steps 4-5
    plan.sweep(H, X, m, v0=v0, ritz=ritz, ...)         # steps 1-5
    f, mu = chefsi.occupations(ritz, n_occ, kT)        # Fermi-Dirac occupations
    P = plan.density_blocks(X, f)                      # diagonal density-matrix blocks
    plan.realign(X, V_new, V_old, nr)                  # coefficients onto a new ALB basis
    st = chefsi.SweepState(X, v0); chefsi.run_cycles(plan, H, st, 2, m)
    st.save("run.npz", plan)                           # resumable run (bit-identical)
"""
from ._binding import (  # noqa: F401
    ChefsiError, Plan, orthonormalize, orthonormalize_backward, occupations, library_path, lib, ChefsiLoss, ChebFilter,
    F64, F32, BF16, BF16X3, OP_BOUNDS, OP_FILTER, OP_ORTHONORMALIZE, OP_RAYLEIGH_RITZ, OP_SWEEP,
    OP_FILTER_BACKWARD, OP_LOSS_BACKWARD, OP_DENSITY, OP_LOSS, OP_RAYLEIGH_RITZ_BACKWARD, ERR_NOT_PD, ERR_ARG, ERR_WORKSPACE, ERR_EIG, ERR_HIP,
    ERR_NONFINITE, ERR_UNSUPPORTED,
)
from .state import SweepState, run_cycles  # noqa: F401,E402
