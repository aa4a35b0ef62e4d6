"""Full-size Rayleigh-Ritz parity (Algorithm 1 steps 4-5) at the benchmark
sizes: bulk (N = 110,592, N_s = 4,096) and sheet (N = 184,584, N_s = 8,192).

The input is the same dense orthonormal block on both sides
(synth.make_orthonormal_block).  The expected values -- every Ritz value, every
residual norm and a sample of eigenvectors of the projected matrix -- were
written by tests/golden/make_rr_fullsize.py from the CPU oracle alone (H applied
block by block, LAPACK eigensolver).  The GPU runs chefsi_rayleigh_ritz in the
benchmark's launch configuration (own tridiagonal reduction of all N_s - 1
columns, rocSOLVER dstedc, own back-transformation)."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
WORKLOADS = {"bulk": synth.BULK, "sheet": synth.SHEET}


@pytest.mark.parametrize("name", ["bulk", "sheet"])
def test_rayleigh_ritz_full_spectrum_matches_oracle(lib, name):
    g = np.load(os.path.join(GOLDEN, f"rr_fullsize_{name}.npz"))
    theta_o, resid_o, q_idx, q_o = g["theta"], g["resid"], g["q_idx"], g["q_cols"]
    hh_fro = float(g["hh_fro"])
    w = WORKLOADS[name]
    P = synth.make_problem(w)
    assert theta_o.shape == (w.ns,)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    Yh = torch.from_numpy(synth.make_orthonormal_block(P.N, w.ns)).cuda()
    Hd = torch.from_numpy(P.packed()).cuda()
    Xn, ritz, resid, Q = plan.rayleigh_ritz(Hd, Yh, want_Q=True)
    torch.cuda.synchronize()
    th = ritz.cpu().numpy()
    s = float(np.max(np.abs(theta_o)))
    # every Ritz value (reading: relative to max(|theta|, s))
    e_theta = float(np.max(np.abs(th - theta_o) / np.maximum(np.abs(theta_o), s)))
    # every residual norm r_i = ||H x_i - theta_i x_i||
    e_resid = float(np.max(np.abs(resid.cpu().numpy() - resid_o)) / s)
    # sampled eigenvectors of Hhat (columns of Q; all sampled values are
    # isolated here, so each is compared as a vector: perturbation ~ eps ||Hhat|| / gap)
    Qh = Q.cpu().numpy()
    worst_q = 0.0
    for col, i in enumerate(q_idx):
        gap = min(abs(theta_o[i] - theta_o[i - 1]) if i > 0 else np.inf,
                  abs(theta_o[i + 1] - theta_o[i]) if i + 1 < w.ns else np.inf)
        tol = 1e-12 * hh_fro / gap + 1e-12
        err = float(np.linalg.norm(Qh[:, i] - q_o[:, col]))
        worst_q = max(worst_q, err / tol)
        assert err <= tol, (name, int(i), err, gap)
    # the rotated block stays orthonormal
    orth = float(torch.max(torch.abs(Xn.T @ Xn - torch.eye(w.ns, dtype=torch.float64, device="cuda"))).item())
    print(f"{name}: Ritz values {e_theta:.2e}, residuals {e_resid:.2e}, eigenvectors {worst_q:.2e} of tolerance, "
          f"max|X^T X - I| {orth:.2e}")
    assert e_theta <= 1e-10
    assert e_resid <= 1e-10
    assert orth <= 1e-12
