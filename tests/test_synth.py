"""Seeded input generator: exact symmetry, Haar orthogonality, reproducibility,
packed layout round trip, realised sizes of the workload shapes."""
import numpy as np

import oracle
import synth


def test_blocks_symmetric_and_reproducible():
    P = synth.make_problem(synth.TINY)
    Q = synth.make_problem(synth.TINY)
    assert all(np.array_equal(a, b) for ra, rb in zip(P.blocks, Q.blocks) for a, b in zip(ra, rb))
    for K in range(P.M):
        assert np.array_equal(P.blocks[K][0], P.blocks[K][0].T)
        for s in range(1, P.stencil):
            Kp = synth.slot_neighbour(K, s, P.grid)
            sm = s + 1 if s % 2 == 1 else s - 1
            assert np.array_equal(P.blocks[K][s], P.blocks[Kp][sm].T)
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    assert np.array_equal(H, H.T)


def test_haar_and_spectrum():
    g = synth.rng_for(synth.PURPOSE_HAAR, 7)
    Q = synth.haar_orthogonal(64, g)
    assert np.linalg.norm(Q.T @ Q - np.eye(64)) <= 1e-14 * 64
    P = synth.make_problem(synth.TINY)
    for K in range(P.M):
        w = np.linalg.eigvalsh(P.blocks[K][0])
        assert np.max(np.abs(w - np.sort(P.eigs[K]))) <= 1e-13
        assert P.eigs[K].min() >= -0.5 and P.eigs[K].max() <= 4.0


def test_packed_round_trip_and_sizes():
    J = np.array([8, 16, 24, 8, 16, 8], dtype=np.int32)
    P = synth.make_blocks((3, 2, 1), 5, J)
    flat = P.packed()
    assert flat.size == P.packed_size()
    R = synth.BlockProblem.from_packed(P.grid, P.stencil, P.J, flat)
    assert all(np.array_equal(a, b) for ra, rb in zip(P.blocks, R.blocks) for a, b in zip(ra, rb))
    # sheet workload: mixed ALB counts drawn from {64, 72, ..., 128}
    Js = synth.draw_alb_counts(synth.SHEET)
    assert Js.size == 48 * 40 and set(np.unique(Js)) <= set(range(64, 129, 8))
    assert 170_000 < int(Js.sum()) < 200_000
    assert synth.draw_alb_counts(synth.BULK).sum() == 110_592


def test_start_block_per_element_streams():
    J = np.array([4, 6, 5], dtype=np.int32)
    X = synth.make_start_block(J, 7)
    X2 = synth.make_start_block(J, 7)
    assert np.array_equal(X, X2) and X.shape == (15, 7)
    g = synth.rng_for(synth.PURPOSE_X0, 1)
    assert np.array_equal(X[4:10], g.standard_normal((6, 7)))
