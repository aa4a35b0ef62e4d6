"""Seeded synthetic inputs for DG-CheFSI workloads.

This module only *draws* inputs: periodic element grids, per-element ALB
counts J_K, the stored nonzero blocks H_{K;K'} of a symmetric block-sparse
DG-shaped Hamiltonian, start blocks X and Lanczos start vectors.  It holds
none of the method's arithmetic (no filter, no orthonormalisation, no
Rayleigh-Ritz); both the CPU oracle and the GPU library consume what it makes.

Problem shape (Sec. II A of the paper, eqs. for the block structure of H^DG):
  * the domain is a periodic nx x ny x nz grid of elements, element id
    K = ix + nx*(iy + ny*iz);
  * element K carries J_K basis functions, its rows of any multivector are
    contiguous (element-major row order), N = sum_K J_K;
  * H_{K;K'} (J_K x J_K') is nonzero only for face neighbours K' of K.

Stored-block convention ("slot" order): every element stores one block per
stencil direction, in the order self, -x, +x, -y, +y, -z, +z (7-point
stencil) or self, -x, +x, -y, +y (5-point, in-plane sheets).  A periodic
dimension of length 2 reaches the same neighbour through two slots and a
length-1 dimension reaches the element itself; such blocks *add* when the
dense matrix is formed.  Element K owns its +x/+y/+z faces: the +d block is
drawn as G and the -d block of the neighbour is G^T, which makes the dense
matrix exactly (bitwise) symmetric, except that a length-1 dimension adds
three terms onto a diagonal block and is symmetric to rounding.

Value distributions: diagonal blocks Q diag(lambda) Q^T with lambda ~ U[lo, hi]
and Q Haar-random (QR of a Gaussian matrix with the signs of diag(R) folded
in, Mezzadri 2007), symmetrised; off-diagonal blocks i.i.d. N(0, sigma^2).

Packed ("block-list") layout handed to the library: for K = 0..M-1, for each
slot s, the J_K x J_{K'_s} block in row-major order, back to back, float64.

ALB samples for the basis re-alignment (Sec. II B 3): element K's J_K ALBs
sampled on its own n_r grid points, V_K (n_r x J_K) with orthonormal columns
(the DG basis is orthonormal), drawn as the first J_K columns of a Haar
orthogonal n_r x n_r matrix; the next SCF step's basis is the orthonormalised
V_K + delta G_K (G_K Gaussian), a nearby basis with a different span.  Stored
element-major, each element as V_K^T (J_K rows of n_r samples), row-major.

Random streams: numpy SeedSequence(base_seed, spawn_key=(purpose, K)), so any
element's data can be regenerated on its own.  Purposes: 0 eigenvalues,
1 Haar Q, 2 off-diagonal blocks, 3 start block X, 4 Lanczos start vector,
5 mixed J_K draw, 6 finite-difference entry choice, 7 ALB samples,
8 ALB change between SCF steps, 9 dense orthonormal block.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 1606

# slot order: self, -x, +x, -y, +y, -z, +z
SLOT_DIRS = ((0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))

(PURPOSE_EIG, PURPOSE_HAAR, PURPOSE_OFFDIAG, PURPOSE_X0, PURPOSE_LANCZOS, PURPOSE_JDRAW, PURPOSE_FD,
 PURPOSE_ALB, PURPOSE_ALB_STEP, PURPOSE_ORTH) = range(10)

# Boltzmann constant in Hartree per kelvin (CODATA 2018) and the electronic
# temperature of the paper's runs (Sec. III: 300 K Fermi-Dirac smearing).
BOLTZMANN_HA_PER_K = 3.1668115634556e-6
KT_300K = 300.0 * BOLTZMANN_HA_PER_K
# Grid points per element for the ALB samples (an 8 x 8 x 8 element grid).
NR_PER_ELEMENT = 512


def rng_for(purpose: int, key: int = 0, base_seed: int = BASE_SEED) -> np.random.Generator:
    ss = np.random.SeedSequence(base_seed, spawn_key=(int(purpose), int(key)))
    return np.random.Generator(np.random.PCG64(ss))


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload shape (grid, stencil, ALB counts, states, degree)."""
    name: str
    grid: Tuple[int, int, int]
    stencil: int
    nb: Optional[int]                 # uniform ALBs per element, or None for a mixed draw
    nb_choices: Optional[Tuple[int, ...]] = None
    ns: int = 48
    m: int = 10
    sweeps: int = 1
    lanczos_steps: int = 20
    lam_lo: float = -0.5
    lam_hi: float = 4.0
    sigma_off: float = 0.05

    @property
    def M(self) -> int:
        return self.grid[0] * self.grid[1] * self.grid[2]


# The five workload shapes of the build (tiny, differentiation, bulk 3D,
# bulk 3D mixed precision, 2D sheet with uneven ALB counts).
TINY = Workload("tiny_2x2x2_nb32", (2, 2, 2), 7, 32, ns=48, m=10, sweeps=5)
DIFF = Workload("diff_6x6x6_nb48", (6, 6, 6), 7, 48, ns=512, m=12, sweeps=1)
BULK = Workload("bulk_12x12x12_nb64", (12, 12, 12), 7, 64, ns=4096, m=16, sweeps=4)
SHEET = Workload("sheet_48x40x1_nb64-128", (48, 40, 1), 5, None,
                 nb_choices=tuple(range(64, 129, 8)), ns=8192, m=20, sweeps=4)
WORKLOADS = {w.name: w for w in (TINY, DIFF, BULK, SHEET)}


def element_id(ix: int, iy: int, iz: int, grid: Sequence[int]) -> int:
    nx, ny, nz = grid
    return (ix % nx) + nx * ((iy % ny) + ny * (iz % nz))


def element_coords(K: int, grid: Sequence[int]) -> Tuple[int, int, int]:
    nx, ny, _ = grid
    return K % nx, (K // nx) % ny, K // (nx * ny)


def slot_neighbour(K: int, s: int, grid: Sequence[int]) -> int:
    ix, iy, iz = element_coords(K, grid)
    dx, dy, dz = SLOT_DIRS[s]
    return element_id(ix + dx, iy + dy, iz + dz, grid)


def draw_alb_counts(w: Workload, base_seed: int = BASE_SEED) -> np.ndarray:
    if w.nb is not None:
        return np.full(w.M, w.nb, dtype=np.int32)
    choices = np.asarray(w.nb_choices, dtype=np.int32)
    g = rng_for(PURPOSE_JDRAW, 0, base_seed)
    return choices[g.integers(0, len(choices), size=w.M)].astype(np.int32)


def haar_orthogonal(n: int, g: np.random.Generator) -> np.ndarray:
    z = g.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    return q * np.sign(np.diag(r))[None, :]


@dataclasses.dataclass
class BlockProblem:
    """Stored blocks of a block-sparse H plus its shape data."""
    grid: Tuple[int, int, int]
    stencil: int
    J: np.ndarray                     # int32 [M]
    blocks: List[List[np.ndarray]]    # blocks[K][s], J_K x J_{K'_s}, float64
    eigs: Optional[List[np.ndarray]] = None   # drawn diagonal-block spectra (if any)

    @property
    def M(self) -> int:
        return len(self.J)

    @property
    def N(self) -> int:
        return int(np.sum(self.J, dtype=np.int64))

    def row_offsets(self) -> np.ndarray:
        off = np.zeros(self.M + 1, dtype=np.int64)
        np.cumsum(self.J, out=off[1:])
        return off

    def packed(self, dtype=np.float64) -> np.ndarray:
        """Block-list layout: element-major, slot-minor, each block row-major."""
        parts = [b.ravel() for row in self.blocks for b in row]
        return np.concatenate(parts).astype(dtype, copy=False)

    def packed_size(self) -> int:
        return sum(b.size for row in self.blocks for b in row)

    @staticmethod
    def from_packed(grid, stencil, J, flat: np.ndarray) -> "BlockProblem":
        J = np.asarray(J, dtype=np.int32)
        M = len(J)
        blocks, pos = [], 0
        for K in range(M):
            row = []
            for s in range(stencil):
                Kp = slot_neighbour(K, s, grid)
                n = int(J[K]) * int(J[Kp])
                row.append(np.asarray(flat[pos:pos + n], dtype=np.float64).reshape(int(J[K]), int(J[Kp])))
                pos += n
            blocks.append(row)
        return BlockProblem(tuple(grid), stencil, J, blocks)


def make_blocks(grid: Sequence[int], stencil: int, J: np.ndarray, *,
                lam_lo: float = -0.5, lam_hi: float = 4.0, sigma_off: float = 0.05,
                diag_kind: str = "haar", base_seed: int = BASE_SEED) -> BlockProblem:
    """Draw the stored blocks.

    diag_kind: "haar"   -> Q diag(lambda) Q^T, lambda ~ U[lam_lo, lam_hi]
               "diag"   -> diag(lambda) (no rotation)
    sigma_off = 0 gives a decoupled (block-diagonal) H.
    """
    grid = tuple(int(v) for v in grid)
    assert stencil in (5, 7)
    J = np.asarray(J, dtype=np.int32)
    M = grid[0] * grid[1] * grid[2]
    assert len(J) == M
    blocks: List[List[Optional[np.ndarray]]] = [[None] * stencil for _ in range(M)]
    eigs = []
    for K in range(M):
        n = int(J[K])
        lam = rng_for(PURPOSE_EIG, K, base_seed).uniform(lam_lo, lam_hi, size=n)
        eigs.append(lam)
        if diag_kind == "haar":
            Q = haar_orthogonal(n, rng_for(PURPOSE_HAAR, K, base_seed))
            B = (Q * lam[None, :]) @ Q.T
            B = 0.5 * (B + B.T)
        elif diag_kind == "diag":
            B = np.diag(lam)
        else:
            raise ValueError(diag_kind)
        blocks[K][0] = B
    # owned faces: +x (slot 2), +y (slot 4), +z (slot 6); the neighbour's
    # opposite slot gets the transpose.
    owned = (2, 4, 6) if stencil == 7 else (2, 4)
    for K in range(M):
        g = rng_for(PURPOSE_OFFDIAG, K, base_seed)
        for s in owned:
            Kp = slot_neighbour(K, s, grid)
            G = g.normal(0.0, 1.0, size=(int(J[K]), int(J[Kp]))) * sigma_off
            blocks[K][s] = G
            blocks[Kp][s - 1] = G.T.copy()
    return BlockProblem(grid, stencil, J, blocks, eigs)


def make_scalar_lattice(grid: Sequence[int], stencil: int, nb: int, d: float, t: float) -> BlockProblem:
    """Diagonal blocks d*I and every stored off-diagonal block t*I."""
    grid = tuple(int(v) for v in grid)
    M = grid[0] * grid[1] * grid[2]
    J = np.full(M, nb, dtype=np.int32)
    blocks = [[(d if s == 0 else t) * np.eye(nb) for s in range(stencil)] for _ in range(M)]
    return BlockProblem(grid, stencil, J, blocks)


def make_problem(w: Workload, base_seed: int = BASE_SEED, **kw) -> BlockProblem:
    J = draw_alb_counts(w, base_seed)
    return make_blocks(w.grid, w.stencil, J, lam_lo=w.lam_lo, lam_hi=w.lam_hi,
                       sigma_off=w.sigma_off, base_seed=base_seed, **kw)


def make_start_block(J: np.ndarray, ns: int, base_seed: int = BASE_SEED, dtype=np.float64,
                     threads: int = 0) -> np.ndarray:
    """X0 ~ N(0,1), N x ns, drawn element by element (rows of element K).

    Each element has its own stream, so drawing them on several threads gives
    the same array."""
    import concurrent.futures as cf
    import os
    J = np.asarray(J)
    N = int(np.sum(J, dtype=np.int64))
    X = np.empty((N, ns), dtype=dtype)
    off = np.zeros(len(J) + 1, dtype=np.int64)
    off[1:] = np.cumsum(J)

    def fill(K):
        g = rng_for(PURPOSE_X0, K, base_seed)
        if dtype == np.float64:
            g.standard_normal((int(J[K]), ns), out=X[off[K]:off[K + 1]])
        else:
            X[off[K]:off[K + 1]] = g.standard_normal((int(J[K]), ns))

    nthr = threads or min(16, os.cpu_count() or 1)
    if nthr <= 1 or N * ns < (1 << 22):
        for K in range(len(J)):
            fill(K)
    else:
        with cf.ThreadPoolExecutor(nthr) as ex:
            list(ex.map(fill, range(len(J))))
    return X


def make_lanczos_start(N: int, base_seed: int = BASE_SEED) -> np.ndarray:
    return rng_for(PURPOSE_LANCZOS, 0, base_seed).standard_normal(N)


def make_orthonormal_block(N: int, ns: int, base_seed: int = BASE_SEED, threads: int = 0) -> np.ndarray:
    """A dense N x ns block with orthonormal columns, cheap to draw at any size:
    ns distinct columns of the orthonormal DCT-II basis of length N (random
    frequencies k_j), with the rows permuted and their signs flipped at random,
        Y[i, j] = d_i c_{k_j} cos(pi (2 p_i + 1) k_j / (2N)),
    c_0 = sqrt(1/N), c_k = sqrt(2/N) otherwise, p a random permutation and d
    random signs.  The argument (2p+1)k is reduced modulo 4N in integers
    before the cosine, so every entry is accurate to rounding.  Rows are drawn
    in blocks on several threads; the result does not depend on the count."""
    import concurrent.futures as cf
    import os
    if not (1 <= ns <= N):
        raise ValueError("need 1 <= ns <= N")
    g = rng_for(PURPOSE_ORTH, 0, base_seed)
    k = np.sort(g.choice(N, size=ns, replace=False)).astype(np.int64)
    perm = g.permutation(N).astype(np.int64)
    sign = np.where(g.integers(0, 2, size=N) == 1, 1.0, -1.0)
    scale = np.where(k == 0, np.sqrt(1.0 / N), np.sqrt(2.0 / N))
    Y = np.empty((N, ns), dtype=np.float64)
    step = 2048

    def fill(r0):
        r1 = min(N, r0 + step)
        m = ((2 * perm[r0:r1, None] + 1) * k[None, :]) % (4 * N)
        Y[r0:r1] = np.cos((np.pi / (2 * N)) * m) * scale[None, :] * sign[r0:r1, None]

    nthr = threads or min(16, os.cpu_count() or 1)
    starts = range(0, N, step)
    if nthr <= 1:
        for r0 in starts:
            fill(r0)
    else:
        with cf.ThreadPoolExecutor(nthr) as ex:
            list(ex.map(fill, starts))
    return Y


def fd_entries(P: BlockProblem, count: int, base_seed: int = BASE_SEED):
    """Random (K, s, i, j) positions of stored blocks for finite-difference checks."""
    g = rng_for(PURPOSE_FD, 0, base_seed)
    out = []
    for _ in range(count):
        K = int(g.integers(0, P.M))
        s = int(g.integers(0, P.stencil))
        b = P.blocks[K][s]
        out.append((K, s, int(g.integers(0, b.shape[0])), int(g.integers(0, b.shape[1]))))
    return out


def occupied_count(ns: int) -> float:
    """Occupied orbital pairs N_e / 2 for an ns-state block: the lowest 3/4
    of the states (the part a few cycles converge), the rest the buffer of
    partially occupied and empty states."""
    return 0.75 * ns


def _orthonormal_columns(A: np.ndarray) -> np.ndarray:
    q, r = np.linalg.qr(A)
    return q * np.sign(np.diag(r))[None, :]


def make_alb_samples(J: np.ndarray, nr: int = NR_PER_ELEMENT, base_seed: int = BASE_SEED) -> np.ndarray:
    """Packed V_K^T for every element (element-major, J_K x n_r each): the
    first J_K columns of a Haar n_r x n_r orthogonal matrix."""
    J = np.asarray(J)
    if nr < int(J.max()):
        raise ValueError("n_r must be at least the largest ALB count")
    parts = []
    for K in range(len(J)):
        g = rng_for(PURPOSE_ALB, K, base_seed)
        V = _orthonormal_columns(g.standard_normal((nr, int(J[K]))))
        parts.append(V.T.ravel())
    return np.concatenate(parts)


def make_next_alb_samples(J: np.ndarray, V_packed: np.ndarray, nr: int = NR_PER_ELEMENT,
                          delta: float = 0.05, base_seed: int = BASE_SEED) -> np.ndarray:
    """The next SCF step's samples: orthonormalised V_K + delta G_K per
    element, G_K ~ N(0, 1) (signs fixed so that the new basis stays close to
    the old one)."""
    J = np.asarray(J)
    off = np.zeros(len(J) + 1, dtype=np.int64)
    off[1:] = np.cumsum(J)
    parts = []
    for K in range(len(J)):
        V = np.asarray(V_packed[nr * off[K]:nr * off[K + 1]]).reshape(int(J[K]), nr).T
        g = rng_for(PURPOSE_ALB_STEP, K, base_seed)
        Vn = _orthonormal_columns(V + delta * g.standard_normal(V.shape))
        parts.append(Vn.T.ravel())
    return np.concatenate(parts)
