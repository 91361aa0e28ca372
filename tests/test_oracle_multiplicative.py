"""Pins of the oracle's multiplicative Schwarz sweep and its block colouring
(Section 3.2, the multiplicative formula after the additive one).

* one-unknown blocks in index order are forward Gauss-Seidel: B = (D+L)^{-1},
  checked against scipy's sparse triangular solve, and B^T against the
  transposed triangular solve;
* two disjoint blocks covering everything are block Gauss-Seidel: B is the
  inverse of the block lower triangle (numpy dense solve);
* one block over everything is the exact inverse;
* overlapping blocks: I - B A equals the textbook product of the block
  projections prod_j (I - E_j inv(A_j) R_j A), built with numpy.linalg.inv,
  and apply_transpose is B^T;
* unknowns in no block follow as one-unknown blocks in index order;
* the colouring: blocks of a colour are disjoint and uncoupled (brute force
  over the pattern), the colours are first-fit, a chain colours 0,1,0,1,...,
  reordering blocks inside a colour leaves the sweep unchanged, and the
  coupling pattern drops rounding-level entries but keeps real ones;
* the transposed V-cycle with the multiplicative smoother is the exact
  transpose of the V-cycle (y^T (M x) = (M^T y)^T x on random vectors).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.krylov import fgmres
from oracle.multigrid import Hierarchy
from oracle.schwarz import (MultiplicativeSchwarz, block_colouring, build_blocks,
                            colour_major, coupling_pattern)
from paper_1909_13201_amd import inputs


def random_matrix(N, seed, density=0.15):
    """Non-symmetric sparse matrix with a dominant diagonal."""
    rng = np.random.default_rng(seed)
    R = sp.random(N, N, density=density, random_state=rng, data_rvs=rng.standard_normal)
    return (R + sp.diags(4.0 + rng.random(N))).tocsr()


def dense_of(apply, N):
    return np.column_stack([apply(e) for e in np.eye(N)])


def test_singletons_are_gauss_seidel():
    N = 30
    A = random_matrix(N, 1)
    S = MultiplicativeSchwarz(A, [np.array([i]) for i in range(N)])
    r = np.random.default_rng(2).standard_normal(N)
    gs = spla.spsolve_triangular(sp.tril(A).tocsr(), r, lower=True)
    np.testing.assert_allclose(S.apply(r), gs, rtol=1e-12, atol=1e-14)
    gst = spla.spsolve_triangular(sp.tril(A).T.tocsr(), r, lower=False)
    np.testing.assert_allclose(S.apply_transpose(r), gst, rtol=1e-12, atol=1e-14)


def test_unknowns_outside_blocks_are_singletons_last():
    N = 24
    A = random_matrix(N, 3)
    blocks = [np.arange(0, 8), np.arange(6, 15)]
    S = MultiplicativeSchwarz(A, blocks)
    T = MultiplicativeSchwarz(A, blocks + [np.array([i]) for i in range(15, N)])
    r = np.random.default_rng(4).standard_normal(N)
    np.testing.assert_allclose(S.apply(r), T.apply(r), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(S.apply_transpose(r), T.apply_transpose(r), rtol=1e-13,
                               atol=1e-15)


def test_two_blocks_are_block_gauss_seidel():
    N, k = 26, 11
    A = random_matrix(N, 5).toarray()
    S = MultiplicativeSchwarz(sp.csr_matrix(A), [np.arange(k), np.arange(k, N)])
    Lb = A.copy()
    Lb[:k, k:] = 0.0
    r = np.random.default_rng(6).standard_normal(N)
    np.testing.assert_allclose(S.apply(r), np.linalg.solve(Lb, r), rtol=1e-12)


def test_one_block_is_exact():
    N = 20
    A = random_matrix(N, 7)
    S = MultiplicativeSchwarz(A, [np.arange(N)])
    r = np.random.default_rng(8).standard_normal(N)
    np.testing.assert_allclose(A @ S.apply(r), r, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(A.T @ S.apply_transpose(r), r, rtol=1e-12, atol=1e-12)


def test_overlapping_product_form_and_transpose():
    N = 28
    A = random_matrix(N, 9)
    Ad = A.toarray()
    blocks = [np.arange(0, 10), np.array([3, 8, 9, 10, 11, 12, 20]), np.arange(12, 22),
              np.array([1, 21, 22, 23, 24, 25])]
    S = MultiplicativeSchwarz(A, blocks)
    covered = np.zeros(N, bool)
    for I in blocks:
        covered[I] = True
    order = list(blocks) + [np.array([i]) for i in np.where(~covered)[0]]
    E = np.eye(N)
    for I in order:
        Rj = np.eye(N)[I]
        E = (np.eye(N) - Rj.T @ np.linalg.inv(Ad[np.ix_(I, I)]) @ Rj @ Ad) @ E
    B = dense_of(S.apply, N)
    np.testing.assert_allclose(B @ Ad, np.eye(N) - E, atol=1e-12)
    np.testing.assert_allclose(dense_of(S.apply_transpose, N), B.T, atol=1e-12)


def test_chain_colours_alternate():
    N = 20
    A = sp.diags([np.ones(N - 1), 2 * np.ones(N), np.ones(N - 1)], [-1, 0, 1]).tocsr()
    blocks = [np.arange(4 * j, 4 * j + 4) for j in range(5)]
    assert block_colouring(A, blocks).tolist() == [0, 1, 0, 1, 0]
    # a gap of one unknown between blocks leaves them uncoupled: one colour
    blocks = [np.arange(5 * j, 5 * j + 4) for j in range(4)]
    assert block_colouring(A, blocks).tolist() == [0, 0, 0, 0]
    # a one-way coupling is enough for a conflict
    B = sp.lil_matrix((8, 8))
    B.setdiag(1.0)
    B[0, 7] = 1.0
    assert block_colouring(B.tocsr(), [np.arange(0, 4), np.arange(4, 8)]).tolist() == [0, 1]


def test_coupling_pattern_threshold():
    P = sp.csr_matrix(np.array([[1.0, 1e-17, 1e-9], [0.0, 2.0, 0.0], [3e-16, 0.0, 5.0]]))
    Q = sp.csr_matrix(np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0]]))
    pat = coupling_pattern([P, Q]).toarray()
    assert pat.tolist() == [[1, 0, 1], [0, 1, 0], [1, 0, 1]]


@pytest.fixture(scope="module")
def c2small():
    cfg = inputs.with_levels(inputs.config("c2"), 3)
    return cfg, Hierarchy(cfg, inputs.advecting_field(cfg), build_smoothers=False)


def test_colouring_valid_and_first_fit(c2small):
    cfg, H = c2small
    for l in range(1, H.L):
        pat = H.coupling_pattern(l)
        blocks, _ = build_blocks(H.levels[l], cfg["core"], cfg["halo"])
        col = block_colouring(pat, blocks)
        sym = (pat + pat.T).tocsr()
        reach = []
        for I in blocks:
            touched = set(I.tolist())
            for a in I:
                touched.update(sym.indices[sym.indptr[a]:sym.indptr[a + 1]].tolist())
            reach.append(touched)
        nb = len(blocks)
        for j in range(nb):
            seen = set()
            for k in range(nb):
                if k == j:
                    continue
                clash = bool(reach[j].intersection(blocks[k].tolist()))
                if clash and k < j:
                    seen.add(int(col[k]))
                if col[k] == col[j]:
                    assert not clash, (l, j, k)
            # first fit: every smaller colour is taken by an earlier neighbour
            assert set(range(col[j])) <= seen, (l, j)
        assert col.max() + 1 <= 8


def test_order_inside_a_colour_does_not_matter(c2small):
    cfg, H = c2small
    l = H.L - 1
    blocks, _ = build_blocks(H.levels[l], cfg["core"], cfg["halo"])
    blocks, colours = colour_major(blocks, block_colouring(H.coupling_pattern(l), blocks))
    colours = np.array(colours)
    rng = np.random.default_rng(11)
    perm = np.concatenate([rng.permutation(np.where(colours == c)[0])
                           for c in range(colours.max() + 1)])
    S1 = MultiplicativeSchwarz(H.A[l], blocks)
    S2 = MultiplicativeSchwarz(H.A[l], [blocks[j] for j in perm])
    r = rng.standard_normal(H.A[l].shape[0])
    a, b = S1.apply(r), S2.apply(r)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))
    a, b = S1.apply_transpose(r), S2.apply_transpose(r)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_multiplicative_vcycle_transpose_and_convergence():
    cfg = dict(inputs.config("c1"), schwarz="multiplicative")
    H = Hierarchy(cfg)
    rng = np.random.default_rng(12)
    N = H.A[-1].shape[0]
    X, Y = rng.standard_normal((N, 4)), rng.standard_normal((N, 4))
    MX = np.column_stack([H.vcycle(x) for x in X.T])
    MtY = np.column_stack([H.vcycle(y, transpose=True) for y in Y.T])
    lhs, rhs = Y.T @ MX, MtY.T @ X
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-12 * np.abs(lhs).max())
    b = H.rhs(inputs.body_force(cfg))
    x, info = fgmres(lambda v: H.A[-1] @ v, H.vcycle, b, rtol=1e-10)
    assert info["converged"]
    Ha = Hierarchy(inputs.config("c1"))
    _, info_a = fgmres(lambda v: Ha.A[-1] @ v, Ha.vcycle, b, rtol=1e-10)
    assert info["iters"] < info_a["iters"]
