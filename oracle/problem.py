"""Problem data for  min <C,X>  s.t.  A(X) = b,  X psd  (paper eq. prob:sdp).

The constraint map is kept in the form the paper's Section 3.3-3.4 describes:
each A_k is flattened into a row of the stacked matrix  Abf  (m x n^2), and only
the nonzero columns of  Abf  are kept.  A column is a position (a, b) of the
n x n matrix, so for X = U V^T the compressed vector  xbar  holds
xbar_p = U[a_p] . V[b_p]  and  A(U V^T) = Abf_compressed @ xbar.  The adjoint is
A*(y) = mat(Abf^T y), built as an n x n sparse matrix.

Test infrastructure only (see the package docstring).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class SDPProblem:
    n: int                    # matrix dimension
    m: int                    # number of constraints
    C: sp.csr_matrix          # objective matrix (symmetric, n x n)
    col_a: np.ndarray         # row position a_p of each nonzero column of Abf
    col_b: np.ndarray         # column position b_p of each nonzero column of Abf
    Abar: sp.csr_matrix       # m x ncols stacked constraint matrix (nonzero columns only)
    b: np.ndarray             # right-hand side, length m
    kind: str = "general"
    # Per-row rank of the factor (several blocks with their own ranks): row i of
    # R keeps columns < row_rank[i] and holds zeros in the others; None: every
    # row uses every column.
    row_rank: np.ndarray | None = None

    def rank_mask(self, r: int) -> np.ndarray | None:
        """n x r 0/1 mask of the free entries of an n x r factor (None: all free)."""
        if self.row_rank is None:
            return None
        return (np.arange(r)[None, :] < self.row_rank[:, None]).astype(np.float64)

    # ---- the linear map and its adjoint (Section 3.3, eq. At) ----
    def A_of(self, U: np.ndarray, V: np.ndarray | None = None) -> np.ndarray:
        """A(U V^T): compressed outer product over the nonzero columns, then Abf."""
        if V is None:
            V = U
        xbar = np.einsum("pc,pc->p", U[self.col_a], V[self.col_b])
        return self.Abar @ xbar

    def A_adj(self, y: np.ndarray) -> sp.csr_matrix:
        """A*(y) = sum_k y_k A_k = mat(Abf^T y) as an n x n sparse matrix."""
        vals = self.Abar.T @ y
        return sp.csr_matrix((vals, (self.col_a, self.col_b)), shape=(self.n, self.n))

    def objective(self, U: np.ndarray, V: np.ndarray | None = None) -> float:
        """<C, U V^T> = trace(C V U^T) = sum_i (C V)_i . U_i."""
        if V is None:
            V = U
        return float(np.sum((self.C @ V) * U))

    @property
    def c_l1(self) -> float:
        """||vec(C)||_1, the normaliser of the dual infeasibility err2."""
        return float(np.abs(self.C.data).sum())


def _stack_constraints(n, m, k_idx, a_idx, b_idx, vals):
    """Build the compressed Abf from triplets: A_k[a, b] = val."""
    key = a_idx.astype(np.int64) * n + b_idx.astype(np.int64)
    ukey, col = np.unique(key, return_inverse=True)
    Abar = sp.csr_matrix((vals, (k_idx, col)), shape=(m, ukey.size))
    Abar.sum_duplicates()
    return (ukey // n).astype(np.int64), (ukey % n).astype(np.int64), Abar


def laplacian(n: int, u: np.ndarray, v: np.ndarray, w: np.ndarray | None) -> sp.csr_matrix:
    """Weighted graph Laplacian as the paper's MaxCut section defines it:
    L_ij = -w_ij for each edge (both orientations), L_ii = sum_k w_ik."""
    if w is None:
        w = np.ones(len(u))
    w = np.asarray(w, dtype=np.float64)
    rows = np.concatenate([u, v])
    cols = np.concatenate([v, u])
    off = sp.csr_matrix((-np.concatenate([w, w]), (rows, cols)), shape=(n, n))
    deg = np.zeros(n)
    np.add.at(deg, u, w)
    np.add.at(deg, v, w)
    return (off + sp.diags(deg)).tocsr()


def maxcut_problem(n: int, u, v, w=None) -> SDPProblem:
    """MaxCut SDP in minimisation form: max <L/4, X> = -min <-L/4, X>, X_ii = 1."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    C = (-0.25 * laplacian(n, u, v, w)).tocsr()
    C.sum_duplicates()
    k = np.arange(n)
    col_a, col_b, Abar = _stack_constraints(n, n, k, k, k, np.ones(n))
    return SDPProblem(n=n, m=n, C=C, col_a=col_a, col_b=col_b, Abar=Abar,
                      b=np.ones(n), kind="maxcut")


def completion_problem(n1: int, n2: int, i, j, Mij) -> SDPProblem:
    """Nuclear-norm matrix completion as an SDP (paper, matrix completion section).

    X = [[W1, M], [M^T, W2]] of order n1 + n2, objective <I, X>, and for each
    observed entry k = (i, j):  <E_{i, n1+j} + E_{n1+j, i}, X> = 2 M_ij.
    """
    n = n1 + n2
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    m = len(i)
    k = np.arange(m)
    k_idx = np.concatenate([k, k])
    a_idx = np.concatenate([i, n1 + j])
    b_idx = np.concatenate([n1 + j, i])
    col_a, col_b, Abar = _stack_constraints(n, m, k_idx, a_idx, b_idx, np.ones(2 * m))
    C = sp.identity(n, format="csr")
    return SDPProblem(n=n, m=m, C=C, col_a=col_a, col_b=col_b, Abar=Abar,
                      b=2.0 * np.asarray(Mij, dtype=np.float64), kind="completion")


def general_problem(n: int, c_row, c_col, c_val, m: int, a_con, a_row, a_col, a_val, b) -> SDPProblem:
    """min <C, X> s.t. <A_k, X> = b_k (k < m), X psd of order n (the paper's
    problem, eq. prob:sdp, with one block), from triplets of symmetric C and A_k:
    an off-diagonal triplet (r, c, v), r != c, is the pair of entries (r, c)
    and (c, r), both v; repeated triplets add up.  The constraint map is the
    plain inner product <A_k, X> = sum_ab A_k[a, b] X[a, b] over the full
    matrix (both triangles), stacked as in Section 3.3."""
    c_row = np.asarray(c_row, dtype=np.int64)
    c_col = np.asarray(c_col, dtype=np.int64)
    c_val = np.asarray(c_val, dtype=np.float64)
    off = c_row != c_col
    C = sp.csr_matrix((np.concatenate([c_val, c_val[off]]),
                       (np.concatenate([c_row, c_col[off]]), np.concatenate([c_col, c_row[off]]))), shape=(n, n))
    C.sum_duplicates()
    a_con = np.asarray(a_con, dtype=np.int64)
    a_row = np.asarray(a_row, dtype=np.int64)
    a_col = np.asarray(a_col, dtype=np.int64)
    a_val = np.asarray(a_val, dtype=np.float64)
    off = a_row != a_col
    col_a, col_b, Abar = _stack_constraints(
        n, m, np.concatenate([a_con, a_con[off]]), np.concatenate([a_row, a_col[off]]),
        np.concatenate([a_col, a_row[off]]), np.concatenate([a_val, a_val[off]]))
    return SDPProblem(n=n, m=m, C=C, col_a=col_a, col_b=col_b, Abar=Abar,
                      b=np.asarray(b, dtype=np.float64), kind="general")


def general_blocks_problem(block_n, c_blk, c_row, c_col, c_val, m, a_con, a_blk, a_row, a_col, a_val,
                           b, block_rank=None) -> SDPProblem:
    """Several PSD blocks: min sum_j <C_j, X_j> s.t. sum_j <A_kj, X_j> = b_k, read
    as one problem in X = diag(X_1, ..., X_p) with C = diag(C_j) and
    A_k = diag(A_kj) (block_diag of the per-block matrices; the triplet
    convention of general_problem inside each block).  block_rank: the rank of
    each block's factor, X_j = R_j R_j^T with R_j of block_rank[j] columns (the
    multi-block case of appendix A.2, one factor per block variable); the
    rows of block j in the stacked factor hold zeros past column block_rank[j]."""
    block_n = [int(x) for x in block_n]
    c_blk, c_row, c_col, c_val = (np.asarray(x) for x in (c_blk, c_row, c_col, c_val))
    a_con, a_blk, a_row, a_col, a_val = (np.asarray(x) for x in (a_con, a_blk, a_row, a_col, a_val))

    def sym(r, c, v, nj):
        off = r != c
        M = sp.csr_matrix((np.concatenate([v, v[off]]), (np.concatenate([r, c[off]]), np.concatenate([c, r[off]]))),
                          shape=(nj, nj))
        M.sum_duplicates()
        return M

    C = sp.block_diag([sym(c_row[c_blk == j], c_col[c_blk == j], c_val[c_blk == j].astype(np.float64), nj)
                       for j, nj in enumerate(block_n)], format="csr")
    n = sum(block_n)
    k_idx, a_idx, b_idx, vals = [], [], [], []
    for k in range(m):
        sel = a_con == k
        Ak = sp.block_diag([sym(a_row[sel & (a_blk == j)], a_col[sel & (a_blk == j)],
                                a_val[sel & (a_blk == j)].astype(np.float64), nj)
                            for j, nj in enumerate(block_n)], format="coo")
        k_idx.append(np.full(Ak.nnz, k))
        a_idx.append(Ak.row)
        b_idx.append(Ak.col)
        vals.append(Ak.data)
    col_a, col_b, Abar = _stack_constraints(n, m, np.concatenate(k_idx), np.concatenate(a_idx),
                                            np.concatenate(b_idx), np.concatenate(vals))
    row_rank = None if block_rank is None else np.repeat(np.asarray(block_rank, dtype=np.int64), block_n)
    return SDPProblem(n=n, m=m, C=C, col_a=col_a, col_b=col_b, Abar=Abar,
                      b=np.asarray(b, dtype=np.float64), kind="general", row_rank=row_rank)
