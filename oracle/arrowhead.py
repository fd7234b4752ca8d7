"""Monolithic assembly of the arrowhead KKT system (test infrastructure only).

K (Eq. hessianPerm, section 4.1) in the ordering u = (u_1, ..., u_N, u_g) of
Eq. orderingMPOPF:

    [ A_1              B_1^T ]
    [      ...          ...  ]
    [           A_N    B_N^T ]
    [ B_1  ...  B_N    C     ]

with the MPOPF border of Eq. B12N: B_n is (N*Ns) x nA with block row m equal
to 0 for m < n, C_1 for m = n and C_0 for m > n (periods numbered 1..N).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def block_lower(inst, n: int) -> sp.csc_matrix:
    """Stored lower triangle of A_n (0-based period n)."""
    return sp.csc_matrix((inst.vals[n], inst.rowind.astype(np.int64), inst.colptr),
                         shape=(inst.n_A, inst.n_A))


def block(inst, n: int) -> sp.csr_matrix:
    """Full symmetric A_n."""
    L = block_lower(inst, n)
    D = sp.diags(L.diagonal())
    return (L + L.T - D).tocsr()


def coupling(inst):
    """(C_0, C_1) as Ns x nA CSR matrices."""
    C0 = sp.csr_matrix((inst.C0_vals, inst.C0_colind.astype(np.int64), inst.C0_rowptr),
                       shape=(inst.ns, inst.n_A))
    C1 = sp.csr_matrix((inst.C1_vals, inst.C1_colind.astype(np.int64), inst.C1_rowptr),
                       shape=(inst.ns, inst.n_A))
    return C0, C1


def border(inst, n: int) -> sp.csr_matrix:
    """B_n of Eq. B12N, 0-based period n: block rows m < n zero, m == n C_1,
    m > n C_0."""
    C0, C1 = coupling(inst)
    rows = []
    for m in range(inst.N):
        if m < n:
            rows.append(sp.csr_matrix((inst.ns, inst.n_A)))
        elif m == n:
            rows.append(C1)
        else:
            rows.append(C0)
    return sp.vstack(rows, format="csr")


def corner(inst) -> sp.csr_matrix:
    return sp.diags(inst.corner_diag).tocsr()


def assemble(inst) -> sp.csr_matrix:
    """The monolithic symmetric KKT matrix K."""
    N = inst.N
    blocks = [[None] * (N + 1) for _ in range(N + 1)]
    for n in range(N):
        blocks[n][n] = block(inst, n)
        if inst.n_g:
            Bn = border(inst, n)
            blocks[N][n] = Bn
            blocks[n][N] = Bn.T
    if inst.n_g:
        blocks[N][N] = corner(inst)
    return sp.bmat(blocks, format="csr")


def split(inst, v: np.ndarray):
    """Split a vector (or [.., n_total] array) in u order into
    ([b_1..b_N] as [N, nA, ...], b_C)."""
    v = np.asarray(v)
    nA, N = inst.n_A, inst.N
    parts = v[..., : N * nA].reshape(v.shape[:-1] + (N, nA))
    return parts, v[..., N * nA:]


def residual(inst, x: np.ndarray, b: np.ndarray, K=None):
    """r = b - K x for x, b of shape [nrhs, n_total]; returns (r, K)."""
    K = assemble(inst) if K is None else K
    r = b - (K @ x.T).T
    return r, K


def rel_residual(inst, x, b, K=None):
    """max over right-hand sides of ||b - K x||_2 / ||b||_2 (FP64)."""
    r, K = residual(inst, x, b, K)
    return float(np.max(np.linalg.norm(r, axis=-1) / np.linalg.norm(b, axis=-1))), K


def residual_ld(inst, x, b, K=None):
    """r = b - K x with the products and sums in extended precision
    (numpy.longdouble, a 64-bit significand on x86), rounded to FP64 at the
    end, and the relative residual ||r||_2 / ||b||_2 of every right-hand side
    from the extended-precision r. This resolves the residual of an FP64 x
    below the rounding error that a plain FP64 evaluation carries
    (eps || |K||x| + |b| ||). Returns (r [nrhs, n], rel [nrhs])."""
    K = (assemble(inst) if K is None else K).tocsr()
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    data = K.data.astype(np.longdouble)
    nonempty = np.diff(K.indptr) > 0
    starts = K.indptr[:-1][nonempty]
    r64 = np.empty_like(b)
    rel = np.empty(b.shape[0])
    for k in range(x.shape[0]):
        prod = data * x[k, K.indices].astype(np.longdouble)
        Kx = np.zeros(K.shape[0], dtype=np.longdouble)
        Kx[nonempty] = np.add.reduceat(prod, starts)     # row sums, in row order
        r = b[k].astype(np.longdouble) - Kx
        r64[k] = r.astype(np.float64)
        bl = b[k].astype(np.longdouble)
        rel[k] = float(np.sqrt(np.sum(r * r)) / np.sqrt(np.sum(bl * bl)))
    return r64, rel


def rel_residual_ld(inst, x, b, K=None):
    """max over right-hand sides of ||b - K x||_2 / ||b||_2 evaluated in
    extended precision (see residual_ld)."""
    return float(np.max(residual_ld(inst, x, b, K)[1]))


def backward_error(inst, x, b, K=None):
    """Componentwise backward error omega = max_i |r_i| / (|K||x| + |b|)_i."""
    K = assemble(inst) if K is None else K
    r = b - (K @ x.T).T
    den = (abs(K) @ np.abs(x).T).T + np.abs(b)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(den > 0, np.abs(r) / den, 0.0)
    return float(np.max(w))


# ----------------------------------------------------------------------------
# line-flow slacks (section 2.1, Eqs. SCOPFslackAtEnd, SCOPFhessianReduced,
# SCOPFslackReduction)
# ----------------------------------------------------------------------------

def assemble_unreduced(inst) -> sp.csr_matrix:
    """K with the eliminated slacks put back: order (u_1..u_N, u_g, s_1..s_N)
    (slacks last, as in Eq. SCOPFslackAtEnd). Slack j of period n has the
    diagonal L_s[n, j] and the entry -1 linking it to its flow row
    lam_row[j] of A_n."""
    sl = inst.meta["slack"]
    K = assemble(inst)
    N, nA, ne = inst.N, inst.n_A, len(sl["lam_row"])
    rows = (np.arange(N)[:, None] * nA + sl["lam_row"][None, :]).ravel()
    E = sp.csr_matrix((-np.ones(N * ne), (rows, np.arange(N * ne))), shape=(K.shape[0], N * ne))
    Ls = sp.diags(sl["Ls"].ravel())
    return sp.bmat([[K, E], [E.T, Ls]], format="csr")


def rhs_unreduced(inst) -> np.ndarray:
    """[b, r_s]: the right-hand sides of the unreduced system."""
    return np.concatenate([inst.b, inst.meta["slack"]["rs"]], axis=1)


def reduce_slacks(inst):
    """The reduced system of Eq. SCOPFhessianReduced: eliminating slack j
    (row  -lambda_I,j + L_s,j s_j = r_j) subtracts 1/L_s,j from the diagonal
    of its flow row and adds r_j / L_s,j to that row's right-hand side.
    Returns a copy of inst with those values and right-hand sides."""
    import copy
    sl = inst.meta["slack"]
    out = copy.copy(inst)
    vals = inst.vals.copy()
    b = inst.b.copy()
    N, nA, ne = inst.N, inst.n_A, len(sl["lam_row"])
    diag_pos = inst.colptr[sl["lam_row"]]           # the diagonal leads its column
    vals[:, diag_pos] -= 1.0 / sl["Ls"]
    rs = sl["rs"].reshape(-1, N, ne)
    for n in range(N):
        b[:, n * nA + sl["lam_row"]] += rs[:, n, :] / sl["Ls"][n]
    out.vals, out.b = vals, b
    return out


def recover_slacks(inst, x) -> np.ndarray:
    """Eq. SCOPFslackReduction: L_s,j s_j = r_j + lambda_I,j, from the solution
    x of the reduced system. Returns [nrhs, N * n_elim]."""
    sl = inst.meta["slack"]
    x = np.atleast_2d(x)
    N, nA, ne = inst.N, inst.n_A, len(sl["lam_row"])
    lam = np.stack([x[:, n * nA + sl["lam_row"]] for n in range(N)], axis=1)   # [nrhs, N, ne]
    return ((sl["rs"].reshape(-1, N, ne) + lam) / sl["Ls"][None]).reshape(x.shape[0], N * ne)
