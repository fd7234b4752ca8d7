"""Algorithm 1: Schur-complement decomposition of the arrowhead KKT system
(test infrastructure only; section 4.2, Eqs. SCform, SCsolve, SCsolve1, and
the MPOPF local Schur structure of section 4.3, Eqs. LocalSchurBs,
LocalSchurBs3), and the structured elimination of S of section 4.3.

Readings of the paper (the equations win where the algorithm listing differs):
  * Sign convention: S = C - sum_i B_i A_i^-1 B_i^T (Eq. SCform); the
    per-period contribution of section 4.3 is S_n := -B_n A_n^-1 B_n^T, so
    S = C + sum_n S_n.
  * Local solve: A_i du_i = b_i - B_i^T du_g (Eq. SCsolve1); the listing's
    final step has the sign and the transpose the other way round.
  * r = sum_i B_i A_i^-1 b_i and S du_g = b_C - r (Eq. SCsolve).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import arrowhead as ah
from .ldlt import ldlt, ldlt_solve, inertia_from_d


class BlockFactor:
    """Factor of one diagonal block A_n: the oracle's own dense LDL^T for
    small blocks (with inertia), else SuperLU as a library solve primitive
    (the solution A_n^-1 y is unique, inertia is then not reported): with
    diagonal pivots by default, or with threshold partial pivoting
    (pivot_thresh > 0, a stabler preconditioner for refinement on badly
    scaled blocks)."""

    def __init__(self, A: sp.spmatrix, n_primal: int, dense_limit: int = 2500, eps: float = 1e-20,
                 pivot_thresh: float = 0.0):
        n = A.shape[0]
        self.n = n
        if n <= dense_limit:
            signs = np.where(np.arange(n) < n_primal, 1.0, -1.0)
            self.L, self.d, self.n_perturbed, raw = ldlt(A.toarray(), signs=signs, eps=eps, return_raw=True)
            self.inertia = inertia_from_d(raw)
            self.kind = "dense"
        elif pivot_thresh > 0.0:
            self.lu = spla.splu(A.tocsc(), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=pivot_thresh)
            self.inertia = None
            self.n_perturbed = 0
            self.kind = "splu"
        else:
            self.lu = spla.splu(A.tocsc(), permc_spec="MMD_AT_PLUS_A",
                                diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
            self.inertia = None
            self.n_perturbed = 0
            self.kind = "splu"

    def solve(self, y: np.ndarray) -> np.ndarray:
        """A_n^-1 y for y of shape [n] or [n, k]."""
        if self.kind == "dense":
            return ldlt_solve(self.L, self.d, y)
        return self.lu.solve(np.asarray(y, dtype=np.float64))


def local_schur_bar(inst, Fn: BlockFactor) -> np.ndarray:
    """S_bar_n = [[S_11, S_10^T], [S_10, S_00]] with S_ij = -C_i A_n^-1 C_j^T
    (Eq. LocalSchurBs3): 2*Ns right-hand sides [C_1^T C_0^T]."""
    C0, C1 = ah.coupling(inst)
    Chat = sp.vstack([C1, C0]).tocsr()           # 2Ns x nA
    W = Fn.solve(Chat.T.toarray())               # nA x 2Ns = A^-1 Chat^T
    return -(Chat @ W)


def place_local_schur(inst, n: int, Sbar: np.ndarray) -> np.ndarray:
    """Dense S_n (n_g x n_g) of Eq. LocalSchurBs for 0-based period n: zero in
    block rows/cols m < n, S_11 at (n, n), S_10 at (m, n) for m > n, S_00 at
    (m, m') for m, m' > n (plus the transposes above the diagonal)."""
    ns, N = inst.ns, inst.N
    S11, S10, S00 = Sbar[:ns, :ns], Sbar[ns:, :ns], Sbar[ns:, ns:]
    Sn = np.zeros((inst.n_g, inst.n_g))
    blk = lambda m: slice(m * ns, (m + 1) * ns)
    Sn[blk(n), blk(n)] = S11
    for m in range(n + 1, N):
        Sn[blk(m), blk(n)] = S10
        Sn[blk(n), blk(m)] = S10.T
        for mp in range(n + 1, N):
            Sn[blk(m), blk(mp)] = S00
    return Sn


def assemble_schur_prefix(inst, Sbar) -> np.ndarray:
    """S = C + sum_n S_n with each S_n placed as Eq. LocalSchurBs places it,
    summed block by block instead of matrix by matrix: block (m, m) collects
    S_11 of period m and S_00 of every earlier period; block (m, m') below
    the diagonal (m > m') collects S_10 of period m' and S_00 of every period
    before m' (Eq. GlobalSchur: the same matrix for every m > m'). Both
    triangles are filled. O(n_g^2) memory without forming any S_n."""
    ns, N = inst.ns, inst.N
    S = np.zeros((inst.n_g, inst.n_g))
    blk = lambda m: slice(m * ns, (m + 1) * ns)
    P = np.zeros((ns, ns))                    # sum of S_00,n over n < m'
    for mp in range(N):
        S11, S10, S00 = Sbar[mp][:ns, :ns], Sbar[mp][ns:, :ns], Sbar[mp][ns:, ns:]
        S[blk(mp), blk(mp)] = P + S11
        below = P + S10
        for m in range(mp + 1, N):
            S[blk(m), blk(mp)] = below
            S[blk(mp), blk(m)] = below.T
        P = P + S00
    S[np.diag_indices(inst.n_g)] += inst.corner_diag
    return S


def algorithm1(inst, b=None, structured: bool = True, dense_limit: int = 2500, eps: float = 1e-20,
               factors=None, assembly: str = "place", schur_factor: str = "ldlt", pivot_thresh: float = 0.0,
               schur=None):
    """Solve K x = b by Algorithm 1 on one process. Returns a dict with x
    ([nrhs, n_total]), S (dense n_g x n_g), Sbar ([N, 2Ns, 2Ns], structured
    only), r ([nrhs, n_g]), ug, the block factors, inertia (when every block
    was factored densely) and the perturbed-pivot count.

    assembly "place" adds every S_n as an n_g x n_g matrix; "prefix" sums the
    same blocks per block position (assemble_schur_prefix), for large n_g.
    schur_factor "ldlt" is the oracle's own LDL^T of S; "cholesky" is LAPACK's
    Cholesky of -S (a library primitive; S is negative definite whenever
    every A_n and K have the inertia the IPM expects, and the call fails
    otherwise), for large n_g. A later call can pass the returned factors
    and `schur` (the returned dict's "schur_fac") to solve other
    right-hand sides without refactoring."""
    b = inst.b if b is None else np.atleast_2d(b)
    N, nA, ng = inst.N, inst.n_A, inst.n_g
    bparts, bC = ah.split(inst, b)              # [nrhs, N, nA], [nrhs, n_g]
    # step 2: factor every diagonal block
    if factors is None:
        factors = [BlockFactor(ah.block(inst, n), inst.n_primal, dense_limit, eps, pivot_thresh)
                   for n in range(N)]
    # steps 3-6: Schur complement S = C - sum_n B_n A_n^-1 B_n^T
    Sbar = np.zeros((N, 2 * inst.ns, 2 * inst.ns))
    if schur is not None:
        S = None
    elif assembly == "prefix":
        for n in range(N):
            Sbar[n] = local_schur_bar(inst, factors[n])
        S = assemble_schur_prefix(inst, Sbar) if ng else np.zeros((0, 0))
    else:
        S = np.diag(inst.corner_diag).astype(np.float64)
        if ng:
            for n in range(N):
                if structured:
                    Sbar[n] = local_schur_bar(inst, factors[n])
                    S += place_local_schur(inst, n, Sbar[n])
                else:
                    Bn = ah.border(inst, n)
                    S -= Bn @ factors[n].solve(Bn.T.toarray())
    # steps 8-11: r = sum_n B_n A_n^-1 b_n
    y = np.stack([factors[n].solve(bparts[:, n, :].T).T.reshape(b.shape[0], nA) for n in range(N)], 1)
    r = np.zeros((b.shape[0], ng))
    if ng:
        for n in range(N):
            r += (ah.border(inst, n) @ y[:, n, :].T).T
    # steps 12-13: S = L_s D_s L_s^T, solve S du_g = b_C - r
    import scipy.linalg as sl
    schur_fac = schur
    if ng and (schur_factor == "cholesky" or (schur is not None and schur[0] == "cholesky")):
        if schur_fac is None:
            S *= -1.0                                # in place: -S, then its Cholesky factor
            schur_fac = ("cholesky", sl.cho_factor(S, lower=True, overwrite_a=True, check_finite=False))
            S = None
        ug = -sl.cho_solve(schur_fac[1], (bC - r).T, check_finite=False).T
        ds = raw_s = -np.ones(ng)                    # Cholesky of -S succeeded: S negative definite
        npert_s = 0
    elif ng:
        if schur_fac is None:
            Ls, ds, npert_s, raw_s = ldlt(S, signs=-np.ones(ng), eps=eps, return_raw=True)
            schur_fac = ("ldlt", (Ls, ds, npert_s, raw_s))
        Ls, ds, npert_s, raw_s = schur_fac[1]
        ug = ldlt_solve(Ls, ds, (bC - r).T).T
    else:
        ds = raw_s = np.zeros(0)
        npert_s = 0
        ug = np.zeros((b.shape[0], 0))
    # step 16: A_n du_n = b_n - B_n^T du_g
    x = np.zeros_like(b, dtype=np.float64)
    for n in range(N):
        rhs = bparts[:, n, :]
        if ng:
            rhs = rhs - (ah.border(inst, n).T @ ug.T).T
        x[:, n * nA:(n + 1) * nA] = factors[n].solve(rhs.T).T.reshape(b.shape[0], nA)
    x[:, N * nA:] = ug
    inertia = None
    if all(f.inertia is not None for f in factors):
        pos = sum(f.inertia[0] for f in factors)
        neg = sum(f.inertia[1] for f in factors)
        zer = sum(f.inertia[2] for f in factors)
        ps, ns_, zs = inertia_from_d(raw_s)
        inertia = (pos + ps, neg + ns_, zer + zs)
    return dict(x=x, S=S, Sbar=Sbar if (structured or assembly == "prefix") else None, r=r, ug=ug,
                factors=factors, inertia=inertia, schur_d=ds, schur_fac=schur_fac,
                n_perturbed=sum(f.n_perturbed for f in factors) + npert_s)


def structured_schur_solve(S, N: int, ns: int, rhs, eps: float = 1e-20):
    """Solve S x = rhs by block elimination over the N block columns of S
    (section 4.3, Eq. GlobalSchur): every block below the diagonal of block
    column j is the same N_s x N_s matrix S_o[j] (the block just below the
    diagonal), so eliminating columns 0..j-1 subtracts one common matrix U_j
    from every trailing block. Reading (the paper states the structure and
    the complexity, not these steps): with U_0 = 0,
        A_j = S_jj - U_j,  B_j = S_o[j] - U_j,  U_{j+1} = U_j + B_j A_j^-1 B_j^T,
    A_j = L_j D_j L_j^T (the oracle's LDL^T and pivot rule), and every block of
    the block factor below the diagonal of column j equals
    W_j = B_j L_j^-T D_j^-1. Forward: z_j = L_j^-1 (r_j - s_j) with the running
    sum s_{j+1} = s_j + W_j z_j; then w = z / D; backward:
    x_j = L_j^-T (w_j - W_j^T t_j) with t_j = sum_{m>j} x_m.
    Returns x ([nrhs, N ns]), the inertia (sum over the pivot blocks) and the
    list of U_j."""
    rhs = np.atleast_2d(np.asarray(rhs, dtype=np.float64))
    blk = lambda a, i, j: a[i * ns:(i + 1) * ns, j * ns:(j + 1) * ns]
    U = np.zeros((ns, ns))
    Ls, ds, Ws, Us, raws = [], [], [], [], []
    for j in range(N):
        Us.append(U.copy())
        A = blk(S, j, j) - U
        L, d, _, raw = ldlt(A, signs=-np.ones(ns), eps=eps, return_raw=True)
        Ls.append(L)
        ds.append(d)
        raws.append(raw)
        if j + 1 < N:
            B = blk(S, j + 1, j) - U
            # W = B L^-T D^-1, i.e. W D L^T = B
            W = np.linalg.solve(L, B.T).T / d
            Ws.append(W)
            U = U + (W * d) @ W.T
    x = np.zeros_like(rhs)
    z = np.zeros_like(rhs)
    s = np.zeros((rhs.shape[0], ns))
    for j in range(N):
        z[:, j * ns:(j + 1) * ns] = np.linalg.solve(Ls[j], (rhs[:, j * ns:(j + 1) * ns] - s).T).T
        if j + 1 < N:
            s = s + (Ws[j] @ z[:, j * ns:(j + 1) * ns].T).T
    t = np.zeros((rhs.shape[0], ns))
    for j in range(N - 1, -1, -1):
        w = z[:, j * ns:(j + 1) * ns] / ds[j]
        v = w - (Ws[j].T @ t.T).T if j + 1 < N else w
        x[:, j * ns:(j + 1) * ns] = np.linalg.solve(Ls[j].T, v.T).T
        t = t + x[:, j * ns:(j + 1) * ns]
    inertia = tuple(int(sum(inertia_from_d(r)[k] for r in raws)) for k in range(3))
    return x, inertia, Us


def solve_mono(inst, b=None, dense_limit: int = 4000):
    """Monolithic reference: assemble K and solve it directly (LAPACK
    dgesv when dense, SuperLU otherwise)."""
    b = inst.b if b is None else np.atleast_2d(b)
    K = ah.assemble(inst)
    if K.shape[0] <= dense_limit:
        x = np.linalg.solve(K.toarray(), b.T).T
    else:
        lu = spla.splu(K.tocsc(), permc_spec="MMD_AT_PLUS_A")
        x = lu.solve(b.T).T
    return x, K


def refine(inst, x, b, solve_fn, tol: float = 1e-12, maxit: int = 10, K=None, extended: bool = False):
    """Iterative refinement x <- x + solve(b - K x) (section 2.1) until the
    relative residual is below tol, stagnates (no 2x gain over two steps) or
    maxit. The residual is evaluated in FP64, or with `extended` in extended
    precision (arrowhead.residual_ld), which lets x approach the correctly
    rounded FP64 solution. Returns (x, history of relative residuals)."""
    K = ah.assemble(inst) if K is None else K
    hist = []
    for it in range(maxit + 1):
        if extended:
            r, rels = ah.residual_ld(inst, x, b, K)
            rel = float(np.max(rels))
        else:
            r = b - (K @ x.T).T
            rel = float(np.max(np.linalg.norm(r, axis=-1) / np.linalg.norm(b, axis=-1)))
        hist.append(rel)
        if rel <= tol or it == maxit:
            break
        if len(hist) >= 3 and hist[-1] > 0.5 * hist[-3]:
            break
        x = x + solve_fn(r)
    return x, hist
