"""Write tests/golden/mesh2000_N96_reference.npz: the FP64 oracle's solution
of the 2000-bus / 96-period / 4-right-hand-side workload, for the full-size
GPU parity tests. Calls only oracle/ and kktgen/ (test infrastructure).

The oracle solves K x = b by Algorithm 1 (section 4.2, Eqs. SCform, SCsolve,
SCsolve1): every period block factored by SuperLU (a library solve
primitive), the local Schur blocks of Eq. LocalSchurBs3 from 2 Ns right-hand
sides per period, S summed per block position (Eq. LocalSchurBs), S factored
by LAPACK's Cholesky of -S (S is negative definite when K has the inertia the
IPM expects, section 2.3), then iterative refinement (section 2.1) with
residuals evaluated in extended precision until they stop improving. The
best relative residual it reaches is what the FP64 solution of this instance
can reach; the stored samples are that solution's entries.

Stored: the residual history, the best relative residual per right-hand
side (extended-precision evaluation) and the FP64-evaluated one, sampled
entries of x (seeded indices in the period rows and the border rows), the
leading 64 x 64 corner of six blocks of S, and check sums of the generated
instance (so a test can tell that it regenerated the same inputs).

Run from the repository root (about ten minutes on 8 cores, 8 GB of memory):
    python tests/golden/make_mesh2000_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import kktgen                                   # noqa: E402
from oracle import arrowhead as ah              # noqa: E402
from oracle import schur as sc                  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mesh2000_N96_reference.npz")
S_BLOCKS = [(0, 0), (1, 0), (95, 0), (47, 47), (95, 47), (95, 95)]


def instance_sums(inst):
    return np.array([inst.vals.sum(), np.abs(inst.vals).sum(), inst.b.sum(), np.abs(inst.b).sum(),
                     inst.C0_vals.sum(), inst.C1_vals.sum()])


def main():
    t0 = time.time()
    inst = kktgen.make_workload(2)
    K = ah.assemble(inst)
    print(f"instance: n = {inst.n_total}, nnz(K) = {K.nnz} ({time.time() - t0:.0f} s)", flush=True)
    out = sc.algorithm1(inst, assembly="prefix", schur_factor="cholesky", dense_limit=0)
    print(f"Algorithm 1 ({time.time() - t0:.0f} s)", flush=True)
    ns = inst.ns
    Sblk = np.zeros((len(S_BLOCKS), 64, 64))
    # S was factored in place; rebuild the sampled blocks from the local blocks
    P = np.zeros((ns, ns))
    pref = [P]
    for n in range(inst.N):
        P = P + out["Sbar"][n][ns:, ns:]
        pref.append(P)
    for q, (m, mp) in enumerate(S_BLOCKS):
        Sb = out["Sbar"][mp]
        blk = pref[mp] + (Sb[:ns, :ns] if m == mp else Sb[ns:, :ns])
        if m == mp:
            blk = blk + np.diag(inst.corner_diag[mp * ns:(mp + 1) * ns])
        Sblk[q] = blk[:64, :64]
    solve = lambda r: sc.algorithm1(inst, b=r, factors=out["factors"], schur=out["schur_fac"])["x"]
    x, hist = sc.refine(inst, out["x"], inst.b, solve, tol=1e-16, maxit=8, K=K, extended=True)
    print(f"refined: history {['%.2e' % h for h in hist]} ({time.time() - t0:.0f} s)", flush=True)
    _, rel_ld = ah.residual_ld(inst, x, inst.b, K)
    r64 = inst.b - (K @ x.T).T
    rel_fp64 = np.linalg.norm(r64, axis=1) / np.linalg.norm(inst.b, axis=1)
    rng = np.random.default_rng(20190712)
    idx_p = np.sort(rng.choice(inst.N * inst.n_A, size=4096, replace=False))
    idx_g = inst.N * inst.n_A + np.sort(rng.choice(inst.n_g, size=2048, replace=False))
    idx = np.concatenate([idx_p, idx_g])
    np.savez_compressed(OUT, hist=np.array(hist), best_rel=rel_ld, rel_fp64=rel_fp64, idx=idx, x=x[:, idx],
                        x_inf=np.max(np.abs(x), axis=1), S_blocks=np.array(S_BLOCKS), S=Sblk,
                        sums=instance_sums(inst))
    print(f"wrote {OUT}: best rel_res {rel_ld} (FP64-evaluated {rel_fp64}) ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
