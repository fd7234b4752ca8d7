// Device buffer plan of a context: one function computes every allocation so
// that the planning query and the context agree byte for byte.
#pragma once
#include <cstddef>
#include <cstdint>

#include "../../include/kkt.h"
#include "symbolic.hpp"

namespace kkt {

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// restart length of the flexible GMRES refinement
constexpr int KRYLOV_M = 8;
constexpr int KRYLOV_PART = 512;  // partial sums per Krylov reduction
inline bool uses_krylov(const kkt_options &o) { return o.refine_method == KKT_REFINE_FGMRES && o.refine_max > 0; }

struct DevPlan {
    // symbolic maps
    size_t amap, adiag, c0map, c1map, rows, rowptr, snmeta, rel, relptr, perm, pivsign, child;
    // numeric
    size_t L, U, tau, counters, amax;
    size_t S, prefix;          // dense Schur + running sums of S_00
    // solve workspace for nrhs right-hand sides
    size_t xperm, uvec, r, xg, res, dx, norms;
    size_t krylov;             // V, Z bases, coefficients and reduction partials (FGMRES only)
    size_t total_static() const {
        return amap + adiag + c0map + c1map + rows + rowptr + snmeta + rel + relptr + perm + pivsign + child +
               L + U + tau + counters + amax + S + prefix;
    }
    size_t total_solve() const { return xperm + uvec + r + xg + res + dx + norms + krylov; }
};

inline DevPlan make_plan(const Symbolic &Sy, int64_t N, int precision, int64_t nrhs, bool krylov) {
    DevPlan p{};
    const size_t w = precision == 1 ? 4 : 8;  // factor word size (KKT_MIXED = 1)
    const int64_t ng = N * Sy.Ns, nb = Sy.nbord;
    p.amap = align_up(8 * Sy.nnzA);
    p.adiag = align_up(Sy.nnzA);
    p.c0map = align_up(8 * Sy.nnzC0);
    p.c1map = align_up(8 * Sy.nnzC1);
    p.rows = align_up(4 * Sy.rows.size());
    p.rowptr = align_up(8 * (Sy.nsup + 1));
    p.snmeta = align_up(4 * 4 * Sy.nsup) + align_up(8 * 2 * Sy.nsup);  // first,ncol,nrow,parent + Loff,Uoff
    p.rel = align_up(4 * Sy.rel.size());
    p.relptr = align_up(8 * (Sy.nsup + 1));
    p.perm = align_up(4 * Sy.nA);
    p.pivsign = align_up(Sy.nA);
    p.child = align_up(4 * (Sy.nsup + 1)) + align_up(4 * (Sy.child_list.size() + 1));
    p.L = align_up(w * Sy.Lsize * N);
    p.U = align_up(w * Sy.Usize * N);
    p.tau = align_up(8 * Sy.nA * N) + (ng ? align_up(8 * ng) : 0);
    p.counters = align_up(8 * 4 * (N + 1));
    p.amax = align_up(8 * (N + 1));
    p.S = ng ? align_up(8 * ng * ng) : 0;
    p.prefix = ng ? align_up(8 * (N + 1) * Sy.Ns * Sy.Ns) + align_up(8 * 256 * 256) : 0;  // + inverse staging
    // solve workspace
    p.xperm = align_up(8 * (Sy.nA + nb) * N * nrhs);
    p.uvec = align_up(8 * Sy.Usize_vec() * N * nrhs);
    p.r = align_up(8 * (ng + 1) * nrhs);
    p.xg = align_up(8 * (ng + 1) * nrhs);
    int64_t ntot = N * Sy.nA + ng;
    p.res = align_up(8 * ntot * nrhs);
    p.dx = align_up(8 * ntot * nrhs);
    p.norms = align_up(8 * 4 * nrhs + 64) +
              align_up(8 * (N * Sy.Ns * nrhs + 2 * 512 * nrhs + ((Sy.nA + 255) / 256) * N * nrhs + 8));
    const int ldh = KRYLOV_M + 1;
    p.krylov = krylov ? align_up(8 * (2 * KRYLOV_M + 1) * ntot * nrhs) + align_up(8 * 3 * ldh * nrhs + 8 * nrhs) +
                            align_up(8 * (int64_t)KRYLOV_PART * ldh * nrhs)
                      : 0;
    return p;
}

inline size_t device_bytes(const Symbolic &Sy, int64_t N, int precision, int64_t nrhs, bool krylov) {
    DevPlan p = make_plan(Sy, N, precision, nrhs, krylov);
    return p.total_static() + p.total_solve();
}

}  // namespace kkt
