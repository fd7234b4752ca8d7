// Host-only entry points: options, error strings and the planning query.
#include <algorithm>
#include <cstdio>
#include <cstring>

#include "../../include/kkt.h"
#include "symbolic.hpp"
#include "footprint.hpp"

extern "C" void kkt_default_options(kkt_options *opt) {
    if (!opt) return;
    opt->precision = KKT_FP64;
    opt->pivot_eps = 0.0;
    opt->refine_tol = 1e-10;
    opt->refine_max = 20;
    opt->verbose = 0;
    opt->refine_method = KKT_REFINE_FGMRES;
    opt->big_tile_rows = 0;
    opt->schur_mode = KKT_SCHUR_DENSE;
    opt->recompute_periods = 0;
    opt->dual_wait = 0;
}

extern "C" const char *kkt_strerror(int code) {
    switch (code) {
        case KKT_OK: return "ok";
        case KKT_ERR_ARG: return "bad argument";
        case KKT_ERR_NOMEM: return "out of device memory";
        case KKT_ERR_ORDER: return "wrong call order";
        case KKT_ERR_STRUCT: return "structural problem in the pattern";
        case KKT_ERR_HIP: return "HIP runtime error";
        case KKT_ERR_NONFINITE: return "non-finite input";
        case KKT_ERR_TOOBIG: return "workspace larger than the fixed array of kkt_solve_noalloc";
        case KKT_WARN_PERTURBED: return "warning: pivots perturbed";
        case KKT_WARN_INERTIA: return "warning: inertia differs from the expected one";
        case KKT_WARN_REFINE: return "warning: refinement stopped above tolerance";
        default: return "unknown status";
    }
}

namespace kkt {
SymbolicInput make_input(const kkt_structure *s, const kkt_options &o) {
    SymbolicInput in;
    // FP32 factors cannot absorb the growth that early duals cause
    in.dual_wait = o.dual_wait > 0 ? o.dual_wait : (o.precision == KKT_MIXED ? (1 << 30) : 4);
    in.pair_duals = true;
    in.nA = s->nA;
    in.n_primal = s->n_primal;
    in.Ns = s->Ns;
    in.colptr = s->A_colptr;
    in.rowind = s->A_rowind;
    in.C0p = s->C0_rowptr;
    in.C0i = s->C0_colind;
    in.C1p = s->C1_rowptr;
    in.C1i = s->C1_colind;
    return in;
}

void fill_stats(const Symbolic &S, kkt_symbolic_stats *st) {
    st->n_supernodes = S.nsup;
    st->n_levels = S.nlevels;
    st->nnz_L = S.nnzL;
    st->u_entries = S.Usize;
    st->max_front = S.max_front;
    st->max_pivots = S.max_pivots;
    st->flops_factor = S.flops;
    st->device_bytes = 0;
}
}  // namespace kkt

extern "C" int kkt_plan(const kkt_structure *s, const kkt_options *opt, int64_t nrhs_max,
                        kkt_symbolic_stats *st, int32_t *perm) {
    if (!s || !st || s->N < 1 || s->Ns < 0 || nrhs_max < 1) return KKT_ERR_ARG;
    kkt_options o;
    kkt_default_options(&o);
    if (opt) o = *opt;
    kkt::Symbolic S;
    std::string err;
    try {
        err = kkt::analyze(kkt::make_input(s, o), S);
    } catch (...) {
        return KKT_ERR_NOMEM;
    }
    if (!err.empty()) return KKT_ERR_STRUCT;
    kkt::fill_stats(S, st);
    size_t bytes = 0;
    const int rc = kkt::plan_device_bytes(s, o, nrhs_max, &bytes);
    if (rc) return rc;
    st->device_bytes = (int64_t)bytes;
    if (perm) std::memcpy(perm, S.perm.data(), sizeof(int32_t) * S.nA);
    return KKT_OK;
}
