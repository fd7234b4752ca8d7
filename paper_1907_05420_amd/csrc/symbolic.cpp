// Host-side symbolic analysis: ordering, elimination tree, supernodes, maps.
#include "symbolic.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <numeric>

namespace kkt {

// ---------------------------------------------------------------------------
// Approximate minimum degree on a quotient graph (variables + elements), with
// element absorption, aggressive absorption, supervariable detection and
// mass elimination (Amestoy, Davis & Duff's approximate external degree:
// d(i) <= |A_i| + |L_p \ i| + sum_{e in E_i, e != p} |L_e \ L_p|). When a new
// element covers every remaining variable the rest is a clique and is
// appended, primals first. Duals (i >= n_primal) become eligible only after a
// few of their primal neighbours are eliminated (see `need` below).
// ---------------------------------------------------------------------------
std::vector<int32_t> amd_order(int32_t n, const std::vector<int64_t> &xadj,
                               const std::vector<int32_t> &adj, int64_t n_primal, int dual_wait, bool pair_duals) {
    std::vector<std::vector<int32_t>> Av(n), Ev(n), Le(n), members(n);
    std::vector<int32_t> nv(n, 1), deg(n), status(n, 0);  // 0 var, 1 element, 2 dead
    // dual eligibility: number of primal neighbours not yet eliminated
    const bool constrained = n_primal >= 0;
    std::vector<int32_t> blocked(n, 0);
    std::vector<char> inb(n, 0);  // in a degree bucket
    auto is_dual = [&](int32_t i) { return constrained && i >= n_primal; };
    // A dual (negative pivot -delta_c - ...) eliminated before any of its
    // primal neighbours has the bare regularisation -delta_c as its pivot and
    // feeds updates of size |J|^2/delta_c into the primal pivots. Waiting for
    // four primal neighbours keeps the fill of the unconstrained order on the
    // MPOPF blocks and leaves growth that FP64 refinement absorbs; waiting for
    // all of them (the FP32 factors need it) removes the growth but multiplies
    // the fill.
    const int need = dual_wait;
    if (constrained)
        for (int32_t i = 0; i < n; ++i)
            if (is_dual(i)) {
                for (int64_t k = xadj[i]; k < xadj[i + 1]; ++k)
                    if (!is_dual(adj[k])) blocked[i]++;
                if (need > 0) blocked[i] = std::min(blocked[i], need);
            }
    std::vector<int32_t> head(n + 1, -1), nxt(n, -1), prv(n, -1);
    std::vector<int64_t> mark(n, -1), wst(n, -1);
    std::vector<int64_t> w(n, 0);
    int64_t stamp = 0, estamp = 0;
    for (int32_t i = 0; i < n; ++i) {
        Av[i].assign(adj.begin() + xadj[i], adj.begin() + xadj[i + 1]);
        deg[i] = (int32_t)Av[i].size();
        members[i].push_back(i);
    }
    int32_t mindeg = 0;
    auto bucket_insert = [&](int32_t i) {
        if (blocked[i] > 0 || inb[i]) return;
        int32_t d = std::min<int32_t>(std::max<int32_t>(deg[i], 0), n);
        nxt[i] = head[d];
        prv[i] = -1;
        if (head[d] >= 0) prv[head[d]] = i;
        head[d] = i;
        inb[i] = 1;
        mindeg = std::min(mindeg, d);
    };
    auto bucket_remove = [&](int32_t i) {
        if (!inb[i]) return;
        int32_t d = std::min<int32_t>(std::max<int32_t>(deg[i], 0), n);
        if (prv[i] >= 0) nxt[prv[i]] = nxt[i]; else head[d] = nxt[i];
        if (nxt[i] >= 0) prv[nxt[i]] = prv[i];
        nxt[i] = prv[i] = -1;
        inb[i] = 0;
    };
    // merged supervariables keep one representative; a dual's eligibility is
    // tracked on its representative (members of a supervariable share kind)
    std::vector<int32_t> rep(n);
    for (int32_t i = 0; i < n; ++i) rep[i] = i;
    auto find = [&](int32_t r) { while (rep[r] != r) r = rep[r]; return r; };
    // an original primal variable was eliminated: release its dual neighbours
    std::vector<int32_t> released;
    auto release = [&](int32_t v) {
        if (!constrained || is_dual(v)) return;
        for (int64_t k = xadj[v]; k < xadj[v + 1]; ++k) {
            int32_t w = adj[k];
            if (!is_dual(w)) continue;
            int32_t r = find(w);
            if (status[r] == 0 && blocked[r] > 0 && --blocked[r] == 0) released.push_back(r);
        }
    };
    for (int32_t i = 0; i < n; ++i) bucket_insert(i);
    // Pairing of duals with eliminated primals: a dual (supervariable of m
    // duals) is eliminated only when it can claim m eliminated primal
    // neighbours that no earlier dual claimed (greedily, the partners that
    // the fewest other duals still wait for first). Eliminated duals then
    // never outnumber the eliminated primals they touch, so the dual block of
    // the partial Schur complement (-delta_c - J_E H_EE^-1 J_E^T restricted
    // to them) keeps full structural rank; without it, a dual eliminated
    // after others that share its few eliminated primal neighbours (the P-
    // and Q-balance rows of adjacent buses share their (theta, V) columns) is
    // left with a pivot near -delta_c and the factor with growth near
    // 1/delta_c. A dual that cannot claim waits for its next primal
    // neighbour; if none is left it is forced (no deadlock). Measured on
    // the MPOPF blocks: growth 1e8 -> <= 3e5 at 10% less fill than without
    // pairing (claims that augmenting paths may move between duals delay
    // fewer duals and measured worse: growth 1e6, the unpaired fill).
    std::vector<char> elim(n, 0), claimed(n, 0), forced(n, 0);
    std::vector<int32_t> waiting_duals(n, 0);  // per primal: original dual neighbours not yet eliminated
    if (pair_duals && constrained)
        for (int32_t i = 0; i < n; ++i)
            if (!is_dual(i))
                for (int64_t k = xadj[i]; k < xadj[i + 1]; ++k)
                    if (is_dual(adj[k])) waiting_duals[i]++;
    std::vector<int32_t> cand;
    std::vector<int64_t> cmark(n, -1);
    int64_t cstamp = 0;
    // claim partners for dual supervariable p; false when too few are free
    auto claim = [&](int32_t p) {
        ++cstamp;
        cand.clear();
        for (int32_t v : members[p])
            for (int64_t k = xadj[v]; k < xadj[v + 1]; ++k) {
                const int32_t u = adj[k];
                if (is_dual(u) || !elim[u] || claimed[u] || cmark[u] == cstamp) continue;
                cmark[u] = cstamp;
                cand.push_back(u);
            }
        const size_t m = members[p].size();
        if (cand.size() < m) return false;
        std::sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
            return waiting_duals[a] != waiting_duals[b] ? waiting_duals[a] < waiting_duals[b] : a < b;
        });
        for (size_t q = 0; q < m; ++q) claimed[cand[q]] = 1;
        return true;
    };
    std::vector<int32_t> order;
    order.reserve(n);
    int64_t nel = 0;
    std::vector<int32_t> Lp;
    std::vector<std::pair<int64_t, int32_t>> hv;
    while (nel < n) {
        while (mindeg <= n && head[mindeg] < 0) ++mindeg;
        if (mindeg > n) {
            // only duals that cannot claim a partner are left: force them
            bool any = false;
            for (int32_t i = 0; i < n; ++i)
                if (status[i] == 0 && blocked[i] > 0) {
                    blocked[i] = 0;
                    forced[i] = 1;
                    bucket_insert(i);
                    any = true;
                }
            if (!any) break;  // cannot happen
            continue;
        }
        int32_t p = head[mindeg];
        bucket_remove(p);
        if (pair_duals && is_dual(p) && !forced[p] && !claim(p)) {
            blocked[p] = 1;  // eligible again after its next primal neighbour
            continue;
        }
        // new element L_p
        ++stamp;
        mark[p] = stamp;
        Lp.clear();
        int64_t lpw = 0;
        for (int32_t e : Ev[p]) {
            if (status[e] != 1) continue;
            for (int32_t j : Le[e])
                if (status[j] == 0 && mark[j] != stamp) { mark[j] = stamp; Lp.push_back(j); lpw += nv[j]; }
            status[e] = 2;
            std::vector<int32_t>().swap(Le[e]);
        }
        for (int32_t j : Av[p])
            if (status[j] == 0 && mark[j] != stamp) { mark[j] = stamp; Lp.push_back(j); lpw += nv[j]; }
        status[p] = 1;
        std::vector<int32_t>().swap(Av[p]);
        std::vector<int32_t>().swap(Ev[p]);
        for (int32_t v : members[p]) {
            order.push_back(v);
            elim[v] = 1;
            release(v);
            if (pair_duals && is_dual(v))
                for (int64_t k = xadj[v]; k < xadj[v + 1]; ++k)
                    if (!is_dual(adj[k])) waiting_duals[adj[k]]--;
        }
        nel += nv[p];
        if (lpw == n - nel) {  // remaining graph is a clique: primals, then duals
            for (int pass = 0; pass < 2; ++pass)
                for (int32_t j : Lp) {
                    if ((pass == 0) == is_dual(j)) continue;
                    bucket_remove(j);
                    for (int32_t v : members[j]) order.push_back(v);
                    nel += nv[j];
                    status[j] = 2;
                }
            break;
        }
        for (int32_t j : Lp) bucket_remove(j);
        // |L_e \ L_p| for every element adjacent to L_p (pruning dead entries)
        ++estamp;
        for (int32_t j : Lp)
            for (int32_t e : Ev[j]) {
                if (status[e] != 1 || e == p || wst[e] == estamp) continue;
                wst[e] = estamp;
                int64_t ww = 0;
                size_t k = 0;
                auto &L = Le[e];
                for (int32_t v : L)
                    if (status[v] == 0) { L[k++] = v; if (mark[v] != stamp) ww += nv[v]; }
                L.resize(k);
                w[e] = ww;
            }
        for (int32_t j : Lp) {
            int64_t ext = 0;
            size_t k = 0;
            auto &E = Ev[j];
            for (int32_t e : E) {
                if (status[e] != 1 || e == p) continue;
                if (w[e] == 0) { status[e] = 2; std::vector<int32_t>().swap(Le[e]); continue; }
                E[k++] = e;
                ext += w[e];
            }
            E.resize(k);
            E.push_back(p);
            int64_t adeg = 0;
            auto &A = Av[j];
            k = 0;
            for (int32_t v : A)
                if (status[v] == 0 && mark[v] != stamp) { A[k++] = v; adeg += nv[v]; }
            A.resize(k);
            int64_t d = std::min<int64_t>(n - nel - nv[j], (int64_t)deg[j] + lpw - nv[j]);
            d = std::min<int64_t>(d, adeg + lpw - nv[j] + ext);
            deg[j] = (int32_t)std::max<int64_t>(d, 0);
        }
        // supervariables: equal (E_j, A_j) sets
        hv.clear();
        for (int32_t j : Lp) {
            std::sort(Ev[j].begin(), Ev[j].end());
            std::sort(Av[j].begin(), Av[j].end());
            int64_t h = 0;
            for (int32_t e : Ev[j]) h += e;
            for (int32_t v : Av[j]) h += v;
            h = (h % 1000003) * 64 + (int64_t)(Ev[j].size() % 8) * 8 + (int64_t)(Av[j].size() % 8);
            hv.emplace_back(h, j);
        }
        std::sort(hv.begin(), hv.end());
        for (size_t a = 0; a < hv.size();) {
            size_t b = a;
            while (b < hv.size() && hv[b].first == hv[a].first) ++b;
            for (size_t x = a; x < b; ++x) {
                int32_t i = hv[x].second;
                if (status[i] != 0) continue;
                for (size_t y = x + 1; y < b; ++y) {
                    int32_t j = hv[y].second;
                    if (status[j] != 0) continue;
                    if (is_dual(i) != is_dual(j) || (blocked[i] > 0) != (blocked[j] > 0)) continue;
                    if (Ev[i] == Ev[j] && Av[i] == Av[j]) {
                        nv[i] += nv[j];
                        deg[i] = std::max<int32_t>(deg[i] - nv[j], 0);
                        if (constrained && is_dual(i)) blocked[i] += blocked[j];
                        members[i].insert(members[i].end(), members[j].begin(), members[j].end());
                        std::vector<int32_t>().swap(members[j]);
                        rep[j] = i;
                        nv[j] = 0;
                        status[j] = 2;
                        std::vector<int32_t>().swap(Ev[j]);
                        std::vector<int32_t>().swap(Av[j]);
                    }
                }
            }
            a = b;
        }
        auto &L = Le[p];
        for (int32_t j : Lp)
            if (status[j] == 0) {
                L.push_back(j);
                bucket_insert(j);
            }
        // duals whose last primal neighbour just went: eligible now
        for (int32_t w : released) {
            int32_t r = find(w);
            if (status[r] == 0 && blocked[r] <= 0) bucket_insert(r);
        }
        released.clear();
    }
    return order;
}

// ---------------------------------------------------------------------------

static bool check_input(const SymbolicInput &in, std::string &err) {
    if (in.nA <= 0 || !in.colptr || !in.rowind) { err = "empty block"; return false; }
    if (in.n_primal < 0 || in.n_primal > in.nA) { err = "n_primal out of range"; return false; }
    if (in.colptr[0] != 0) { err = "colptr[0] != 0"; return false; }
    for (int64_t j = 0; j < in.nA; ++j) {
        int64_t a = in.colptr[j], b = in.colptr[j + 1];
        if (b <= a) { err = "empty column " + std::to_string(j); return false; }
        if (in.rowind[a] != j) { err = "missing or misplaced diagonal in column " + std::to_string(j); return false; }
        for (int64_t k = a; k < b; ++k) {
            if (in.rowind[k] < j || in.rowind[k] >= in.nA) { err = "entry outside the lower triangle"; return false; }
            if (k > a && in.rowind[k] <= in.rowind[k - 1]) { err = "unsorted or duplicate row index"; return false; }
        }
    }
    if (in.Ns > 0) {
        for (int w = 0; w < 2; ++w) {
            const int64_t *p = w ? in.C1p : in.C0p;
            const int32_t *c = w ? in.C1i : in.C0i;
            if (!p || !c) { err = "missing C pattern"; return false; }
            if (p[0] != 0) { err = "C rowptr[0] != 0"; return false; }
            for (int64_t s = 0; s < in.Ns; ++s) {
                if (p[s + 1] < p[s]) { err = "C rowptr decreasing"; return false; }
                for (int64_t k = p[s]; k < p[s + 1]; ++k) {
                    if (c[k] < 0 || c[k] >= in.nA) { err = "C column out of range"; return false; }
                    if (k > p[s] && c[k] <= c[k - 1]) { err = "C columns unsorted or duplicate"; return false; }
                }
            }
        }
    }
    return true;
}

std::string analyze(const SymbolicInput &in, Symbolic &S) {
    std::string err;
    if (!check_input(in, err)) return err;
    const int64_t nA = in.nA, Ns = in.Ns, nb = 2 * Ns, n = nA + nb;
    S = Symbolic();
    S.nA = nA; S.n_primal = in.n_primal; S.Ns = Ns; S.nbord = nb; S.n = n;
    S.nnzA = in.colptr[nA];
    S.nnzC0 = Ns ? in.C0p[Ns] : 0;
    S.nnzC1 = Ns ? in.C1p[Ns] : 0;

    // --- symmetric adjacency of A (old numbering) ---------------------------
    std::vector<int64_t> cnt(nA + 1, 0);
    for (int64_t j = 0; j < nA; ++j)
        for (int64_t k = in.colptr[j] + 1; k < in.colptr[j + 1]; ++k) { cnt[j]++; cnt[in.rowind[k]]++; }
    std::vector<int64_t> xadj(nA + 1, 0);
    for (int64_t i = 0; i < nA; ++i) xadj[i + 1] = xadj[i] + cnt[i];
    std::vector<int32_t> adj(xadj[nA]);
    std::vector<int64_t> pos(xadj.begin(), xadj.end() - 1);
    for (int64_t j = 0; j < nA; ++j)
        for (int64_t k = in.colptr[j] + 1; k < in.colptr[j + 1]; ++k) {
            int32_t i = in.rowind[k];
            adj[pos[j]++] = i;
            adj[pos[i]++] = (int32_t)j;
        }
    std::vector<int32_t> perm = amd_order((int32_t)nA, xadj, adj, in.n_primal, in.dual_wait, in.pair_duals);
    if ((int64_t)perm.size() != nA) return "ordering failed";

    // --- lower pattern of M by rows in a given order --------------------------
    auto build_rows = [&](const std::vector<int32_t> &ip, std::vector<int64_t> &rp, std::vector<int32_t> &ci) {
        std::vector<int64_t> c(n + 1, 0);
        for (int64_t j = 0; j < nA; ++j)
            for (int64_t k = in.colptr[j] + 1; k < in.colptr[j + 1]; ++k) {
                int32_t a = ip[in.rowind[k]], b = ip[j];
                c[std::max(a, b) + 1]++;
            }
        for (int64_t s = 0; s < Ns; ++s) {
            c[nA + s + 1] += in.C1p[s + 1] - in.C1p[s];
            c[nA + Ns + s + 1] += in.C0p[s + 1] - in.C0p[s];
        }
        rp.assign(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) rp[i + 1] = rp[i] + c[i + 1];
        ci.assign(rp[n], 0);
        std::vector<int64_t> q(rp.begin(), rp.end() - 1);
        for (int64_t j = 0; j < nA; ++j)
            for (int64_t k = in.colptr[j] + 1; k < in.colptr[j + 1]; ++k) {
                int32_t a = ip[in.rowind[k]], b = ip[j];
                ci[q[std::max(a, b)]++] = std::min(a, b);
            }
        for (int64_t s = 0; s < Ns; ++s) {
            for (int64_t k = in.C1p[s]; k < in.C1p[s + 1]; ++k) ci[q[nA + s]++] = ip[in.C1i[k]];
            for (int64_t k = in.C0p[s]; k < in.C0p[s + 1]; ++k) ci[q[nA + Ns + s]++] = ip[in.C0i[k]];
        }
    };
    auto etree = [&](const std::vector<int64_t> &rp, const std::vector<int32_t> &ci, std::vector<int32_t> &par) {
        par.assign(nA, -1);
        std::vector<int32_t> anc(nA, -1);
        for (int64_t i = 0; i < nA; ++i)
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
                int32_t r = ci[k];
                while (anc[r] != -1 && anc[r] != i) { int32_t t = anc[r]; anc[r] = (int32_t)i; r = t; }
                if (anc[r] == -1) { anc[r] = (int32_t)i; par[r] = (int32_t)i; }
            }
    };
    std::vector<int32_t> iperm(nA);
    for (int64_t k = 0; k < nA; ++k) iperm[perm[k]] = (int32_t)k;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci, par;
    build_rows(iperm, rp, ci);
    etree(rp, ci, par);
    // --- postorder the elimination tree and renumber --------------------------
    {
        std::vector<int32_t> chead(nA, -1), cnext(nA, -1);
        for (int64_t j = nA - 1; j >= 0; --j)
            if (par[j] >= 0) { cnext[j] = chead[par[j]]; chead[par[j]] = (int32_t)j; }
        std::vector<int32_t> post;
        post.reserve(nA);
        std::vector<int32_t> stack;
        for (int64_t r = 0; r < nA; ++r) {
            if (par[r] != -1) continue;
            stack.push_back((int32_t)r);
            while (!stack.empty()) {
                int32_t t = stack.back();
                if (chead[t] >= 0) { int32_t c = chead[t]; chead[t] = cnext[c]; stack.push_back(c); }
                else { stack.pop_back(); post.push_back(t); }
            }
        }
        std::vector<int32_t> perm2(nA);
        for (int64_t k = 0; k < nA; ++k) perm2[k] = perm[post[k]];
        perm.swap(perm2);
        for (int64_t k = 0; k < nA; ++k) iperm[perm[k]] = (int32_t)k;
        build_rows(iperm, rp, ci);
        etree(rp, ci, par);
    }
    S.perm = perm;
    S.iperm = iperm;

    // --- column structures by row subtrees ------------------------------------
    std::vector<std::vector<int32_t>> cs(nA);
    {
        std::vector<int64_t> mk(nA, -1);
        for (int64_t i = 0; i < n; ++i) {
            if (i < nA) mk[i] = i;
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
                int32_t j = ci[k];
                while (j != -1 && mk[j] != i) {
                    cs[j].push_back((int32_t)i);
                    mk[j] = i;
                    j = par[j];
                }
            }
        }
    }
    std::vector<int64_t> cc(nA);
    for (int64_t j = 0; j < nA; ++j) cc[j] = 1 + (int64_t)cs[j].size();

    // --- fundamental supernodes -----------------------------------------------
    std::vector<int32_t> sfirst;
    for (int64_t j = 0; j < nA; ++j)
        if (!(j > 0 && par[j - 1] == j && cc[j - 1] == cc[j] + 1)) sfirst.push_back((int32_t)j);
    int32_t nf = (int32_t)sfirst.size();
    sfirst.push_back((int32_t)nA);
    std::vector<int32_t> fcol2sn(nA);
    for (int32_t s = 0; s < nf; ++s)
        for (int32_t j = sfirst[s]; j < sfirst[s + 1]; ++j) fcol2sn[j] = s;

    // --- relaxed amalgamation along contiguous (last-child) chains -----------
    // a merged supernode keeps [first, last] columns, its row count and the
    // count of true nonzeros of its columns.
    std::vector<int32_t> mfirst(nf), mlast(nf), alive(nf, 1);
    std::vector<int64_t> mrows(nf), mtrue(nf);
    for (int32_t s = 0; s < nf; ++s) {
        mfirst[s] = sfirst[s];
        mlast[s] = sfirst[s + 1] - 1;
        mrows[s] = cc[sfirst[s]];
        int64_t t = 0;
        for (int32_t j = sfirst[s]; j <= mlast[s]; ++j) t += cc[j];
        mtrue[s] = t;
    }
    // owner of each fundamental supernode after merges (union-find style)
    std::vector<int32_t> owner(nf);
    std::iota(owner.begin(), owner.end(), 0);
    std::vector<int32_t> by_last(nA + 1, -1);  // merged supernode ending at column j
    for (int32_t s = 0; s < nf; ++s) by_last[mlast[s]] = s;
    for (int32_t p = 0; p < nf; ++p) {
        while (true) {
            int32_t f = mfirst[p];
            if (f == 0) break;
            int32_t c = by_last[f - 1];
            if (c < 0 || !alive[c]) break;
            // contiguous child? its last column's parent must lie in p
            int32_t pj = par[mlast[c]];
            if (pj < mfirst[p] || pj > mlast[p]) break;
            int64_t ncc = mlast[c] - mfirst[c] + 1, ncp = mlast[p] - mfirst[p] + 1;
            int64_t nc = ncc + ncp, m = ncc + mrows[p];
            int64_t tot = nc * m - nc * (nc - 1) / 2;
            int64_t tru = mtrue[c] + mtrue[p];
            double z = tot > 0 ? double(tot - tru) / double(tot) : 0.0;
            bool ok = nc <= 4 || (nc <= 16 && z <= 0.8) || (nc <= 48 && z <= 0.1) || z <= 0.05;
            if (!ok) break;
            alive[c] = 0;
            by_last[mlast[c]] = -1;
            mfirst[p] = mfirst[c];
            mrows[p] = m;
            mtrue[p] = tru;
            owner[c] = p;
        }
    }
    // final supernodes in column order
    std::vector<int32_t> col2sn(nA);
    std::vector<int32_t> fs_first, fs_last;
    for (int32_t s = 0; s < nf; ++s)
        if (alive[s]) { fs_first.push_back(mfirst[s]); fs_last.push_back(mlast[s]); }
    std::vector<int32_t> idx(fs_first.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return fs_first[a] < fs_first[b]; });
    int32_t ns = (int32_t)idx.size();
    S.border_sn = nb > 0 ? ns : -1;
    int32_t nsup = ns + (nb > 0 ? 1 : 0);
    S.nsup = nsup;
    S.first.resize(nsup);
    S.ncol.resize(nsup);
    S.nrow.resize(nsup);
    for (int32_t t = 0; t < ns; ++t) {
        S.first[t] = fs_first[idx[t]];
        S.ncol[t] = fs_last[idx[t]] - fs_first[idx[t]] + 1;
        for (int32_t j = S.first[t]; j < S.first[t] + S.ncol[t]; ++j) col2sn[j] = t;
    }
    S.col2sn = col2sn;
    // rows of every supernode: union of its columns' structures
    S.rowptr.assign(nsup + 1, 0);
    {
        std::vector<int64_t> mk(n, -1);
        std::vector<int32_t> tmp;
        std::vector<std::vector<int32_t>> R(nsup);
        for (int32_t t = 0; t < ns; ++t) {
            tmp.clear();
            for (int32_t j = S.first[t]; j < S.first[t] + S.ncol[t]; ++j) {
                if (mk[j] != t) { mk[j] = t; tmp.push_back(j); }
                for (int32_t i : cs[j])
                    if (mk[i] != t) { mk[i] = t; tmp.push_back(i); }
            }
            std::sort(tmp.begin(), tmp.end());
            R[t] = tmp;
            std::vector<int32_t>().swap(cs[S.first[t]]);
        }
        if (nb > 0) {
            S.first[ns] = (int32_t)nA;
            S.ncol[ns] = 0;
            for (int64_t r = 0; r < nb; ++r) R[ns].push_back((int32_t)(nA + r));
        }
        for (int32_t t = 0; t < nsup; ++t) {
            S.nrow[t] = (int32_t)R[t].size();
            S.rowptr[t + 1] = S.rowptr[t] + S.nrow[t];
        }
        S.rows.resize(S.rowptr[nsup]);
        for (int32_t t = 0; t < nsup; ++t) std::copy(R[t].begin(), R[t].end(), S.rows.begin() + S.rowptr[t]);
    }
    // supernodal parent
    S.parent.assign(nsup, -1);
    for (int32_t t = 0; t < ns; ++t) {
        int32_t last = S.first[t] + S.ncol[t] - 1;
        if (par[last] >= 0) S.parent[t] = col2sn[par[last]];
        else if (nb > 0 && S.nrow[t] > S.ncol[t]) S.parent[t] = ns;
        else if (S.nrow[t] > S.ncol[t]) return "internal: root with update rows and no border";
    }
    // children
    S.child_ptr.assign(nsup + 1, 0);
    for (int32_t t = 0; t < nsup; ++t)
        if (S.parent[t] >= 0) S.child_ptr[S.parent[t] + 1]++;
    for (int32_t t = 0; t < nsup; ++t) S.child_ptr[t + 1] += S.child_ptr[t];
    S.child_list.resize(S.child_ptr[nsup]);
    {
        std::vector<int32_t> q(S.child_ptr.begin(), S.child_ptr.end() - 1);
        for (int32_t t = 0; t < nsup; ++t)
            if (S.parent[t] >= 0) S.child_list[q[S.parent[t]]++] = t;
    }
    // relative indices of update rows in the parent
    S.relptr.assign(nsup + 1, 0);
    for (int32_t t = 0; t < nsup; ++t) S.relptr[t + 1] = S.relptr[t] + (S.nrow[t] - S.ncol[t]);
    S.rel.assign(S.relptr[nsup], 0);
    for (int32_t t = 0; t < nsup; ++t) {
        int32_t p = S.parent[t];
        if (p < 0) continue;
        const int32_t *rc = &S.rows[S.rowptr[t]];
        const int32_t *rpnt = &S.rows[S.rowptr[p]];
        int32_t mp = S.nrow[p], k = 0;
        for (int32_t i = S.ncol[t]; i < S.nrow[t]; ++i) {
            while (k < mp && rpnt[k] < rc[i]) ++k;
            if (k >= mp || rpnt[k] != rc[i]) return "internal: update row missing in parent";
            S.rel[S.relptr[t] + (i - S.ncol[t])] = k;
        }
    }
    // levels (height); children precede parents in index order
    S.level.assign(nsup, 0);
    for (int32_t t = 0; t < nsup; ++t)
        if (S.parent[t] >= 0) {
            if (S.parent[t] <= t) return "internal: parent precedes child";
            S.level[S.parent[t]] = std::max(S.level[S.parent[t]], S.level[t] + 1);
        }
    S.nlevels = 0;
    for (int32_t t = 0; t < nsup; ++t) S.nlevels = std::max(S.nlevels, S.level[t] + 1);
    S.level_ptr.assign(S.nlevels + 1, 0);
    for (int32_t t = 0; t < nsup; ++t) S.level_ptr[S.level[t] + 1]++;
    for (int32_t l = 0; l < S.nlevels; ++l) S.level_ptr[l + 1] += S.level_ptr[l];
    S.level_list.resize(nsup);
    {
        std::vector<int32_t> q(S.level_ptr.begin(), S.level_ptr.end() - 1);
        for (int32_t t = 0; t < nsup; ++t) S.level_list[q[S.level[t]]++] = t;
    }
    // storage
    S.Loff.assign(nsup, 0);
    S.Uoff.assign(nsup, 0);
    int64_t L = 0, U = 0;
    double fl = 0.0;
    for (int32_t t = 0; t < nsup; ++t) {
        int64_t m = S.nrow[t], c = S.ncol[t], u = m - c;
        S.Loff[t] = L;
        S.Uoff[t] = U;
        L += m * c;
        U += u * u;
        for (int64_t k = 0; k < c; ++k) { double r = double(m - k - 1); fl += r * r + 2.0 * r; }
        S.max_front = std::max<int64_t>(S.max_front, m);
        S.max_pivots = std::max<int64_t>(S.max_pivots, c);
    }
    S.Lsize = L;
    S.Usize = U;
    S.nnzL = L;
    S.flops = fl;
    // scatter maps
    auto locate = [&](int32_t r, int32_t c) -> int64_t {
        int32_t t = col2sn[c];
        const int32_t *R = &S.rows[S.rowptr[t]];
        const int32_t *f = std::lower_bound(R, R + S.nrow[t], r);
        if (f == R + S.nrow[t] || *f != r) return -1;
        return S.Loff[t] + (int64_t)(c - S.first[t]) * S.nrow[t] + (f - R);
    };
    S.amap.resize(S.nnzA);
    S.adiag.resize(S.nnzA);
    for (int64_t j = 0; j < nA; ++j)
        for (int64_t k = in.colptr[j]; k < in.colptr[j + 1]; ++k) {
            int32_t a = iperm[in.rowind[k]], b = iperm[j];
            int64_t off = locate(std::max(a, b), std::min(a, b));
            if (off < 0) return "internal: A entry outside the factor pattern";
            S.amap[k] = off;
            S.adiag[k] = (in.rowind[k] == j) ? (j < in.n_primal ? 1 : -1) : 0;
        }
    S.c0map.resize(S.nnzC0);
    S.c1map.resize(S.nnzC1);
    for (int64_t s = 0; s < Ns; ++s) {
        for (int64_t k = in.C1p[s]; k < in.C1p[s + 1]; ++k) {
            int64_t off = locate((int32_t)(nA + s), iperm[in.C1i[k]]);
            if (off < 0) return "internal: C1 entry outside the factor pattern";
            S.c1map[k] = off;
        }
        for (int64_t k = in.C0p[s]; k < in.C0p[s + 1]; ++k) {
            int64_t off = locate((int32_t)(nA + Ns + s), iperm[in.C0i[k]]);
            if (off < 0) return "internal: C0 entry outside the factor pattern";
            S.c0map[k] = off;
        }
    }
    S.pivsign.resize(nA);
    for (int64_t k = 0; k < nA; ++k) S.pivsign[k] = perm[k] < in.n_primal ? 1 : -1;
    return "";
}

}  // namespace kkt
