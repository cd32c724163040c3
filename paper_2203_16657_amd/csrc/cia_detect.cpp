// P1 on graphs that come without labels: communities chosen to minimise the
// work of one CIA right-hand side.  Sec. 3.1 obtains the communities from a
// community-detection method; here the objective is the method's own cost.
// For a partition whose kept communities c have lambda_c members and e_c
// inner (undirected) edges, one RHS gathers
//
//   nnz(S-neg) + nnz(S-pos) + alpha * (members of kept communities)
//     = 2|E| + sum_c [ lambda_c (lambda_c - 1 + alpha) - 4 e_c ],
//
// (missing intra pairs, edges leaving communities, E1 per member; alpha is
// the dense_alpha of P1's cost rule), so the detection minimises
// Q = sum_c q_c, q_c = lambda_c (lambda_c - 1 + alpha) - 4 e_c.  Moving a node
// of size s (an aggregate of s original nodes) from community A to B changes
// Q by 2 s (lambda_B - lambda_A + s) - 4 (k_B - k_A), k_X the edges from the
// node to the other members of X (alpha and the node's own inner edges
// cancel).  Louvain-style: local moving over the nodes in index order until
// no move lowers Q, then aggregation of communities into nodes, repeated;
// finally communities with q_c >= 0 (P1's cost rule) or a single member are
// dissolved into -1.  Every step is sequential and in a fixed order, so the
// result is deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

namespace cia {

namespace {

struct Level {
    int64_t n = 0;
    // adjacency without self entries; w empty = unit weights (the input graph)
    const int64_t *rp = nullptr;
    const int32_t *col = nullptr;
    const int64_t *w = nullptr;
    std::vector<int64_t> rp_s, w_s;
    std::vector<int32_t> col_s;
    std::vector<int64_t> size;   // original nodes per node
};

// One round of local moving passes; returns whether any node moved.
bool local_moving(const Level &G, std::vector<int32_t> &comm, std::vector<int64_t> &csize, int max_passes) {
    const int64_t n = G.n;
    std::vector<int64_t> kin(n, 0);
    std::vector<int32_t> touched;
    std::vector<int32_t> empty;
    for (int64_t c = n - 1; c >= 0; c--)
        if (csize[c] == 0) empty.push_back((int32_t)c);
    bool any = false;
    for (int pass = 0; pass < max_passes; pass++) {
        bool moved = false;
        for (int64_t i = 0; i < n; i++) {
            const int32_t A = comm[i];
            const int64_t s = G.size[i];
            touched.clear();
            for (int64_t e = G.rp[i]; e < G.rp[i + 1]; e++) {
                const int32_t c = comm[G.col[e]];
                if (kin[c] == 0) touched.push_back(c);
                kin[c] += G.w ? G.w[e] : 1;
            }
            const int64_t kA = kin[A], lamA = csize[A];
            int32_t best = A;
            int64_t bestd = 0;
            for (int32_t B : touched) {
                if (B == A) continue;
                const int64_t d = 2 * s * (csize[B] - lamA + s) - 4 * (kin[B] - kA);
                if (d < bestd || (d == bestd && d < 0 && B < best)) {
                    bestd = d;
                    best = B;
                }
            }
            if (lamA > s && !empty.empty()) {
                const int64_t d = 2 * s * (s - lamA) + 4 * kA;   // into an empty community
                if (d < bestd) {
                    bestd = d;
                    best = empty.back();
                }
            }
            for (int32_t c : touched) kin[c] = 0;
            if (best != A) {
                if (!empty.empty() && best == empty.back()) empty.pop_back();
                csize[A] -= s;
                csize[best] += s;
                comm[i] = best;
                if (csize[A] == 0) empty.push_back(A);
                moved = true;
            }
        }
        any |= moved;
        if (!moved) break;
    }
    return any;
}

// Communities of G as the nodes of the next level (numbered by first member).
void aggregate(const Level &G, const std::vector<int32_t> &comm, std::vector<int32_t> &renum, Level &H) {
    const int64_t n = G.n;
    renum.assign(n, -1);
    int32_t m = 0;
    for (int64_t i = 0; i < n; i++)
        if (renum[comm[i]] < 0) renum[comm[i]] = m++;
    H.n = m;
    H.size.assign(m, 0);
    std::vector<std::vector<int64_t>> members(m);
    for (int64_t i = 0; i < n; i++) {
        H.size[renum[comm[i]]] += G.size[i];
        members[renum[comm[i]]].push_back(i);
    }
    H.rp_s.assign(m + 1, 0);
    H.col_s.clear();
    H.w_s.clear();
    std::vector<int64_t> acc(m, 0);
    std::vector<int32_t> nb;
    for (int32_t c = 0; c < m; c++) {
        nb.clear();
        for (int64_t i : members[c])
            for (int64_t e = G.rp[i]; e < G.rp[i + 1]; e++) {
                const int32_t d = renum[comm[G.col[e]]];
                if (d == c) continue;
                if (acc[d] == 0) nb.push_back(d);
                acc[d] += G.w ? G.w[e] : 1;
            }
        std::sort(nb.begin(), nb.end());
        for (int32_t d : nb) {
            H.col_s.push_back(d);
            H.w_s.push_back(acc[d]);
            acc[d] = 0;
        }
        H.rp_s[c + 1] = (int64_t)H.col_s.size();
    }
    H.rp = H.rp_s.data();
    H.col = H.col_s.data();
    H.w = H.w_s.data();
}

}  // namespace

cia_status detect_communities(const cia_graph *g, const int32_t *init, double alpha, int32_t *labels, double *work) {
    if (!g || !labels) return set_error(CIA_EINVAL, "NULL pointer");
    if (g->kind != CIA_GRAPH_CSR) return set_error(CIA_EUNSUPPORTED, "community detection needs a CSR graph");
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return set_error(CIA_EINVAL, "dense_alpha must be finite and >= 0");
    {
        // validation of the graph (symmetry, sorted rows, no self loops)
        P1 chk;
        CIA_TRY(p1_build(g, nullptr, alpha, true, true, false, chk));
    }
    const int64_t n = g->n;
    if (n > INT32_MAX) return set_error(CIA_EUNSUPPORTED, "n too large");
    Level L0;
    L0.n = n;
    L0.rp = g->row_ptr;
    L0.col = g->col;
    L0.size.assign(n, 1);
    // start: the given labels (refinement) or singletons
    std::vector<int32_t> comm(n);
    std::vector<int64_t> csize(n, 0);
    if (init) {
        std::vector<int32_t> lab2c;
        int32_t maxl = -1;
        for (int64_t i = 0; i < n; i++) {
            if (init[i] < -1) return set_error(CIA_EINVAL, "init label %d < -1", init[i]);
            maxl = std::max(maxl, init[i]);
        }
        lab2c.assign((size_t)maxl + 1, -1);
        for (int64_t i = 0; i < n; i++) {
            if (init[i] < 0) {
                comm[i] = (int32_t)i;
            } else {
                if (lab2c[init[i]] < 0) lab2c[init[i]] = (int32_t)i;
                comm[i] = lab2c[init[i]];
            }
        }
    } else {
        for (int64_t i = 0; i < n; i++) comm[i] = (int32_t)i;
    }
    for (int64_t i = 0; i < n; i++) csize[comm[i]] += 1;

    // node of the current level of every original node
    std::vector<int32_t> top(n);
    for (int64_t i = 0; i < n; i++) top[i] = (int32_t)i;
    std::vector<Level> levels;
    levels.reserve(64);
    const Level *G = &L0;
    for (int lev = 0; lev < 64; lev++) {
        const bool moved = local_moving(*G, comm, csize, 64);
        if (!moved && lev > 0) break;
        std::vector<int32_t> renum;
        levels.emplace_back();
        Level &H = levels.back();
        aggregate(*G, comm, renum, H);
        for (int64_t i = 0; i < n; i++) top[i] = renum[comm[top[i]]];
        const bool shrank = H.n < G->n;
        G = &H;
        comm.assign(G->n, 0);
        csize.assign(G->n, 0);
        for (int64_t c = 0; c < G->n; c++) {
            comm[c] = (int32_t)c;
            csize[c] = G->size[c];
        }
        if (!shrank) break;
    }

    // communities of the top level: sizes, inner edges, the cost rule
    const int64_t m = G->n;
    std::vector<int64_t> lam(m, 0), inner2(m, 0);
    for (int64_t i = 0; i < n; i++) lam[top[i]]++;
    int64_t nnz = g->row_ptr[n];
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; e++)
            if (top[g->col[e]] == top[i]) inner2[top[i]]++;   // each inner edge twice
    std::vector<int32_t> keep(m, -1);
    int32_t k = 0;
    double neg = 0.0, pos = (double)nnz, e1 = 0.0;
    for (int64_t i = 0; i < n; i++) {
        const int32_t c = top[i];
        if (keep[c] != -1) continue;
        const double l = (double)lam[c], e = (double)inner2[c] / 2.0;
        const double q = l * (l - 1.0 + alpha) - 4.0 * e;
        if (lam[c] >= 2 && q < 0.0) {
            keep[c] = k++;
            neg += l * (l - 1.0) - 2.0 * e;
            pos -= 2.0 * e;
            e1 += alpha * l;
        } else {
            keep[c] = -2;   // dissolved
        }
    }
    for (int64_t i = 0; i < n; i++) labels[i] = keep[top[i]] >= 0 ? keep[top[i]] : -1;
    if (work) *work = neg + pos + e1;
    return CIA_OK;
}

}  // namespace cia

extern "C" cia_status cia_detect_communities(const cia_graph *g, const int32_t *init_labels, double dense_alpha,
                                             int32_t *labels, double *work) {
    cia::clear_error();
    try {
        return cia::detect_communities(g, init_labels, dense_alpha, labels, work);
    } catch (const std::bad_alloc &) {
        return cia::set_error(CIA_ENOMEM, "host allocation failed");
    }
}
