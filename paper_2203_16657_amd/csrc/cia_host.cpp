// Host-side pre-simulation: step P1 (community permutation and the sparse
// remainder S, Sec. 3.1 and App. A.1) and step P2 for sampled couplings
// (real Fourier coefficients, Sec. 3.1 / App. A.2), plus error reporting.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <unordered_map>

#include "internal.h"

namespace cia {

static thread_local std::string g_last_error;

cia_status set_error(cia_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

void clear_error() { g_last_error.clear(); }

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Structural checks of a CSR adjacency: monotone row pointers, columns in
// range, rows strictly increasing (no duplicates), no self-loops, symmetric.
// Symmetry is checked by comparing order-independent hash sums of all
// (u,v) and all (v,u) pairs (two independent 64-bit mixes).
static cia_status validate_csr(int64_t n, const int64_t *rp, const int32_t *col) {
    if (rp[0] != 0) return set_error(CIA_EINVAL, "graph: row_ptr[0] = %lld, expected 0", (long long)rp[0]);
    for (int64_t u = 0; u < n; u++)
        if (rp[u + 1] < rp[u])
            return set_error(CIA_EINVAL, "graph: row_ptr decreases at row %lld", (long long)u);
    int64_t bad_row = -1;
    int bad_kind = 0;
    uint64_t h1 = 0, h2 = 0, g1 = 0, g2 = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : h1, h2, g1, g2)
    for (int64_t u = 0; u < n; u++) {
        int32_t prev = -1;
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
            int32_t v = col[e];
            int kind = 0;
            if (v < 0 || v >= n) kind = 1;
            else if (v == u) kind = 2;
            else if (v <= prev) kind = 3;
            if (kind) {
#pragma omp critical
                {
                    if (bad_row < 0 || u < bad_row) { bad_row = u; bad_kind = kind; }
                }
                break;
            }
            prev = v;
            uint64_t a = ((uint64_t)u << 32) | (uint32_t)v, b = ((uint64_t)v << 32) | (uint32_t)u;
            h1 += mix64(a);
            h2 += mix64(b);
            g1 += mix64(a ^ 0x5555555555555555ULL);
            g2 += mix64(b ^ 0x5555555555555555ULL);
        }
    }
    if (bad_row >= 0) {
        const char *what = bad_kind == 1 ? "column out of range"
                           : bad_kind == 2 ? "self-loop"
                                           : "row not strictly increasing (unsorted or duplicate)";
        return set_error(CIA_EINVAL, "graph: %s in row %lld", what, (long long)bad_row);
    }
    if (h1 != h2 || g1 != g2) return set_error(CIA_EINVAL, "graph: adjacency is not symmetric");
    return CIA_OK;
}

cia_status p1_build(const cia_graph *g, const int32_t *labels, double dense_alpha,
                    bool keep_labels, bool validate, bool with_s, P1 &out) {
    if (!g) return set_error(CIA_EINVAL, "graph is NULL");
    const int64_t n = g->n;
    if (n <= 0) return set_error(CIA_EINVAL, "graph: n = %lld, need n >= 1", (long long)n);
    if (n > 0x7fffffffLL) return set_error(CIA_EUNSUPPORTED, "graph: n above 2^31 - 1");
    const bool complete = g->kind == CIA_GRAPH_COMPLETE;
    if (!complete && g->kind != CIA_GRAPH_CSR)
        return set_error(CIA_EINVAL, "graph: unknown kind %d", g->kind);
    if (!complete && (!g->row_ptr || (!g->col && g->row_ptr[n] > 0)))
        return set_error(CIA_EINVAL, "graph: CSR arrays are NULL");
    const int64_t *rp = g->row_ptr;
    const int32_t *col = g->col;
    if (!complete && validate) CIA_TRY(validate_csr(n, rp, col));

    out = P1();
    out.n = n;
    out.complete = complete;
    out.nnz_graph = complete ? n * (n - 1) : rp[n];

    // ---- labels -> dense ids (sorted unique), -1 = no community ----
    std::vector<int32_t> lab(n, 0);
    int32_t nlab = 1;
    if (labels) {
        std::vector<int32_t> uniq;
        for (int64_t u = 0; u < n; u++) {
            if (labels[u] < -1)
                return set_error(CIA_EINVAL, "labels[%lld] = %d; labels must be >= -1", (long long)u,
                                 labels[u]);
            if (labels[u] >= 0) uniq.push_back(labels[u]);
        }
        std::sort(uniq.begin(), uniq.end());
        uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
        nlab = (int32_t)uniq.size();
#pragma omp parallel for schedule(static)
        for (int64_t u = 0; u < n; u++)
            lab[u] = labels[u] < 0 ? -1
                                   : (int32_t)(std::lower_bound(uniq.begin(), uniq.end(), labels[u]) -
                                               uniq.begin());
    }
    if (complete && nlab > 1)
        return set_error(CIA_EUNSUPPORTED, "complete graph: only a single community is supported");
    if (complete)
        for (int64_t u = 0; u < n; u++)
            if (lab[u] < 0)
                return set_error(CIA_EUNSUPPORTED, "complete graph: every node must be in the community");

    // ---- community sizes and intra-entry counts; cost rule (App. A.1) ----
    std::vector<int64_t> size(nlab, 0), intra(nlab, 0);
    for (int64_t u = 0; u < n; u++)
        if (lab[u] >= 0) size[lab[u]]++;
    if (complete) {
        intra[0] = n * (n - 1);
    } else {
        std::vector<int64_t> intra_row(n, 0);
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t u = 0; u < n; u++) {
            int32_t c = lab[u];
            if (c < 0) continue;
            int64_t k = 0;
            for (int64_t e = rp[u]; e < rp[u + 1]; e++) k += lab[col[e]] == c;
            intra_row[u] = k;
        }
        for (int64_t u = 0; u < n; u++)
            if (lab[u] >= 0) intra[lab[u]] += intra_row[u];
    }
    std::vector<int32_t> dense_id(nlab, -1);
    int32_t ncomm = 0;
    for (int32_t c = 0; c < nlab; c++) {
        int64_t lam = size[c];
        if (lam == 0) continue;
        int64_t neg = lam * (lam - 1) - intra[c];
        bool keep = keep_labels || ((double)neg + dense_alpha * (double)lam < (double)intra[c]);
        if (keep) dense_id[c] = ncomm++;
    }
    out.ncomm = ncomm;

    // ---- permutation: communities contiguous (increasing user id inside),
    //      nodes of no community last ----
    out.comm_off.assign(ncomm + 1, 0);
    std::vector<int32_t> dl(n);
    for (int64_t u = 0; u < n; u++) {
        int32_t d = lab[u] >= 0 ? dense_id[lab[u]] : -1;
        dl[u] = d;
        if (d >= 0) out.comm_off[d + 1]++;
    }
    for (int32_t c = 0; c < ncomm; c++) out.comm_off[c + 1] += out.comm_off[c];
    for (int32_t c = 0; c < ncomm; c++)
        if (out.comm_off[c + 1] - out.comm_off[c] > 0x7fffffff)
            return set_error(CIA_EUNSUPPORTED, "community too large");
    out.perm.resize(n);
    out.inv.resize(n);
    out.comm_of_pos.resize(n);
    {
        std::vector<int64_t> fill(out.comm_off.begin(), out.comm_off.end());
        int64_t tail = out.comm_off[ncomm];
        for (int64_t u = 0; u < n; u++) {
            int32_t d = dl[u];
            int64_t pos = d >= 0 ? fill[d]++ : tail++;
            out.perm[pos] = (int32_t)u;
            out.inv[u] = (int32_t)pos;
            out.comm_of_pos[pos] = d;
        }
    }
    if (!with_s) return CIA_OK;

    // ---- S: S-neg (missing intra partners) and S-pos (everything else) ----
    out.negptr.assign(n + 1, 0);
    out.posptr.assign(n + 1, 0);
    if (complete) {
        // one dense community, no remainder; the diagonal is handled analytically
        out.neg_local.clear();
        out.pos.clear();
        return CIA_OK;
    }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; i++) {
        int32_t u = out.perm[i];
        int32_t c = out.comm_of_pos[i];
        int64_t deg = rp[u + 1] - rp[u];
        if (c < 0) {
            out.posptr[i + 1] = deg;
            continue;
        }
        int64_t k = 0;
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) k += dl[col[e]] == c;
        int64_t lam = out.comm_off[c + 1] - out.comm_off[c];
        out.negptr[i + 1] = lam - 1 - k;
        out.posptr[i + 1] = deg - k;
    }
    for (int64_t i = 0; i < n; i++) {
        out.negptr[i + 1] += out.negptr[i];
        out.posptr[i + 1] += out.posptr[i];
    }
    out.neg_local.resize(out.negptr[n]);
    out.pos.resize(out.posptr[n]);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; i++) {
        int32_t u = out.perm[i];
        int32_t c = out.comm_of_pos[i];
        int32_t *pw = out.pos.data() + out.posptr[i];
        int32_t *pb = pw;
        if (c < 0) {
            for (int64_t e = rp[u]; e < rp[u + 1]; e++) *pw++ = out.inv[col[e]];
        } else {
            const int32_t off = out.comm_off[c];
            const int32_t lam = out.comm_off[c + 1] - off;
            const int32_t self = (int32_t)i - off;
            int32_t *nw = out.neg_local.data() + out.negptr[i];
            // intra partners arrive in increasing local order (positions inside a
            // community follow user ids); walk the community range once and emit
            // every local index that is neither self nor a partner
            int32_t next = 0;  // next local index not yet accounted for
            for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
                int32_t v = col[e];
                if (dl[v] != c) {
                    *pw++ = out.inv[v];
                    continue;
                }
                int32_t loc = out.inv[v] - off;
                for (; next < loc; next++)
                    if (next != self) *nw++ = next;
                next = loc + 1;
            }
            for (; next < lam; next++)
                if (next != self) *nw++ = next;
        }
        std::sort(pb, pw);
    }
    return CIA_OK;
}

cia_status p1_permuted_adjacency(const cia_graph *g, const P1 &p1, std::vector<int64_t> &rp,
                                 std::vector<int32_t> &col) {
    const int64_t n = p1.n;
    const int64_t *grp = g->row_ptr;
    const int32_t *gcol = g->col;
    try {
        rp.assign(n + 1, 0);
        for (int64_t i = 0; i < n; i++) {
            int32_t u = p1.perm[i];
            rp[i + 1] = rp[i] + (grp[u + 1] - grp[u]);
        }
        col.resize(rp[n]);
    } catch (const std::bad_alloc &) {
        return set_error(CIA_ENOMEM, "host allocation of the permuted adjacency failed");
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; i++) {
        int32_t u = p1.perm[i];
        int32_t *w = col.data() + rp[i];
        int64_t d = grp[u + 1] - grp[u];
        for (int64_t e = 0; e < d; e++) w[e] = p1.inv[gcol[grp[u] + e]];
        // positions inside one community follow user order, so the row is a
        // few increasing runs; a sort keeps the general case simple
        if (!std::is_sorted(w, w + d)) std::sort(w, w + d);
    }
    return CIA_OK;
}

}  // namespace cia

using namespace cia;

extern "C" {

const char *cia_last_error(void) { return cia::g_last_error.c_str(); }

void cia_options_default(cia_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->method = CIA_METHOD_CIA;
    o->precision = CIA_F32;
    o->stepper = CIA_RK4;
    o->flags = 0;
    o->dense_alpha = 2.0;
    o->unit_work = 0;
    o->block = 0;
    o->judge_tol = 1e-3;
    o->device = -1;
}

void cia_coupling_default(cia_coupling *c) {
    if (!c) return;
    static const double ds[2] = {0.0, 1.0}, dc[2] = {0.0, 0.0};
    std::memset(c, 0, sizeof(*c));
    c->model = CIA_MODEL_PHASE;
    c->p = 1;
    c->d_sin = ds;
    c->d_cos = dc;
    c->K = 1.0;
    c->cs_K = 1.0;
    c->cs_sigma = 1.0;
    c->cs_beta = 0.25;
    c->cs_L = 20.0;
    c->cs_basis = CIA_BASIS_EXACT;
    c->rank = 32;
    c->poly_q = -1;
}

cia_status cia_fourier_coeffs(const double *samples, int64_t m, int32_t p, double *d_sin,
                              double *d_cos) {
    clear_error();
    if (!samples || !d_sin || !d_cos) return set_error(CIA_EINVAL, "NULL pointer");
    if (p < 0 || m < 2 * (int64_t)p + 1)
        return set_error(CIA_EINVAL, "need m >= 2p+1 samples (m = %lld, p = %d)", (long long)m, p);
    // trapezoidal rule on the periodic grid = discrete Fourier transform
    for (int32_t k = 0; k <= p; k++) {
        double sc = 0.0, ss = 0.0;
        for (int64_t j = 0; j < m; j++) {
            double x = 2.0 * M_PI * (double)j / (double)m;
            sc += samples[j] * std::cos(k * x);
            ss += samples[j] * std::sin(k * x);
        }
        double w = (k == 0 || 2 * (int64_t)k == m) ? 1.0 / (double)m : 2.0 / (double)m;
        d_cos[k] = w * sc;
        d_sin[k] = k == 0 ? 0.0 : w * ss;
    }
    return CIA_OK;
}

cia_status cia_p1_build(const cia_graph *g, const int32_t *labels, const cia_options *o,
                        cia_p1 **out) {
    clear_error();
    if (!out) return set_error(CIA_EINVAL, "out is NULL");
    *out = nullptr;
    cia_options def;
    cia_options_default(&def);
    if (!o) o = &def;
    cia_p1 *h = new (std::nothrow) cia_p1();
    if (!h) return set_error(CIA_ENOMEM, "host allocation failed");
    cia_status st;
    try {
        st = p1_build(g, labels, o->dense_alpha, (o->flags & CIA_FLAG_KEEP_LABELS) != 0,
                      (o->flags & CIA_FLAG_NO_VALIDATE) == 0, true, h->p1);
    } catch (const std::bad_alloc &) {
        st = set_error(CIA_ENOMEM, "host allocation failed");
    }
    if (st != CIA_OK) {
        delete h;
        return st;
    }
    *out = h;
    return CIA_OK;
}

cia_status cia_p1_sizes(const cia_p1 *h, int64_t sizes[6]) {
    if (!h || !sizes) return set_error(CIA_EINVAL, "NULL pointer");
    const P1 &p = h->p1;
    sizes[0] = p.n;
    sizes[1] = p.ncomm;
    sizes[2] = (int64_t)p.neg_local.size();
    sizes[3] = (int64_t)p.pos.size();
    sizes[4] = p.n - (p.ncomm ? p.comm_off[p.ncomm] : 0);
    sizes[5] = p.nnz_graph;
    return CIA_OK;
}

cia_status cia_p1_export(const cia_p1 *h, int32_t *perm, int32_t *comm_off, int64_t *negptr,
                         int32_t *neg, int64_t *posptr, int32_t *pos) {
    if (!h) return set_error(CIA_EINVAL, "NULL handle");
    const P1 &p = h->p1;
    if (perm) std::memcpy(perm, p.perm.data(), sizeof(int32_t) * p.n);
    if (comm_off) std::memcpy(comm_off, p.comm_off.data(), sizeof(int32_t) * (p.ncomm + 1));
    if (negptr && !p.negptr.empty()) std::memcpy(negptr, p.negptr.data(), sizeof(int64_t) * (p.n + 1));
    if (posptr && !p.posptr.empty()) std::memcpy(posptr, p.posptr.data(), sizeof(int64_t) * (p.n + 1));
    if (neg) {
        for (int64_t i = 0; i < p.n; i++) {
            int32_t c = p.comm_of_pos[i];
            for (int64_t e = p.negptr[i]; e < p.negptr[i + 1]; e++) neg[e] = p.neg_local[e] + p.comm_off[c];
        }
    }
    if (pos && !p.pos.empty()) std::memcpy(pos, p.pos.data(), sizeof(int32_t) * p.pos.size());
    return CIA_OK;
}

cia_status cia_p1_free(cia_p1 *h) {
    delete h;
    return CIA_OK;
}

size_t cia_abi_sizeof(const char *name) {
    if (!name) return 0;
    if (!std::strcmp(name, "cia_graph")) return sizeof(cia_graph);
    if (!std::strcmp(name, "cia_hypergraph")) return sizeof(cia_hypergraph);
    if (!std::strcmp(name, "cia_coupling")) return sizeof(cia_coupling);
    if (!std::strcmp(name, "cia_options")) return sizeof(cia_options);
    if (!std::strcmp(name, "cia_plan_info")) return sizeof(cia_plan_info);
    if (!std::strcmp(name, "cia_timing")) return sizeof(cia_timing);
    if (!std::strcmp(name, "cia_tune_report")) return sizeof(cia_tune_report);
    return 0;
}

}  // extern "C"
