// Batched ensembles: many phase-model networks integrated as one plan.
//
// The instances are joined into their disjoint union (instance b owns user
// ids [off_b, off_b + N_b) of the joined state).  Communities never span two
// instances, so P1 (permutation, cost rule, S-neg / S-pos) of the union is
// P1 of every instance, and one launch per RK stage covers the work units of
// every instance.  What differs per instance is the coupling scale K_b / N_b
// (eq. 2.1 with each instance's own N), carried per node, and the order
// parameter, reduced per instance.
//
// The union is built incrementally: each added instance runs P1 on its own
// graph and appends its community sizes, row lists and frequencies; the
// caller may free the instance's graph as soon as cia_batch_add returns, so
// host memory peaks at one instance's adjacency plus the remainder lists
// gathered so far.  cia_batch_finish lays out the union exactly as P1 of the
// joined graph would (communities of every instance in order, then every
// instance's nodes of no community) and builds the plan from it.
#include <cmath>
#include <cstring>
#include <new>

#include "plan.h"

namespace cia {

static cia_status batch_check_coupling(const BatchAcc &A, int32_t b, const cia_coupling *c) {
    if (!c) return set_error(CIA_EINVAL, "batch instance %d: coupling is NULL", b);
    if (c->model != CIA_MODEL_PHASE)
        return set_error(CIA_EUNSUPPORTED, "batch instance %d: only the phase model can be batched", b);
    if (c->p < 1 || c->p > 8) return set_error(CIA_EINVAL, "batch instance %d: coupling.p = %d; supported 1..8", b, c->p);
    if (!c->d_sin || !c->d_cos) return set_error(CIA_EINVAL, "batch instance %d: coupling.d_sin/d_cos are NULL", b);
    if (c->gen_c11 || c->gen_c12 || c->gen_c21 || c->gen_c22)
        return set_error(CIA_EUNSUPPORTED, "batch instance %d: general coupling: ensembles are not batched", b);
    if (A.p >= 0) {
        if (c->p != A.p) return set_error(CIA_EINVAL, "batch instance %d: every instance needs the same coupling function", b);
        for (int k = 0; k <= c->p; k++)
            if (c->d_sin[k] != A.dsin[k] || c->d_cos[k] != A.dcos[k])
                return set_error(CIA_EINVAL, "batch instance %d: every instance needs the same coupling function", b);
    }
    if (!std::isfinite(c->K)) return set_error(CIA_EINVAL, "batch instance %d: K is not finite", b);
    return CIA_OK;
}

cia_status batch_add(BatchAcc &A, const cia_graph *g, const int32_t *labels, const cia_coupling *c,
                     const double *omega) {
    const int32_t b = (int32_t)A.ncn.size();
    if (!g) return set_error(CIA_EINVAL, "batch instance %d: graph is NULL", b);
    if (g->kind != CIA_GRAPH_CSR)
        return set_error(CIA_EUNSUPPORTED, "batch instance %d: only CSR graphs can be batched", b);
    if (g->n <= 0) return set_error(CIA_EINVAL, "batch instance %d: n = %lld", b, (long long)g->n);
    if (!g->row_ptr || (g->row_ptr[g->n] > 0 && !g->col))
        return set_error(CIA_EINVAL, "batch instance %d: row_ptr/col is NULL", b);
    CIA_TRY(batch_check_coupling(A, b, c));
    const int64_t nb = g->n, o0 = A.off.back();
    if (o0 + nb > INT32_MAX)
        return set_error(CIA_EUNSUPPORTED, "batch: %lld nodes in total (limit 2^31-1)", (long long)(o0 + nb));
    if (omega)
        for (int64_t i = 0; i < nb; i++)
            if (!std::isfinite(omega[i]))
                return set_error(CIA_EINVAL, "batch instance %d: omega[%lld] is not finite", b, (long long)i);

    // P1 of this instance alone (NULL labels = one community)
    const bool direct = A.o.method == CIA_METHOD_DIRECT;
    const bool validate = (A.o.flags & CIA_FLAG_NO_VALIDATE) == 0;
    const bool keep = direct || (A.o.flags & CIA_FLAG_KEEP_LABELS) != 0;
    P1 q;
    cia_status st = p1_build(g, labels, A.o.dense_alpha, keep, validate, !direct, q);
    if (st != CIA_OK) {
        std::string msg = cia_last_error();
        return set_error(st, "batch instance %d: %s", b, msg.c_str());
    }
    std::vector<int64_t> arp;
    std::vector<int32_t> acol;
    if (direct) {
        CIA_TRY(p1_permuted_adjacency(g, q, arp, acol));
    } else {
        arp.swap(q.posptr);
        acol.swap(q.pos);
    }

    const int64_t ncn = q.ncomm ? q.comm_off[q.ncomm] : 0;
    if (A.p < 0) {
        A.p = c->p;
        A.dsin.assign(c->d_sin, c->d_sin + c->p + 1);
        A.dcos.assign(c->d_cos, c->d_cos + c->p + 1);
    }
    for (int32_t k = 0; k < q.ncomm; k++) A.comm_size.push_back(q.comm_off[k + 1] - q.comm_off[k]);
    for (int64_t i = 0; i < nb; i++) (i < ncn ? A.perm_c : A.perm_u).push_back((int32_t)(q.perm[i] + o0));
    for (int64_t i = 0; i < ncn; i++) {
        if (!direct) {
            A.neg.insert(A.neg.end(), q.neg_local.begin() + q.negptr[i], q.neg_local.begin() + q.negptr[i + 1]);
        }
        A.negptr_c.push_back((int64_t)A.neg.size());
        A.pos_c.insert(A.pos_c.end(), acol.begin() + arp[i], acol.begin() + arp[i + 1]);
        A.posptr_c.push_back((int64_t)A.pos_c.size());
    }
    for (int64_t i = ncn; i < nb; i++) {
        A.pos_u.insert(A.pos_u.end(), acol.begin() + arp[i], acol.begin() + arp[i + 1]);
        A.posptr_u.push_back((int64_t)A.pos_u.size());
    }
    const double knb = c->K / (double)nb;
    A.kn.insert(A.kn.end(), (size_t)nb, knb);
    if (omega && !A.any_omega) {
        A.any_omega = true;
        A.omega.assign((size_t)o0, 0.0);   // earlier instances: zero frequencies
    }
    if (A.any_omega) {
        if (omega) A.omega.insert(A.omega.end(), omega, omega + nb);
        else A.omega.insert(A.omega.end(), (size_t)nb, 0.0);
    }
    A.nnz_graph += g->row_ptr[nb];
    A.ncn.push_back(ncn);
    A.off.push_back(o0 + nb);
    return CIA_OK;
}

// The union's P1 in the layout p1_build gives the joined graph: communities
// in instance order, then the outside rows; partner positions mapped from
// instance positions to union positions (the map is increasing, so sorted
// rows stay sorted).
static cia_status batch_union(BatchAcc &A, P1 &u) {
    const int32_t count = (int32_t)A.ncn.size();
    const int64_t n = A.off.back();
    const int64_t U0 = (int64_t)A.perm_c.size();
    u = P1();
    u.n = n;
    u.nnz_graph = A.nnz_graph;
    u.complete = false;
    u.ncomm = (int32_t)A.comm_size.size();
    u.comm_off.assign(u.ncomm + 1, 0);
    for (int32_t k = 0; k < u.ncomm; k++) u.comm_off[k + 1] = u.comm_off[k] + A.comm_size[k];
    if ((int64_t)u.comm_off[u.ncomm] != U0) return set_error(CIA_EINVAL, "internal: batch community rows disagree");
    u.perm.resize(n);
    std::memcpy(u.perm.data(), A.perm_c.data(), sizeof(int32_t) * U0);
    std::memcpy(u.perm.data() + U0, A.perm_u.data(), sizeof(int32_t) * (n - U0));
    std::vector<int32_t>().swap(A.perm_c);
    std::vector<int32_t>().swap(A.perm_u);
    u.inv.resize(n);
    for (int64_t i = 0; i < n; i++) u.inv[u.perm[i]] = (int32_t)i;
    u.comm_of_pos.assign(n, -1);
    for (int32_t k = 0; k < u.ncomm; k++)
        for (int32_t i = u.comm_off[k]; i < u.comm_off[k + 1]; i++) u.comm_of_pos[i] = k;

    u.negptr.assign(n + 1, 0);
    for (int64_t i = 0; i < U0; i++) u.negptr[i + 1] = A.negptr_c[i + 1];
    for (int64_t i = U0; i < n; i++) u.negptr[i + 1] = u.negptr[i];
    u.neg_local.swap(A.neg);
    std::vector<int64_t>().swap(A.negptr_c);

    // instance position -> union position
    std::vector<int64_t> cbase(count), ubase(count);
    {
        int64_t cb = 0, ub = U0;
        for (int32_t b = 0; b < count; b++) {
            cbase[b] = cb;
            ubase[b] = ub;
            cb += A.ncn[b];
            ub += (A.off[b + 1] - A.off[b]) - A.ncn[b];
        }
    }
    const int64_t npc = (int64_t)A.pos_c.size(), npu = (int64_t)A.pos_u.size();
    u.posptr.assign(n + 1, 0);
    for (int64_t i = 0; i < U0; i++) u.posptr[i + 1] = A.posptr_c[i + 1];
    for (int64_t i = U0; i < n; i++) u.posptr[i + 1] = npc + A.posptr_u[i - U0 + 1];
    std::vector<int64_t>().swap(A.posptr_c);
    std::vector<int64_t>().swap(A.posptr_u);
    u.pos.swap(A.pos_c);
    u.pos.resize(npc + npu);
    std::memcpy(u.pos.data() + npc, A.pos_u.data(), sizeof(int32_t) * npu);
    std::vector<int32_t>().swap(A.pos_u);
    // rows of instance b: community rows [cbase_b, cbase_b + ncn_b), outside
    // rows [ubase_b, ubase_b + N_b - ncn_b)
    for (int32_t b = 0; b < count; b++) {
        const int64_t nc = A.ncn[b], nb = A.off[b + 1] - A.off[b];
        const int64_t cb = cbase[b], ub = ubase[b];
        auto remap = [&](int64_t r0, int64_t r1) {
#pragma omp parallel for schedule(dynamic, 1024)
            for (int64_t i = r0; i < r1; i++)
                for (int64_t e = u.posptr[i]; e < u.posptr[i + 1]; e++) {
                    const int64_t p = u.pos[e];
                    u.pos[e] = (int32_t)(p < nc ? cb + p : ub + (p - nc));
                }
        };
        remap(cb, cb + nc);
        remap(ub, ub + (nb - nc));
    }
    return CIA_OK;
}

cia_status batch_finish(cia_plan *p, BatchAcc &A) {
    const int32_t count = (int32_t)A.ncn.size();
    if (count < 1) return set_error(CIA_EINVAL, "batch: no instance was added");
    P1 u;
    CIA_TRY(batch_union(A, u));
    cia_graph ug{};
    ug.n = A.off.back();
    ug.kind = CIA_GRAPH_CSR;
    cia_coupling c0{};
    c0.model = CIA_MODEL_PHASE;
    c0.p = A.p;
    c0.d_sin = A.dsin.data();
    c0.d_cos = A.dcos.data();
    c0.K = 0.0;   // every node carries its instance's K_b / N_b
    BatchSpec bs{count, A.off.data(), A.kn.data()};
    CIA_TRY(phase_build(p, &ug, nullptr, &c0, A.any_omega ? A.omega.data() : nullptr, &A.o, &bs, &u));
    p->batch_off = A.off;
    return CIA_OK;
}

}  // namespace cia

using namespace cia;

extern "C" {

cia_status cia_batch_begin(const cia_options *o, cia_batch **out) {
    clear_error();
    if (!out) return set_error(CIA_EINVAL, "out is NULL");
    *out = nullptr;
    cia_batch *b = new (std::nothrow) cia_batch();
    if (!b) return set_error(CIA_ENOMEM, "host allocation failed");
    if (o) b->acc.o = *o;
    else cia_options_default(&b->acc.o);
    if (b->acc.o.method != CIA_METHOD_CIA && b->acc.o.method != CIA_METHOD_DIRECT) {
        delete b;
        return set_error(CIA_EINVAL, "options.method = %d", o->method);
    }
    *out = b;
    return CIA_OK;
}

cia_status cia_batch_add(cia_batch *b, const cia_graph *g, const int32_t *labels, const cia_coupling *c,
                         const double *omega) {
    clear_error();
    if (!b) return set_error(CIA_EINVAL, "batch is NULL");
    if (b->acc.failed) return set_error(CIA_EINVAL, "batch: an earlier add ran out of host memory");
    try {
        return batch_add(b->acc, g, labels, c, omega);
    } catch (const std::bad_alloc &) {
        b->acc.failed = true;
        return set_error(CIA_ENOMEM, "host allocation failed (batch instance %d)", (int)b->acc.ncn.size());
    }
}

void cia_batch_abort(cia_batch *b) { delete b; }

}  // extern "C"
