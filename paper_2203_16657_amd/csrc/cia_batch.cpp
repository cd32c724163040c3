// Batched ensembles: many phase-model networks integrated as one plan.
//
// The instances are joined into their disjoint union (instance b owns user
// ids [off_b, off_b + N_b) of the joined state).  Communities never span two
// instances, so P1 (permutation, cost rule, S-neg / S-pos) of the union is
// P1 of every instance, and one launch per RK stage covers the work units of
// every instance.  What differs per instance is the coupling scale K_b / N_b
// (eq. 2.1 with each instance's own N), carried per node, and the order
// parameter, reduced per instance.
#include <cmath>
#include <cstring>
#include <map>
#include <new>

#include "plan.h"

namespace cia {

cia_status batch_build(cia_plan *p, int32_t count, const cia_graph *graphs, const int32_t *const *labels,
                       const cia_coupling *couplings, const double *const *omegas, const cia_options *o) {
    const cia_coupling &c0 = couplings[0];
    for (int32_t b = 0; b < count; b++) {
        const cia_graph &g = graphs[b];
        const cia_coupling &c = couplings[b];
        if (g.kind != CIA_GRAPH_CSR)
            return set_error(CIA_EUNSUPPORTED, "batch instance %d: only CSR graphs can be batched", b);
        if (g.n <= 0) return set_error(CIA_EINVAL, "batch instance %d: n = %lld", b, (long long)g.n);
        if (!g.row_ptr || (g.row_ptr[g.n] > 0 && !g.col))
            return set_error(CIA_EINVAL, "batch instance %d: row_ptr/col is NULL", b);
        if (c.model != CIA_MODEL_PHASE)
            return set_error(CIA_EUNSUPPORTED, "batch instance %d: only the phase model can be batched", b);
        if (c.p != c0.p || !c.d_sin || !c.d_cos)
            return set_error(CIA_EINVAL, "batch instance %d: every instance needs the same coupling function", b);
        for (int k = 0; k <= c.p && c.p >= 0 && c.p <= 8; k++)
            if (c.d_sin[k] != c0.d_sin[k] || c.d_cos[k] != c0.d_cos[k])
                return set_error(CIA_EINVAL, "batch instance %d: every instance needs the same coupling function", b);
        if (!std::isfinite(c.K)) return set_error(CIA_EINVAL, "batch instance %d: K is not finite", b);
    }
    std::vector<int64_t> off(count + 1, 0), eoff(count + 1, 0);
    for (int32_t b = 0; b < count; b++) {
        off[b + 1] = off[b] + graphs[b].n;
        eoff[b + 1] = eoff[b] + graphs[b].row_ptr[graphs[b].n];
    }
    const int64_t n = off[count], nnz = eoff[count];
    if (n > INT32_MAX) return set_error(CIA_EUNSUPPORTED, "batch: %lld nodes in total (limit 2^31-1)", (long long)n);
    std::vector<int64_t> rp(n + 1);
    std::vector<int32_t> col(std::max<int64_t>(nnz, 1));
    std::vector<int32_t> lab(n);
    std::vector<double> kn(n), om;
    bool any_omega = false;
    for (int32_t b = 0; b < count; b++) any_omega |= omegas && omegas[b];
    if (any_omega) om.assign(n, 0.0);
    int32_t comm_base = 0;
    for (int32_t b = 0; b < count; b++) {
        const cia_graph &g = graphs[b];
        const int64_t nb = g.n, o0 = off[b], e0 = eoff[b], r0 = g.row_ptr[0];
        if (r0 != 0) return set_error(CIA_EINVAL, "batch instance %d: row_ptr[0] != 0", b);
        for (int64_t i = 0; i < nb; i++) {
            rp[o0 + i] = e0 + g.row_ptr[i];
            if (g.row_ptr[i + 1] < g.row_ptr[i]) return set_error(CIA_EINVAL, "batch instance %d: row_ptr decreases", b);
        }
        for (int64_t e = 0; e < g.row_ptr[nb]; e++) {
            const int32_t v = g.col[e];
            if (v < 0 || v >= nb)
                return set_error(CIA_EINVAL, "batch instance %d: column %d out of range", b, v);
            col[e0 + e] = (int32_t)(v + o0);
        }
        // labels: dense per instance (sorted distinct ids), offset by the
        // communities of the earlier instances; NULL = one community
        const int32_t *lb = labels ? labels[b] : nullptr;
        if (!lb) {
            for (int64_t i = 0; i < nb; i++) lab[o0 + i] = comm_base;
            comm_base += 1;
        } else {
            std::map<int32_t, int32_t> ids;
            for (int64_t i = 0; i < nb; i++) {
                if (lb[i] < -1) return set_error(CIA_EINVAL, "batch instance %d: label %d < -1", b, lb[i]);
                if (lb[i] >= 0) ids.emplace(lb[i], 0);
            }
            int32_t k = 0;
            for (auto &kv : ids) kv.second = k++;
            for (int64_t i = 0; i < nb; i++) lab[o0 + i] = lb[i] < 0 ? -1 : comm_base + ids[lb[i]];
            comm_base += k;
        }
        const double knb = couplings[b].K / (double)nb;
        for (int64_t i = 0; i < nb; i++) kn[o0 + i] = knb;
        if (any_omega && omegas[b])
            for (int64_t i = 0; i < nb; i++) om[o0 + i] = omegas[b][i];
    }
    rp[n] = nnz;
    cia_graph ug{};
    ug.n = n;
    ug.kind = CIA_GRAPH_CSR;
    ug.row_ptr = rp.data();
    ug.col = col.data();
    BatchSpec bs{count, off.data(), kn.data()};
    CIA_TRY(phase_build(p, &ug, lab.data(), &c0, any_omega ? om.data() : nullptr, o, &bs));
    p->batch_off = off;
    return CIA_OK;
}

}  // namespace cia
