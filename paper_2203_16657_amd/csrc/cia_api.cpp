// The C ABI of libcia: argument checks, device selection, dispatch to the
// model implementations, kernel timing and plan introspection.
#include <cmath>
#include <cstring>
#include <new>

#include <memory>

#include "plan.h"

namespace cia {

cia_status timing_begin(cia_plan *p, hipStream_t s, int kind, int weight) {
    p->ev_open = false;
    if (p->timing_every <= 0) return CIA_OK;
    if (p->tick[kind]++ % p->timing_every != 0) return CIA_OK;
    if (p->ev_used == p->events.size()) {
        cia_plan::EvPair e;
        CIA_HIP(hipEventCreate(&e.a));
        CIA_HIP(hipEventCreate(&e.b));
        e.kind = kind;
        e.weight = weight;
        p->events.push_back(e);
    }
    auto &e = p->events[p->ev_used];
    e.kind = kind;
    e.weight = weight;
    CIA_HIP(hipEventRecord(e.a, s));
    p->last_stream = s;
    p->ev_open = true;
    return CIA_OK;
}

cia_status timing_end(cia_plan *p, hipStream_t s) {
    if (!p->ev_open) return CIA_OK;
    p->ev_open = false;
    CIA_HIP(hipEventRecord(p->events[p->ev_used].b, s));
    p->ev_used++;
    // bound the number of events in flight
    if (p->ev_used >= 8192) CIA_TRY(timing_collect(p));
    return CIA_OK;
}

cia_status timing_collect(cia_plan *p) {
    if (p->ev_used == 0) return CIA_OK;
    CIA_HIP(hipEventSynchronize(p->events[p->ev_used - 1].b));
    for (size_t k = 0; k < p->ev_used; k++) {
        float ms = 0.f;
        CIA_HIP(hipEventElapsedTime(&ms, p->events[k].a, p->events[k].b));
        p->t_ms[p->events[k].kind] += ms;
        p->t_count[p->events[k].kind] += p->events[k].weight;
    }
    p->ev_used = 0;
    return CIA_OK;
}

static cia_status select_device(cia_plan *p) {
    int cur = 0;
    CIA_HIP(hipGetDevice(&cur));
    if (cur != p->device) CIA_HIP(hipSetDevice(p->device));
    return CIA_OK;
}

static void free_plan(cia_plan *p) {
    if (!p) return;
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != p->device) (void)hipSetDevice(p->device);
    for (auto &e : p->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (void *q : p->dev_allocs)
        if (q) (void)hipFree(q);
    phase_free(p);
    flock_free(p);
    struct_free(p);
    if (cur >= 0 && cur != p->device) (void)hipSetDevice(cur);
    delete p;
}

// Checks the options, creates the plan on the selected device and runs
// `fill`; on failure nothing leaks and *out stays NULL.
template <typename Fill>
static cia_status make_plan(const cia_options *o, int64_t n, int32_t model, cia_plan **out, Fill fill) {
    if (o->method != CIA_METHOD_CIA && o->method != CIA_METHOD_DIRECT)
        return set_error(CIA_EINVAL, "options.method = %d", o->method);
    if (o->precision != CIA_F32 && o->precision != CIA_F64)
        return set_error(CIA_EINVAL, "options.precision = %d", o->precision);
    if (o->stepper != CIA_RK4 && o->stepper != CIA_EULER)
        return set_error(CIA_EINVAL, "options.stepper = %d", o->stepper);
    int ndev = 0;
    hipError_t he = hipGetDeviceCount(&ndev);
    if (he != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return set_error(CIA_EHIP, "no HIP device available (%s)", hipGetErrorString(he));
    }
    cia_plan *p = new (std::nothrow) cia_plan();
    if (!p) return set_error(CIA_ENOMEM, "host allocation failed");
    p->model = model;
    p->method = o->method;
    p->precision = o->precision;
    p->stepper = o->stepper;
    p->flags = o->flags;
    p->timing_every = (o->flags & CIA_FLAG_TIMING) ? 1 : 0;
    p->n = n;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) cur = 0;
    p->device = o->device >= 0 ? o->device : cur;
    if (p->device >= ndev) {
        delete p;
        return set_error(CIA_EINVAL, "options.device = %d but only %d devices", o->device, ndev);
    }
    cia_status st = select_device(p);
    if (st == CIA_OK) {
        try {
            st = fill(p);
        } catch (const std::bad_alloc &) {
            st = set_error(CIA_ENOMEM, "host allocation failed");
        }
    }
    if (st == CIA_OK && (o->flags & CIA_FLAG_AUTOTUNE) && p->phase) {
        st = phase_autotune(p, nullptr, nullptr);
        if (st == CIA_EUNSUPPORTED) st = CIA_OK;   // nothing to tune
    }
    if (st != CIA_OK) {
        std::string msg = cia_last_error();
        free_plan(p);
        set_error(st, "%s", msg.c_str());
        return st;
    }
    *out = p;
    return CIA_OK;
}

}  // namespace cia

using namespace cia;

extern "C" {

cia_status cia_build(const cia_graph *g, const int32_t *labels, const cia_coupling *c,
                     const double *omega, const cia_options *o, cia_plan **out) {
    clear_error();
    if (!out) return set_error(CIA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) return set_error(CIA_EINVAL, "graph is NULL");
    if (!c) return set_error(CIA_EINVAL, "coupling is NULL");
    cia_options def;
    cia_options_default(&def);
    if (!o) o = &def;
    if (g->n <= 0) return set_error(CIA_EINVAL, "graph: n = %lld, need n >= 1", (long long)g->n);
    if (c->model != CIA_MODEL_PHASE && c->model != CIA_MODEL_TRIADIC && c->model != CIA_MODEL_FLOCK &&
        c->model != CIA_MODEL_POLY)
        return set_error(CIA_EINVAL, "coupling.model = %d", c->model);
    return make_plan(o, g->n, c->model, out, [&](cia_plan *p) -> cia_status {
        if (g->kind == CIA_GRAPH_RANK1 || g->kind == CIA_GRAPH_RING) return struct_build(p, g, labels, c, omega, o);
        if (c->model == CIA_MODEL_FLOCK) return flock_build(p, g, labels, c, o);
        return phase_build(p, g, labels, c, omega, o);
    });
}

cia_status cia_batch_finish(cia_batch *b, cia_plan **out) {
    clear_error();
    if (!out) {
        delete b;
        return set_error(CIA_EINVAL, "out is NULL");
    }
    *out = nullptr;
    if (!b) return set_error(CIA_EINVAL, "batch is NULL");
    std::unique_ptr<cia_batch> own(b);
    if (b->acc.failed) return set_error(CIA_EINVAL, "batch: an earlier add ran out of host memory");
    if (b->acc.ncn.empty()) return set_error(CIA_EINVAL, "batch: no instance was added");
    const cia_options o = b->acc.o;
    return make_plan(&o, b->acc.off.back(), CIA_MODEL_PHASE, out, [&](cia_plan *p) -> cia_status {
        return batch_finish(p, b->acc);
    });
}

cia_status cia_build_batch(int32_t count, const cia_graph *graphs, const int32_t *const *labels,
                           const cia_coupling *couplings, const double *const *omegas, const cia_options *o,
                           cia_plan **out) {
    clear_error();
    if (!out) return set_error(CIA_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1) return set_error(CIA_EINVAL, "count = %d", count);
    if (!graphs || !couplings) return set_error(CIA_EINVAL, "graphs/couplings is NULL");
    cia_batch *b = nullptr;
    CIA_TRY(cia_batch_begin(o, &b));
    for (int32_t k = 0; k < count; k++) {
        cia_status st = cia_batch_add(b, &graphs[k], labels ? labels[k] : nullptr, &couplings[k],
                                      omegas ? omegas[k] : nullptr);
        if (st != CIA_OK) {
            cia_batch_abort(b);
            return st;
        }
    }
    return cia_batch_finish(b, out);
}

cia_status cia_batch_offsets(const cia_plan *p, int32_t *count, int64_t *offsets) {
    clear_error();
    if (!p || !count) return set_error(CIA_EINVAL, "NULL pointer");
    if (p->batch_off.empty()) {
        *count = 1;
        if (offsets) {
            offsets[0] = 0;
            offsets[1] = p->n;
        }
        return CIA_OK;
    }
    *count = (int32_t)p->batch_off.size() - 1;
    if (offsets)
        for (size_t k = 0; k < p->batch_off.size(); k++) offsets[k] = p->batch_off[k];
    return CIA_OK;
}

cia_status cia_autotune(cia_plan *p, void *stream, cia_tune_report *rep) {
    clear_error();
    if (!p) return set_error(CIA_EINVAL, "plan is NULL");
    if (!p->phase) return set_error(CIA_EUNSUPPORTED, "only phase-model plans are tuned");
    CIA_TRY(select_device(p));
    return phase_autotune(p, static_cast<hipStream_t>(stream), rep);
}

cia_status cia_rhs(cia_plan *p, const void *state, void *dstate, void *stream) {
    clear_error();
    if (!p) return set_error(CIA_EINVAL, "plan is NULL");
    if (!state || !dstate) return set_error(CIA_EINVAL, "state/dstate is NULL");
    if (state == dstate) return set_error(CIA_EINVAL, "dstate must not alias state");
    CIA_TRY(select_device(p));
    hipStream_t s = static_cast<hipStream_t>(stream);
    cia_status st;
    switch (p->structd ? -1 : p->model) {
        case -1: st = struct_rhs(p, state, dstate, s); break;
        case CIA_MODEL_PHASE:
        case CIA_MODEL_POLY:
        case CIA_MODEL_TRIADIC: st = phase_rhs(p, state, dstate, s); break;
        case CIA_MODEL_FLOCK: st = flock_rhs(p, state, dstate, s); break;
        default: st = set_error(CIA_EUNSUPPORTED, "model %d", p->model);
    }
    if (st == CIA_OK && p->timing_every > 0) st = timing_collect(p);
    return st;
}

cia_status cia_integrate(cia_plan *p, void *state, double dt, int64_t steps, double *r_trace,
                         void *stream) {
    clear_error();
    if (!p) return set_error(CIA_EINVAL, "plan is NULL");
    if (!state) return set_error(CIA_EINVAL, "state is NULL");
    if (steps < 0) return set_error(CIA_EINVAL, "steps = %lld < 0", (long long)steps);
    if (!std::isfinite(dt)) return set_error(CIA_EINVAL, "dt is not finite");
    CIA_TRY(select_device(p));
    hipStream_t s = static_cast<hipStream_t>(stream);
    cia_status st;
    switch (p->structd ? -1 : p->model) {
        case -1: st = struct_integrate(p, state, dt, steps, r_trace, s); break;
        case CIA_MODEL_PHASE:
        case CIA_MODEL_TRIADIC: st = phase_integrate(p, state, dt, steps, r_trace, s); break;
        case CIA_MODEL_POLY:
            st = r_trace ? set_error(CIA_EINVAL, "r_trace is defined for the phase models only")
                         : phase_integrate(p, state, dt, steps, nullptr, s);
            break;
        case CIA_MODEL_FLOCK:
            st = r_trace ? set_error(CIA_EINVAL, "r_trace is defined for the phase models only")
                         : flock_integrate(p, state, dt, steps, s);
            break;
        default: st = set_error(CIA_EUNSUPPORTED, "model %d", p->model);
    }
    if (st == CIA_OK && p->timing_every > 0) st = timing_collect(p);
    return st;
}

cia_status cia_integrate_noalloc(cia_plan *p, void *state, double dt, int64_t steps, double *r_trace,
                                 void *stream) {
    clear_error();
    if (!p) return set_error(CIA_EINVAL, "plan is NULL");
    if (!state) return set_error(CIA_EINVAL, "state is NULL");
    if (steps < 0) return set_error(CIA_EINVAL, "steps = %lld < 0", (long long)steps);
    if (!std::isfinite(dt)) return set_error(CIA_EINVAL, "dt is not finite");
    if (p->structd || !p->phase || (p->model != CIA_MODEL_PHASE && p->model != CIA_MODEL_TRIADIC))
        return set_error(CIA_EUNSUPPORTED, "allocation-free integration: phase-model plans only");
    CIA_TRY(select_device(p));
    return phase_integrate_noalloc(p, state, dt, steps, r_trace, static_cast<hipStream_t>(stream));
}

cia_status cia_destroy(cia_plan *p) {
    clear_error();
    free_plan(p);
    return CIA_OK;
}

cia_status cia_plan_get_info(const cia_plan *p, cia_plan_info *info) {
    clear_error();
    if (!p || !info) return set_error(CIA_EINVAL, "NULL pointer");
    *info = p->info;
    if (p->model == CIA_MODEL_FLOCK) {
        cia_plan *q = const_cast<cia_plan *>(p);
        CIA_TRY(select_device(q));
        CIA_TRY(flock_judge_count(q, &info->judge_fallbacks));
    }
    return CIA_OK;
}

cia_status cia_plan_set_timing(cia_plan *p, int32_t every) {
    clear_error();
    if (!p) return set_error(CIA_EINVAL, "plan is NULL");
    if (every < 0) return set_error(CIA_EINVAL, "every = %d", every);
    CIA_TRY(select_device(p));
    CIA_TRY(timing_collect(p));
    p->timing_every = every;
    for (auto &k : p->tick) k = 0;
    return CIA_OK;
}

cia_status cia_plan_get_timing(cia_plan *p, cia_timing *t, int reset) {
    clear_error();
    if (!p || !t) return set_error(CIA_EINVAL, "NULL pointer");
    CIA_TRY(timing_collect(p));
    t->stage_ms = p->t_ms[KK_STAGE];
    t->stage_launches = p->t_count[KK_STAGE];
    t->prep_ms = p->t_ms[KK_PREP];
    t->prep_launches = p->t_count[KK_PREP];
    t->aux_ms = p->t_ms[KK_AUX];
    t->aux_launches = p->t_count[KK_AUX];
    if (reset) {
        for (int k = 0; k < 3; k++) p->t_ms[k] = 0, p->t_count[k] = 0;
    }
    return CIA_OK;
}

cia_status cia_basis_param_count(int32_t rank, int64_t *count) {
    clear_error();
    if (!count) return set_error(CIA_EINVAL, "count is NULL");
    if (rank < 16 || rank > 64 || rank % 16) return set_error(CIA_EINVAL, "rank = %d", rank);
    *count = flock_param_count(rank);
    return CIA_OK;
}

cia_status cia_basis_set_params(cia_plan *p, const float *params, int64_t count, const double lo[3],
                                const double hi[3]) {
    clear_error();
    if (!p || !lo || !hi) return set_error(CIA_EINVAL, "NULL pointer");
    CIA_TRY(select_device(p));
    return flock_basis_set_params(p, params, count, lo, hi);
}

cia_status cia_basis_get_params(cia_plan *p, float *params, int64_t count, double lo[3], double hi[3]) {
    clear_error();
    if (!p) return set_error(CIA_EINVAL, "plan is NULL");
    CIA_TRY(select_device(p));
    return flock_basis_get_params(p, params, count, lo, hi);
}

cia_status cia_basis_train(cia_plan *p, const void *state, int32_t iters, uint64_t seed, double *loss_trace,
                           void *stream) {
    clear_error();
    if (!p) return set_error(CIA_EINVAL, "plan is NULL");
    CIA_TRY(select_device(p));
    return flock_basis_train(p, state, iters, seed, loss_trace, static_cast<hipStream_t>(stream));
}

cia_status cia_basis_loss_grad(cia_plan *p, const float *a, const float *b, const float *t, int64_t pairs,
                               float *grad, double *loss, void *stream) {
    clear_error();
    if (!p) return set_error(CIA_EINVAL, "plan is NULL");
    CIA_TRY(select_device(p));
    return flock_basis_loss_grad(p, a, b, t, pairs, grad, loss, static_cast<hipStream_t>(stream));
}

cia_status cia_basis_features(cia_plan *p, const float *x, int64_t n, float *out, void *stream) {
    clear_error();
    if (!p) return set_error(CIA_EINVAL, "plan is NULL");
    CIA_TRY(select_device(p));
    return flock_basis_features(p, x, n, out, static_cast<hipStream_t>(stream));
}

}  // extern "C"
