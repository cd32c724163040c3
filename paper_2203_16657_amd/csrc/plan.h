// The plan object behind the opaque cia_plan handle, and helpers shared by
// the model implementations.
#pragma once

#include <memory>

#include "internal.h"

namespace cia {

enum KernelKind { KK_STAGE = 0, KK_PREP = 1, KK_AUX = 2 };

struct PhaseState;
struct TriadicState;
struct FlockState;
struct StructState;

}  // namespace cia

struct cia_plan {
    int32_t model = 0, method = 0, precision = 0, stepper = 0;
    uint32_t flags = 0;
    int device = 0;
    int64_t n = 0;
    cia_plan_info info{};
    std::vector<void *> dev_allocs;

    // per-kernel timing (CIA_FLAG_TIMING)
    struct EvPair {
        hipEvent_t a, b;
        int kind;
        int weight;   // launches the bracket stands for
    };
    std::vector<EvPair> events;
    size_t ev_used = 0;
    int32_t timing_every = 0;      // events around one launch in this many per kind (0 = off)
    int64_t tick[3] = {0, 0, 0};   // launches seen per kind
    bool ev_open = false;          // the last timing_begin recorded an event
    double t_ms[3] = {0, 0, 0};
    int64_t t_count[3] = {0, 0, 0};
    hipStream_t last_stream = nullptr;

    std::vector<int64_t> batch_off;   // batched ensembles: instance b owns [off[b], off[b+1])

    cia::PhaseState *phase = nullptr;
    cia::TriadicState *tri = nullptr;
    cia::FlockState *flock = nullptr;
    cia::StructState *structd = nullptr;   // rank-one and ring graphs (App. B)
};

namespace cia {

template <typename T>
cia_status dalloc(cia_plan *p, T **ptr, size_t count) {
    *ptr = nullptr;
    if (count == 0) count = 1;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * count);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(e == hipErrorOutOfMemory ? CIA_ENOMEM : CIA_EHIP,
                         "hipMalloc of %zu bytes failed: %s", sizeof(T) * count, hipGetErrorString(e));
    }
    p->dev_allocs.push_back(q);
    *ptr = static_cast<T *>(q);
    return CIA_OK;
}

template <typename T>
cia_status dupload(cia_plan *p, T **ptr, const T *host, size_t count) {
    CIA_TRY(dalloc(p, ptr, count));
    if (count) CIA_HIP(hipMemcpy(*ptr, host, sizeof(T) * count, hipMemcpyHostToDevice));
    return CIA_OK;
}

// Event bracketing of kernel launches (only with CIA_FLAG_TIMING).
cia_status timing_begin(cia_plan *p, hipStream_t s, int kind, int weight = 1);
cia_status timing_end(cia_plan *p, hipStream_t s);
cia_status timing_collect(cia_plan *p);

// A batched ensemble as one network: the disjoint union of the instances,
// instance b owning user ids [offsets[b], offsets[b+1]) with coupling scale
// kn[u] = K_b / N_b for each of its nodes u.
struct BatchSpec {
    int32_t count;
    const int64_t *offsets;   // [count+1]
    const double *kn;         // [offsets[count]]
};

// model entry points (phase model: cia_phase.hip)
// pre: P1 computed by the caller (batched ensembles), moved from; else P1 of g
cia_status phase_build(cia_plan *p, const cia_graph *g, const int32_t *labels, const cia_coupling *c,
                       const double *omega, const cia_options *o, const BatchSpec *bs = nullptr,
                       P1 *pre = nullptr);
cia_status phase_autotune(cia_plan *p, hipStream_t s, cia_tune_report *rep);
// Accumulator of an incremental batch build (cia_batch.cpp).  Rows of the
// union in P1 order are the community rows of instance 0, 1, ... followed by
// the outside rows of instance 0, 1, ...; partner positions stay
// instance-local until the union's layout is known.
struct BatchAcc {
    cia_options o{};
    int32_t p = -1;
    std::vector<double> dsin, dcos;
    std::vector<int64_t> off{0};        // [count+1] user-id offsets
    std::vector<int64_t> ncn;           // community rows per instance
    std::vector<int32_t> comm_size;     // kept communities in union order
    std::vector<int32_t> perm_c, perm_u;    // global user id of community / outside rows
    std::vector<int64_t> negptr_c{0};   // community rows: S-neg lists (community-local)
    std::vector<int32_t> neg;
    std::vector<int64_t> posptr_c{0}, posptr_u{0};   // S-pos lists (direct: whole rows)
    std::vector<int32_t> pos_c, pos_u;
    std::vector<double> omega, kn;      // per user id of the union
    bool any_omega = false;
    bool failed = false;                // an allocation failed part-way through an add
    int64_t nnz_graph = 0;
};

// incremental batch build (cia_batch.cpp): P1 of each added instance appended
// to the accumulator; batch_finish builds the joined plan from it
cia_status batch_add(BatchAcc &A, const cia_graph *g, const int32_t *labels, const cia_coupling *c,
                     const double *omega);
cia_status batch_finish(cia_plan *p, BatchAcc &A);
cia_status phase_rhs(cia_plan *p, const void *state, void *dstate, hipStream_t s);
cia_status phase_integrate(cia_plan *p, void *state, double dt, int64_t steps, double *r_trace,
                           hipStream_t s);
// allocation-free integration (r(t) in the library's static device array of
// NOALLOC_R_MAX doubles per GPU); noalloc_scratch resolves that array's
// device address on the current device
constexpr int64_t NOALLOC_R_MAX = 1 << 17;
static_assert(NOALLOC_R_MAX == CIA_NOALLOC_R_MAX, "scratch size of the allocation-free entry point");
cia_status phase_integrate_noalloc(cia_plan *p, void *state, double dt, int64_t steps, double *r_trace,
                                   hipStream_t s);
cia_status noalloc_scratch(int dev, double **out);
void phase_free(cia_plan *p);

// Phase model on the structured adjacencies of App. B (rank one, ring).
cia_status struct_build(cia_plan *p, const cia_graph *g, const int32_t *labels, const cia_coupling *c,
                        const double *omega, const cia_options *o);
cia_status struct_rhs(cia_plan *p, const void *state, void *dstate, hipStream_t s);
cia_status struct_integrate(cia_plan *p, void *state, double dt, int64_t steps, double *r_trace, hipStream_t s);
void struct_free(cia_plan *p);

// flock model (cia_flock.hip)
cia_status flock_build(cia_plan *p, const cia_graph *g, const int32_t *labels, const cia_coupling *c,
                       const cia_options *o);
cia_status flock_rhs(cia_plan *p, const void *state, void *dstate, hipStream_t s);
cia_status flock_integrate(cia_plan *p, void *state, double dt, int64_t steps, hipStream_t s);
void flock_free(cia_plan *p);
cia_status flock_judge_count(cia_plan *p, int32_t *count);
cia_status flock_basis_features(cia_plan *p, const float *x, int64_t n, float *out, hipStream_t s);
cia_status flock_basis_set_params(cia_plan *p, const float *params, int64_t count, const double lo[3],
                                  const double hi[3]);
cia_status flock_basis_get_params(cia_plan *p, float *params, int64_t count, double lo[3], double hi[3]);
cia_status flock_basis_train(cia_plan *p, const void *state, int32_t iters, uint64_t seed, double *loss_trace,
                             hipStream_t s);
cia_status flock_basis_loss_grad(cia_plan *p, const float *a, const float *b, const float *t, int64_t P,
                                 float *grad, double *loss, hipStream_t s);
int64_t flock_param_count(int32_t rank);

}  // namespace cia

// opaque handle of the cia_batch_* calls
struct cia_batch {
    cia::BatchAcc acc;
};
