// Internal declarations of libcia (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/cia.h"

namespace cia {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
cia_status set_error(cia_status st, const char *fmt, ...);
void clear_error();

#define CIA_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::cia::set_error(CIA_EHIP, "%s failed: %s (%s:%d)", #call,          \
                                    hipGetErrorString(e_), __FILE__, __LINE__);        \
    } while (0)

#define CIA_TRY(expr)                                                                  \
    do {                                                                               \
        cia_status s_ = (expr);                                                        \
        if (s_ != CIA_OK) return s_;                                                   \
    } while (0)

// ---------------------------------------------------------------------------
// P1: permutation into communities and the sparse remainder S (host)
// ---------------------------------------------------------------------------
struct P1 {
    int64_t n = 0;
    int64_t nnz_graph = 0;
    bool complete = false;
    int32_t ncomm = 0;                 // dense communities kept
    std::vector<int32_t> perm;         // position -> user id
    std::vector<int32_t> inv;          // user id -> position
    std::vector<int32_t> comm_off;     // [ncomm+1]; [comm_off[ncomm], n) = no community
    std::vector<int32_t> comm_of_pos;  // community of each position (-1 = none)
    std::vector<int64_t> negptr;       // [n+1]
    std::vector<int32_t> neg_local;    // missing intra partner, index inside the community
    std::vector<int64_t> posptr;       // [n+1]
    std::vector<int32_t> pos;          // +1 partners as positions, increasing
};

// Validate the graph and labels, apply the cost rule, build the permutation
// and (when with_s) the remainder S.  Returns CIA_OK or an error with message.
cia_status p1_build(const cia_graph *g, const int32_t *labels, double dense_alpha,
                    bool keep_labels, bool validate, bool with_s, P1 &out);

// The adjacency in community order: rows = positions, columns = positions,
// rows increasing.  Used by the direct method.
cia_status p1_permuted_adjacency(const cia_graph *g, const P1 &p1, std::vector<int64_t> &rp,
                                 std::vector<int32_t> &col);

// ---------------------------------------------------------------------------
// device buffer helper
// ---------------------------------------------------------------------------
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace cia

// opaque handle of cia_p1_* calls
struct cia_p1 {
    cia::P1 p1;
};
