// Host-side flexible GCR driver (see gcr.cpp).
#pragma once

#include <vector>

#include "blas.hpp"
#include "cs_internal.hpp"
#include "mg.hpp"

namespace cs {

enum { GCR_OK = 0, GCR_NOT_CONVERGED = 1, GCR_BREAKDOWN = 2, GCR_NONFINITE = 3 };

struct GcrParams {
    int restart, max_iter, n_cy, n_mr;
    double tol;
    int inner, basis;
    double reliable_delta;
    LaunchCfg sap_cfg, dslash_cfg;  // multi-right-hand-side launch shapes
    bool use_graph;                 // replay each iteration as a captured HIP graph
    int block_solver;               // BLOCK_MR or BLOCK_JACOBI (n_mr steps either way)
    const MgData* mg = nullptr;     // multigrid preconditioner in place of SAP (one right-hand side, FP32)
};

struct GcrResult {
    int status, iters, restarts;
    double true_relres, seconds;
};

// Device workspace of one solver configuration, owned by a clover handle.
// Right-hand sides advance in lock step; each has its own scalars and stops
// (freezes) on its own criteria, so every column follows exactly the
// iterations a single-right-hand-side solve would make.
struct GcrWork {
    int m = 0, inner = -1, basis = -1, nrhs = 0;
    size_t zstride = 0, wstride = 0;  // bytes of one field (one right-hand side)
    void* r = nullptr;     // FP64 residuals [nrhs]
    void* rlo = nullptr;   // residuals in the inner precision [nrhs]
    void* Z = nullptr;     // preconditioned directions [m][nrhs], inner precision
    void* W = nullptr;     // basis vectors D z [m][nrhs], basis precision
    void* wtmp = nullptr;  // D z before conversion to the basis precision [nrhs]
    double2* partials = nullptr;
    GcrScalars* sc = nullptr;
    int* host_ku = nullptr;         // pinned [nrhs]: directions each column's solution update uses
    GcrTail* tail = nullptr;
    GcrTail* host_tail = nullptr;   // pinned, two slots of [nrhs] (iteration parity)
    int* active = nullptr;
    int* host_active = nullptr;     // pinned, two slots of [nrhs] (alternating uploads)
    int mask_slot = 0;
    hipEvent_t tail_ready[2] = {nullptr, nullptr};  // host_tail slot filled
    hipStream_t stream = nullptr;   // private stream (graph capture needs a non-null stream)
    std::vector<hipGraphExec_t> graphs;
    std::vector<char> graph_key;
    hipError_t ensure(const Geom& g, int m, int inner, int basis, int nrhs);
    void drop_graphs();
    void release();
    ~GcrWork() { release(); }
};

// Solve D x = b for nrhs right-hand sides (consecutive CS_F64 fields).
// With dagger, solve D^dag x = b as D (g5 x) = g5 b (tmp: nrhs F64 fields).
hipError_t gcr_solve(const OpData& op, const GcrParams& p, GcrWork& w, void* x, const void* b, int nrhs,
                     bool dagger, void* tmp, GcrResult* res, hipStream_t user_stream);

}  // namespace cs
