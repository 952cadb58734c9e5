// Host-side flexible GCR driver (see gcr.cpp).
#pragma once

#include "blas.hpp"
#include "cs_internal.hpp"

namespace cs {

enum { GCR_OK = 0, GCR_NOT_CONVERGED = 1, GCR_BREAKDOWN = 2, GCR_NONFINITE = 3 };

struct GcrParams {
    int restart, max_iter, n_cy, n_mr;
    double tol;
    int inner, basis;
    double reliable_delta;
};

struct GcrResult {
    int status, iters, restarts;
    double true_relres, seconds;
};

// Device workspace of one solver configuration, owned by a clover handle.
struct GcrWork {
    int m = 0, inner = -1, basis = -1;
    size_t zstride = 0, wstride = 0;
    void* r = nullptr;     // FP64 residual
    void* rlo = nullptr;   // residual in the inner precision
    void* Z = nullptr;     // m preconditioned directions, inner precision
    void* W = nullptr;     // m basis vectors D z, basis precision
    void* wtmp = nullptr;  // D z before conversion to the basis precision
    double2* partials = nullptr;
    GcrScalars* sc = nullptr;
    GcrScalars* host_sc = nullptr;  // pinned
    hipError_t ensure(const Geom& g, int m, int inner, int basis);
    void release();
    ~GcrWork() { release(); }
};

hipError_t gcr_solve_one(const OpData& op, const GcrParams& p, GcrWork& w, void* x, const void* b,
                         GcrResult* res, hipStream_t s);
// Solve D^dag x = b as D (g5 x) = g5 b; tmp is one F64 field of workspace.
hipError_t gcr_solve_one_dag(const OpData& op, const GcrParams& p, GcrWork& w, void* x, const void* b,
                             void* tmp, GcrResult* res, hipStream_t s);

}  // namespace cs
