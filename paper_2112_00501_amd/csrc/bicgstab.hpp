// Host-side flexible BiCGStab driver (see bicgstab.cpp).
#pragma once

#include "blas.hpp"
#include "cs_internal.hpp"
#include "gcr.hpp"

namespace cs {

// Device workspace of the BiCGStab solver, owned by a clover handle.  pv is
// the precision of the iteration vectors (F64: flexible BiCGStab on D x = b;
// F32: single-precision inner solves inside an FP64 Richardson iteration,
// which also keeps the FP64 residual r64, the scaled right-hand side bin and
// the inner solution e).
struct BicgWork {
    int inner = -1, pv = -1;
    size_t V = 0;
    void *r = nullptr, *rh = nullptr, *p = nullptr, *v = nullptr, *s = nullptr, *t = nullptr;
    void *plo = nullptr, *slo = nullptr, *zp = nullptr, *zs = nullptr, *w = nullptr;
    void *r64 = nullptr, *bin = nullptr, *e = nullptr;
    double2* partials = nullptr;
    BiScalars* sc = nullptr;
    BiTail* host_tail = nullptr;    // pinned; the finalize kernels write it directly
    hipStream_t stream = nullptr;   // private stream (graph capture needs a non-null stream)
    hipGraphExec_t graph = nullptr;
    hipGraphExec_t mg_graph[3] = {nullptr, nullptr, nullptr};  // the pieces around two coarse phases
    std::vector<char> graph_key;
    hipError_t ensure(const Geom& g, int inner, int pv);
    void drop_graph();
    void release();
    ~BicgWork() { release(); }
};

// Solve D x = b (one CS_F64 field; x holds the start vector) with BiCGStab,
// SAP on the right in precision p.inner.  p.basis = F64: flexible BiCGStab
// with FP64 vectors and reliable restarts; p.basis = F32: FP32 BiCGStab
// inner solves to p.reliable_delta inside an FP64 Richardson iteration.
// Uses p.tol, max_iter, n_cy, n_mr, inner, basis, reliable_delta, use_graph,
// sap_cfg.  With p.mg the preconditioner is the multigrid M_MG (p.inner F32).
hipError_t bicgstab_solve(const OpData& op, const GcrParams& p, BicgWork& w, void* x, const void* b,
                          GcrResult* res, hipStream_t user_stream);

}  // namespace cs
