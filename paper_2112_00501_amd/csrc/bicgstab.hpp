// Host-side flexible BiCGStab driver (see bicgstab.cpp).
#pragma once

#include "blas.hpp"
#include "cs_internal.hpp"
#include "gcr.hpp"

namespace cs {

// Device workspace of the BiCGStab solver, owned by a clover handle.
struct BicgWork {
    int inner = -1;
    size_t V = 0;
    void *r = nullptr, *rh = nullptr, *p = nullptr, *v = nullptr, *s = nullptr, *t = nullptr;
    void *plo = nullptr, *slo = nullptr, *zp = nullptr, *zs = nullptr, *w = nullptr;
    double2* partials = nullptr;
    BiScalars* sc = nullptr;
    BiTail* tail = nullptr;
    BiTail* host_tail = nullptr;    // pinned
    hipStream_t stream = nullptr;   // private stream (graph capture needs a non-null stream)
    hipGraphExec_t graph = nullptr;
    std::vector<char> graph_key;
    hipError_t ensure(const Geom& g, int inner);
    void drop_graph();
    void release();
    ~BicgWork() { release(); }
};

// Solve D x = b (one CS_F64 field; x holds the start vector) with flexible
// BiCGStab, SAP on the right in precision p.inner.  Uses p.tol, max_iter,
// n_cy, n_mr, inner, reliable_delta, use_graph, sap_cfg.
hipError_t bicgstab_solve(const OpData& op, const GcrParams& p, BicgWork& w, void* x, const void* b,
                          GcrResult* res, hipStream_t user_stream);

}  // namespace cs
