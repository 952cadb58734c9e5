// Flexible BiCGStab with the SAP or the multigrid preconditioner on the right
// (host driver): the outer solver of the paper's multigrid code (Section 3), in the
// mixed-precision form of Section 2 (low-precision smoother and w = D z,
// FP64 everything else).  One iteration, all on the device:
//   p = r + beta (p - omega v)               FP64, plus p in the inner precision
//   ph = SAP(p);  v = D ph                   inner precision
//   alpha = rho / <rh, v>;  s = r - alpha v
//   sh = SAP(s);  t = D sh
//   omega = <t, s> / <t, t>
//   x += alpha ph + omega sh;  r = s - omega t
//   rho' = <rh, r>;  beta = (rho' / rho)(alpha / omega)
// followed by a 16-byte read of |r|^2 for the stopping test.  The true
// residual b - D x is recomputed in FP64 when the recursive one meets the
// tolerance, drops below reliable_delta times the last true one, or the
// iteration breaks down (<rh, v> = 0 or omega = 0); unless it meets the
// tolerance the iteration restarts from x with rh = r.  A restart whose true
// residual has not decreased since the previous restart is a breakdown.
// The kernels of one iteration are the same every time, so they are captured
// once as a HIP graph and replayed.  With the multigrid preconditioner the
// iteration is three captured pieces around the two coarse phases, which run
// in chunks with host reads of their stop flags.
//
// Single-precision form (the scheme of the paper's Section 2 for QWS): the
// iteration vectors are FP32 and BiCGStab solves D e = r / |r| to the
// relative tolerance reliable_delta; an FP64 Richardson iteration around it
// recomputes r = b - D x in FP64 and adds |r| e to x until the true residual
// meets the tolerance.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "bicgstab.hpp"

namespace cs {

namespace {

#define BI_CHK(x)                            \
    do {                                     \
        hipError_t e_ = (x);                 \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

int natural_out(int inner) { return inner == P_F64 ? P_F64 : P_F32; }

}  // namespace

void BicgWork::drop_graph() {
    if (graph) hipGraphExecDestroy(graph);
    graph = nullptr;
    for (hipGraphExec_t& g : mg_graph) {
        if (g) hipGraphExecDestroy(g);
        g = nullptr;
    }
    graph_key.clear();
}

void BicgWork::release() {
    drop_graph();
    for (void** q : {&r, &rh, &p, &v, &s, &t, &plo, &slo, &zp, &zs, &w, &r64, &bin, &e}) {
        if (*q) hipFree(*q);
        *q = nullptr;
    }
    if (partials) hipFree(partials);
    if (sc) hipFree(sc);
    if (host_tail) hipHostFree(host_tail);
    if (stream) hipStreamDestroy(stream);
    partials = nullptr;
    sc = nullptr;
    host_tail = nullptr;
    stream = nullptr;
    inner = -1;
    pv = -1;
    V = 0;
}

hipError_t BicgWork::ensure(const Geom& g, int inner_, int pv_) {
    if (inner_ == inner && pv_ == pv && (size_t)g.V == V && r) return hipSuccess;
    release();
    inner = inner_;
    pv = pv_;
    V = g.V;
    const size_t f64 = spinor_bytes_per_site(P_F64) * g.V;
    const size_t vec = spinor_bytes_per_site(pv) * g.V;
    const size_t lo = spinor_bytes_per_site(inner) * g.V;
    const size_t nat = spinor_bytes_per_site(natural_out(inner)) * g.V;
    hipError_t err;
#define E_(x)                                   \
    if ((err = (x)) != hipSuccess) return err
    for (void** q : {&r, &rh, &p, &v, &s, &t}) E_(hipMalloc(q, vec));
    for (void** q : {&plo, &slo, &zp, &zs}) E_(hipMalloc(q, lo));
    E_(hipMalloc(&w, nat));
    if (pv != P_F64) {
        E_(hipMalloc(&r64, f64));
        E_(hipMalloc(&bin, vec));
        E_(hipMalloc(&e, vec));
    }
    E_(hipMalloc((void**)&partials, sizeof(double2) * BLAS_MAX_WG * (MULTIDOT_CHUNK + 2)));
    E_(hipMalloc((void**)&sc, sizeof(BiScalars)));
    // coherent: the finalize kernels write it and the host reads it after a stream wait
    E_(hipHostMalloc((void**)&host_tail, sizeof(BiTail), hipHostMallocCoherent));
    E_(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
#undef E_
    return hipSuccess;
}

namespace {

struct Bicg {
    const OpData& op;
    const GcrParams& p;
    BicgWork& w;
    BlasCtx bc;
    BiFields f;
    hipStream_t s;

    int pv;

    Bicg(const OpData& op_, const GcrParams& p_, BicgWork& w_, void* x)
        : op(op_), p(p_), w(w_), s(w_.stream), pv(w_.pv) {
        bc = BlasCtx{op.g, 1, nullptr, w.partials, nullptr, nullptr};
        // without smoothing the preconditioner is the identity: z is the
        // inner-precision copy itself
        void* zp = p.n_cy > 0 || p.mg ? w.zp : w.plo;
        void* zs = p.n_cy > 0 || p.mg ? w.zs : w.slo;
        f = BiFields{x, w.r, w.rh, w.p, w.v, w.s, w.t, w.plo, w.slo, zp, zs, w.w};
    }

    // the finalize kernels write the tail straight into pinned host memory
    hipError_t read_tail() { return hipStreamSynchronize(s); }

    // z = SAP(v) from zero (z is v itself without smoothing), then w = D z
    hipError_t precondition_apply(void* lo, void* z) {
        for (int cy = 0; cy < p.n_cy; ++cy)
            for (int col = 0; col < 2; ++col) {
                const int mode = cy == 0 ? (col == 0 ? 1 : 2) : 0;
                BI_CHK(launch_sap_halfsweep(op, p.inner, col, p.n_mr, mode, z, lo, 1, p.sap_cfg, s,
                                            p.block_solver));
            }
        const int nout = natural_out(p.inner);
        return launch_dslash(op, p.inner, nout, nout, false, w.w, z, nullptr, 1, s);
    }

    hipError_t iteration() {
        BI_CHK(bicg_update_p(bc, w.sc, f, pv, p.inner, s));
        BI_CHK(precondition_apply(f.plo, f.zp));
        BI_CHK(bicg_alpha(bc, w.sc, f, pv, natural_out(p.inner), s));
        BI_CHK(bicg_update_s(bc, w.sc, f, pv, p.inner, s));
        BI_CHK(precondition_apply(f.slo, f.zs));
        BI_CHK(bicg_omega(bc, w.sc, f, pv, natural_out(p.inner), s));
        return bicg_update_xr(bc, w.sc, w.host_tail, f, pv, p.inner, s);
    }

    // the pieces of an iteration with the multigrid preconditioner: before
    // the coarse phase of p, between the two coarse phases, after that of s
    hipError_t mg_piece(int piece) {
        const int nout = natural_out(p.inner);
        if (piece == 0) return bicg_update_p(bc, w.sc, f, pv, p.inner, s);
        if (piece == 1) {
            BI_CHK(mg_finish(op, *p.mg, f.zp, f.plo, s));
            BI_CHK(launch_dslash(op, p.inner, nout, nout, false, w.w, f.zp, nullptr, 1, s));
            BI_CHK(bicg_alpha(bc, w.sc, f, pv, nout, s));
            return bicg_update_s(bc, w.sc, f, pv, p.inner, s);
        }
        BI_CHK(mg_finish(op, *p.mg, f.zs, f.slo, s));
        BI_CHK(launch_dslash(op, p.inner, nout, nout, false, w.w, f.zs, nullptr, 1, s));
        BI_CHK(bicg_omega(bc, w.sc, f, pv, nout, s));
        return bicg_update_xr(bc, w.sc, w.host_tail, f, pv, p.inner, s);
    }

    std::vector<char> key(const void* x) const {
        std::vector<char> k(256, 0);
        const int vals[] = {p.n_cy, p.n_mr, p.block_solver, p.inner, pv, p.sap_cfg.rhs_tile, p.sap_cfg.persistent_wgs,
                            p.sap_cfg.lanes_per_site};
        std::memcpy(k.data(), vals, sizeof vals);
        const void* ptrs[] = {op.links[0], op.links[1], op.links[2], op.links[3], op.clover64, op.clover32, x, p.mg};
        std::memcpy(k.data() + sizeof vals, ptrs, sizeof ptrs);
        std::memcpy(k.data() + sizeof vals + sizeof ptrs, &op.kappa, sizeof op.kappa);
        if (p.mg) {  // the hierarchy (a fresh id for every allocation) and its shape
            const MgParams& q = p.mg->p;
            const int mv[] = {q.nv, q.n_mr, q.n_coarse, q.n_cy_post, q.coarse_half, q.transfer_half};
            char* at = k.data() + sizeof vals + sizeof ptrs + sizeof op.kappa;
            std::memcpy(at, mv, sizeof mv);
            std::memcpy(at + sizeof mv, &q.tol_coarse, sizeof q.tol_coarse);
            std::memcpy(at + sizeof mv + sizeof q.tol_coarse, &p.mg->id, sizeof p.mg->id);
        }
        return k;
    }

    hipError_t capture(hipGraphExec_t* exec, int piece) {
        hipGraph_t graph;
        BI_CHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = piece < 0 ? iteration() : mg_piece(piece);
        hipError_t e2 = hipStreamEndCapture(s, &graph);
        if (e != hipSuccess) return e;
        if (e2 != hipSuccess) return e2;
        e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) *exec = nullptr;
        return e;
    }

    hipError_t run_iteration(const void* x) {
        if (p.mg) {
            const bool g = p.use_graph;
            if (g) {
                const std::vector<char> kk = key(x);
                if (w.graph_key != kk) {
                    w.drop_graph();
                    w.graph_key = kk;
                }
                for (int i = 0; i < 3; ++i)
                    if (!w.mg_graph[i]) BI_CHK(capture(&w.mg_graph[i], i));
            }
            BI_CHK(g ? hipGraphLaunch(w.mg_graph[0], s) : mg_piece(0));
            BI_CHK(mg_coarse_phase(*p.mg, f.plo, s, g));
            BI_CHK(g ? hipGraphLaunch(w.mg_graph[1], s) : mg_piece(1));
            BI_CHK(mg_coarse_phase(*p.mg, f.slo, s, g));
            return g ? hipGraphLaunch(w.mg_graph[2], s) : mg_piece(2);
        }
        if (!p.use_graph) return iteration();
        const std::vector<char> kk = key(x);
        if (w.graph_key != kk) {
            w.drop_graph();
            hipGraph_t graph;
            BI_CHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            hipError_t e = iteration();
            hipError_t e2 = hipStreamEndCapture(s, &graph);
            if (e != hipSuccess) return e;
            if (e2 != hipSuccess) return e2;
            e = hipGraphInstantiate(&w.graph, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (e != hipSuccess) {
                w.graph = nullptr;
                return e;
            }
            w.graph_key = kk;
        }
        return hipGraphLaunch(w.graph, s);
    }

    // r = b - D x (precision pv), rh = r, p = v = 0, scalars reset; returns |r|
    hipError_t restart(const void* b, const void* x, double* rnorm) {
        const size_t vec = spinor_bytes_per_site(pv) * op.g.V;
        BI_CHK(launch_dslash(op, pv, pv, pv, false, w.r, x, b, 1, s));
        BI_CHK(hipMemsetAsync(w.p, 0, vec, s));
        BI_CHK(hipMemsetAsync(w.v, 0, vec, s));
        BI_CHK(bicg_restart(bc, w.sc, w.host_tail, f, pv, s));
        BI_CHK(read_tail());
        *rnorm = std::sqrt(w.host_tail->rr);
        return hipSuccess;
    }

    // BiCGStab iterations from the current restart state until the recursive
    // residual |r| is <= stop_le or < stop_lt, omega = 0, or iters reaches
    // max_iter; *abandoned: stopped at <rh, v> = 0 (x and r unchanged)
    hipError_t iterate(const void* x, double stop_le, double stop_lt, int* iters, bool* abandoned) {
        *abandoned = false;
        while (*iters < p.max_iter) {
            BI_CHK(run_iteration(x));
            BI_CHK(read_tail());
            const BiTail t = *w.host_tail;
            if (t.flag & 1) {  // x and r unchanged
                *abandoned = true;
                break;
            }
            ++*iters;
            const double rr = std::sqrt(t.rr);
            if (!std::isfinite(rr) || rr <= stop_le || rr < stop_lt || (t.flag & 2)) break;
        }
        return hipSuccess;
    }
};

}  // namespace

hipError_t bicgstab_solve(const OpData& op, const GcrParams& p, BicgWork& w, void* x, const void* b,
                          GcrResult* res, hipStream_t user_stream) {
    const auto t0 = std::chrono::steady_clock::now();
    BI_CHK(hipStreamSynchronize(user_stream));  // inputs written on the caller's stream
    const bool single = w.pv != P_F64;
    Bicg B(op, p, w, single ? w.e : x);
    hipStream_t s = B.s;
    const size_t f64 = spinor_bytes_per_site(P_F64) * op.g.V;
    int status = GCR_NOT_CONVERGED, iters = 0, restarts = 0;
    double rel = 0.0;

    BI_CHK(bicg_norm2(B.bc, w.sc, w.host_tail, b, P_F64, s));
    BI_CHK(B.read_tail());
    const double bnorm = std::sqrt(w.host_tail->rr);
    if (!std::isfinite(bnorm)) {
        status = GCR_NONFINITE;
        rel = bnorm;
    } else if (bnorm == 0.0) {  // D x = 0 has the unique solution x = 0
        BI_CHK(hipMemsetAsync(x, 0, f64, s));
        status = GCR_OK;
    } else {
        double last_true = 0.0;
        for (int outer = 0;; ++outer) {
            // true FP64 residual
            double rt;
            if (single) {
                BI_CHK(launch_dslash(op, P_F64, P_F64, P_F64, false, w.r64, x, b, 1, s));
                BI_CHK(bicg_norm2(B.bc, w.sc, w.host_tail, w.r64, P_F64, s));
                BI_CHK(B.read_tail());
                rt = std::sqrt(w.host_tail->rr);
            } else {
                BI_CHK(B.restart(b, x, &rt));
            }
            rel = rt / bnorm;
            if (!std::isfinite(rel)) { status = GCR_NONFINITE; break; }
            if (rel <= p.tol) { status = GCR_OK; break; }
            if (iters >= p.max_iter) { status = GCR_NOT_CONVERGED; break; }
            if (outer > 0 && !(rt < last_true)) { status = GCR_BREAKDOWN; break; }
            if (outer > 0) ++restarts;
            last_true = rt;
            bool abandoned;
            if (single) {
                // FP32 BiCGStab on D e = r / |r| to reliable_delta, then x += |r| e
                BI_CHK(bicg_demote(B.bc, w.r64, w.bin, 1.0 / rt, s));
                BI_CHK(hipMemsetAsync(w.e, 0, spinor_bytes_per_site(w.pv) * op.g.V, s));
                double r0;
                BI_CHK(B.restart(w.bin, w.e, &r0));
                BI_CHK(B.iterate(w.e, p.reliable_delta * r0, 0.0, &iters, &abandoned));
                BI_CHK(bicg_promote_add(B.bc, x, w.e, rt, s));
            } else {
                BI_CHK(B.iterate(x, p.tol * bnorm, p.reliable_delta > 0.0 ? p.reliable_delta * last_true : 0.0,
                                 &iters, &abandoned));
            }
        }
    }
    BI_CHK(hipStreamSynchronize(s));
    if (res) {
        res->status = status;
        res->iters = iters;
        res->restarts = restarts;
        res->true_relres = rel;
        res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return hipSuccess;
}

}  // namespace cs
