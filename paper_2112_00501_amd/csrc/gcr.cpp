// Flexible GCR(m) outer solver with a SAP or two-level multigrid preconditioner
// (host driver).
//
// Outer arithmetic, reductions and the residual recomputation are FP64; the
// preconditioner and w = D z run in the inner precision.  This is the
// mixed-precision refinement of the paper's Section 2 (a low-precision inner
// solve wrapped in a double-precision outer iteration), with flexible GCR as
// the outer Krylov method because the SAP/MR preconditioner changes from one
// application to the next (the paper's outer solver is flexible as well,
// Section 3).
//
// One iteration k (all on the device; solver scalars stay in device memory):
//   z_k = SAP(r / |r_prev|)            inner precision (r_prev: the residual
//                                      before the update that produced r);
//                                      or z_k = M_MG(r / |r_prev|), FP32
//   w_k = D z_k                        inner precision arithmetic
//   beta_jk = <w_j_hat, w_k>, j < k    classical Gram-Schmidt, FP64
//   w_k -= sum_j beta_jk w_j_hat; nu_k = |w_k|; c_k = <w_k_hat, r>
//   r -= c_k w_k_hat
// followed by one small device-to-host read of |r|^2 and nu_k per right-hand
// side for the stopping test.  At the end of a cycle R gamma = c is solved on
// the host (R upper triangular, R_jk = beta_jk, R_kk = nu_k),
// x += sum_k gamma_k z_k, and the true residual r = b - D x is recomputed in
// FP64.  Convergence is only ever declared on that true residual.
//
// Several right-hand sides advance in lock step through batched kernels
// (multi-right-hand-side SAP and operator launches that reuse links and
// clover); each keeps its own scalars and stops, freezes or restarts on its
// own criteria.  The kernels of one iteration can be captured once per k as a
// HIP graph and replayed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "blas.hpp"
#include "gcr.hpp"

namespace cs {

namespace {

int natural_out(int inner) { return inner == P_F64 ? P_F64 : P_F32; }
int link_for_w(int inner) { return inner == P_F64 ? P_F64 : P_F32; }

#define GCR_CHK(x)                           \
    do {                                     \
        hipError_t e_ = (x);                 \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

}  // namespace

void GcrWork::drop_graphs() {
    for (hipGraphExec_t g : graphs)
        if (g) hipGraphExecDestroy(g);
    graphs.clear();
    graph_key.clear();
}

void GcrWork::release() {
    drop_graphs();
    for (void** p : {&r, &rlo, &Z, &W, &wtmp}) {
        if (*p) hipFree(*p);
        *p = nullptr;
    }
    if (partials) hipFree(partials);
    if (sc) hipFree(sc);
    if (tail) hipFree(tail);
    if (active) hipFree(active);
    if (host_ku) hipHostFree(host_ku);
    if (host_tail) hipHostFree(host_tail);
    if (host_active) hipHostFree(host_active);
    for (hipEvent_t& e : tail_ready) {
        if (e) hipEventDestroy(e);
        e = nullptr;
    }
    if (stream) hipStreamDestroy(stream);
    partials = nullptr;
    sc = nullptr;
    tail = nullptr;
    active = nullptr;
    host_ku = nullptr;
    host_tail = nullptr;
    host_active = nullptr;
    stream = nullptr;
    m = 0;
    nrhs = 0;
}

hipError_t GcrWork::ensure(const Geom& g, int m_, int inner_, int basis_, int nrhs_) {
    if (m_ == m && inner_ == inner && basis_ == basis && nrhs_ == nrhs && W) return hipSuccess;
    release();
    m = m_;
    inner = inner_;
    basis = basis_;
    nrhs = nrhs_;
    const size_t f64 = spinor_bytes_per_site(P_F64) * g.V;
    zstride = spinor_bytes_per_site(inner) * g.V;
    wstride = spinor_bytes_per_site(basis) * g.V;
    hipError_t e;
    if ((e = hipMalloc(&r, f64 * nrhs)) != hipSuccess) return e;
    if ((e = hipMalloc(&rlo, zstride * nrhs)) != hipSuccess) return e;
    if ((e = hipMalloc(&Z, zstride * m * nrhs)) != hipSuccess) return e;
    if ((e = hipMalloc(&W, wstride * m * nrhs)) != hipSuccess) return e;
    if (natural_out(inner) != basis && basis != P_F16 && basis != P_BF16) {
        if ((e = hipMalloc(&wtmp, spinor_bytes_per_site(natural_out(inner)) * g.V * nrhs)) != hipSuccess) return e;
    }
    if ((e = hipMalloc((void**)&partials, sizeof(double2) * BLAS_MAX_WG * (MULTIDOT_CHUNK + 2) * nrhs)) != hipSuccess)
        return e;
    if ((e = hipMalloc((void**)&sc, sizeof(GcrScalars) * nrhs)) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&tail, sizeof(GcrTail) * nrhs)) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&active, sizeof(int) * nrhs)) != hipSuccess) return e;
    // coherent host memory for what kernels read or write directly: no device
    // cache holds a stale copy across solves
    if ((e = hipHostMalloc((void**)&host_ku, sizeof(int) * nrhs, hipHostMallocCoherent)) != hipSuccess) return e;
    if ((e = hipHostMalloc((void**)&host_tail, sizeof(GcrTail) * 2 * nrhs, hipHostMallocCoherent)) != hipSuccess)
        return e;
    if ((e = hipHostMalloc((void**)&host_active, sizeof(int) * 2 * nrhs, hipHostMallocDefault)) != hipSuccess) return e;
    for (hipEvent_t& ev : tail_ready)
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking)) != hipSuccess) return e;
    return hipSuccess;
}

namespace {

struct Solver {
    const OpData& op;
    const GcrParams& p;
    GcrWork& w;
    BlasCtx bc;
    hipStream_t s;
    int n;

    Solver(const OpData& op_, const GcrParams& p_, GcrWork& w_, int nrhs)
        : op(op_), p(p_), w(w_), s(w_.stream), n(nrhs) {
        bc = BlasCtx{op.g, nrhs, w.active, w.partials, w.sc, w.tail};
    }

    size_t f64() const { return spinor_bytes_per_site(P_F64) * op.g.V; }
    // precision of the residual copy the smoother reads (none without smoother)
    int lo_prec() const { return (p.n_cy > 0 || p.mg) ? p.inner : -1; }

    // The copy may run after the host has gone on (an iteration can be queued
    // ahead of it), so consecutive uploads use alternate pinned slots.
    std::vector<char> mask_now;  // the mask last uploaded by this solve
    hipError_t upload_mask(const std::vector<char>& m) {
        if (m == mask_now) return hipSuccess;
        mask_now = m;
        w.mask_slot ^= 1;
        int* h = w.host_active + w.mask_slot * n;
        for (int r = 0; r < n; ++r) h[r] = m[r] ? 1 : 0;
        return hipMemcpyAsync(w.active, h, sizeof(int) * n, hipMemcpyHostToDevice, s);
    }

    // Iteration k, queued without waiting; its kernels write the tails into
    // pinned slot k & 1, and wait_tails(k) returns once they are there.
    hipError_t enqueue_iteration(int k) {
        GCR_CHK(run_iteration(k));
        return hipEventRecord(w.tail_ready[k & 1], s);
    }
    const GcrTail* wait_tails(int k, hipError_t* e) {
        *e = hipEventSynchronize(w.tail_ready[k & 1]);
        return w.host_tail + (k & 1) * n;
    }

    // w = D z for all right-hand sides
    hipError_t apply_w(void* wk, const void* zk) {
        if (w.basis == P_F16 || w.basis == P_BF16) {
            // a 16-bit basis: the operator writes w_k in it directly
            if (n > 1 && p.dslash_cfg.rhs_tile > 1 && p.inner == P_F32)
                return launch_dslash_tiled_to16(op, w.basis, wk, zk, n, p.dslash_cfg, s);
            return launch_dslash(op, p.inner, w.basis, P_F32, false, wk, zk, nullptr, n, s);
        }
        const int nout = natural_out(p.inner);
        const bool tiled = n > 1 && p.dslash_cfg.rhs_tile > 1 && p.inner == nout;
        void* dst = nout == w.basis ? wk : w.wtmp;
        if (tiled) GCR_CHK(launch_dslash_tiled(op, p.inner, false, dst, zk, n, p.dslash_cfg, s));
        else GCR_CHK(launch_dslash(op, p.inner, nout, link_for_w(p.inner), false, dst, zk, nullptr, n, s));
        if (nout != w.basis) GCR_CHK(blas_convert(bc, w.basis, wk, nout, w.wtmp, false, s));
        return hipSuccess;
    }

    // The kernels of iteration k (the part that is graph-captured).
    hipError_t iteration(int k) {
        char* zk = (char*)w.Z + (size_t)k * n * w.zstride;
        char* wk = (char*)w.W + (size_t)k * n * w.wstride;
        if (p.mg) {
            // the coarse phase (restriction and coarse solve) has run already
            GCR_CHK(mg_finish(op, *p.mg, zk, w.rlo, s));
        } else if (p.n_cy > 0) {
            // w.rlo holds the residual in the inner precision, written by the
            // kernel that last updated w.r
            for (int cy = 0; cy < p.n_cy; ++cy)
                for (int col = 0; col < 2; ++col) {
                    const int mode = cy == 0 ? (col == 0 ? 1 : 2) : 0;
                    GCR_CHK(launch_sap_halfsweep(op, p.inner, col, p.n_mr, mode, zk, w.rlo, n, p.sap_cfg, s,
                                                 p.block_solver));
                }
        } else {
            GCR_CHK(blas_convert(bc, p.inner, zk, P_F64, w.r, true, s));
        }
        GCR_CHK(apply_w(wk, zk));
        // the kernels write this iteration's tails straight into pinned host
        // slot k & 1, which the host reads once the iteration's event is done
        BlasCtx bk = bc;
        bk.tail = w.host_tail + (k & 1) * n;
        if (k > 0) GCR_CHK(blas_gcr_project(bk, w.basis, w.W, w.wstride, k, s));
        GCR_CHK(blas_gcr_orthonormalise(bk, w.basis, w.W, w.wstride, k, w.r, s));
        GCR_CHK(blas_gcr_residual_update(bk, w.basis, w.W, w.wstride, k, w.r, lo_prec(), w.rlo, s));
        return hipSuccess;
    }

    std::vector<char> key() const {
        std::vector<char> kbuf(256, 0);
        const int vals[] = {p.restart, p.n_cy, p.n_mr, p.block_solver, p.inner, p.basis, p.sap_cfg.rhs_tile,
                            p.sap_cfg.persistent_wgs, p.sap_cfg.lanes_per_site, p.dslash_cfg.rhs_tile,
                            p.dslash_cfg.persistent_wgs, n};
        std::memcpy(kbuf.data(), vals, sizeof vals);
        const void* ptrs[] = {op.links[0], op.links[1], op.links[2], op.links[3], op.clover64, op.clover32,
                              p.mg, p.mg ? p.mg->P : nullptr, p.mg ? p.mg->Dc : nullptr};
        std::memcpy(kbuf.data() + sizeof vals, ptrs, sizeof ptrs);
        std::memcpy(kbuf.data() + sizeof vals + sizeof ptrs, &op.kappa, sizeof op.kappa);
        if (p.mg) {  // the hierarchy (a fresh id for every allocation) and its shape
            const MgParams& q = p.mg->p;
            const int mv[] = {q.nv, q.n_mr, q.n_coarse, q.n_cy_post, q.coarse_half, q.transfer_half};
            char* at = kbuf.data() + sizeof vals + sizeof ptrs + sizeof op.kappa;
            std::memcpy(at, mv, sizeof mv);
            std::memcpy(at + sizeof mv, &q.tol_coarse, sizeof q.tol_coarse);
            std::memcpy(at + sizeof mv + sizeof q.tol_coarse, &p.mg->id, sizeof p.mg->id);
        }
        return kbuf;
    }

    hipError_t run_iteration(int k) {
        // the multigrid coarse phase runs first, in chunks with host checks
        if (p.mg) GCR_CHK(mg_coarse_phase(*p.mg, w.rlo, s, p.use_graph));
        if (!p.use_graph) return iteration(k);
        const std::vector<char> kk = key();
        if (w.graph_key != kk) {
            w.drop_graphs();
            w.graph_key = kk;
        }
        if ((int)w.graphs.size() < p.restart) w.graphs.resize(p.restart, nullptr);
        if (!w.graphs[k]) {
            hipGraph_t graph;
            GCR_CHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            hipError_t e = iteration(k);
            hipError_t e2 = hipStreamEndCapture(s, &graph);
            if (e != hipSuccess) return e;
            if (e2 != hipSuccess) return e2;
            hipGraphExec_t exec;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (e != hipSuccess) return e;
            w.graphs[k] = exec;
        }
        return hipGraphLaunch(w.graphs[k], s);
    }
};

}  // namespace

hipError_t gcr_solve(const OpData& op, const GcrParams& p, GcrWork& w, void* x, const void* b, int nrhs,
                     bool dagger, void* tmp, GcrResult* res, hipStream_t user_stream) {
    const auto t0 = std::chrono::steady_clock::now();
    GCR_CHK(hipStreamSynchronize(user_stream));  // inputs written on the caller's stream
    Solver S(op, p, w, nrhs);
    hipStream_t s = S.s;
    const size_t f64 = S.f64();
    const int n = nrhs;

    const void* rhs = b;
    if (dagger) {  // D^dag x = b  <=>  D (g5 x) = g5 b
        BlasCtx bc0 = S.bc;
        bc0.active = nullptr;
        GCR_CHK(blas_gamma5(bc0, tmp, b, s));
        GCR_CHK(blas_gamma5(bc0, x, x, s));
        rhs = tmp;
    }

    std::vector<double> bnorm(n), rel(n), r_true(n);
    std::vector<int> status(n, GCR_NOT_CONVERGED), iters(n, 0), cycles(n, 0), k_used(n, 0);
    std::vector<char> done(n, 0), cyc(n, 0), brk(n, 0);

    // |b| into pinned slot 1, then the first true residual r = b - D x
    // (every column) into slot 0, written there by the kernels: one wait
    BlasCtx b_slot1 = S.bc, b_slot0 = S.bc;
    b_slot1.active = b_slot0.active = nullptr;
    b_slot1.tail = w.host_tail + n;
    b_slot0.tail = w.host_tail;
    GCR_CHK(blas_norm_to_scalars(b_slot1, rhs, -1, nullptr, s));
    GCR_CHK(launch_dslash(op, P_F64, P_F64, P_F64, false, w.r, x, rhs, n, s));
    GCR_CHK(blas_norm_to_scalars(b_slot0, w.r, S.lo_prec(), w.rlo, s));
    GCR_CHK(hipStreamSynchronize(s));
    for (int r = 0; r < n; ++r) {
        bnorm[r] = std::sqrt(w.host_tail[n + r].rnorm2);
        if (!std::isfinite(bnorm[r])) {
            status[r] = GCR_NONFINITE;
            rel[r] = bnorm[r];
            done[r] = 1;
        } else if (bnorm[r] == 0.0) {  // D x = 0 has the unique solution x = 0
            GCR_CHK(hipMemsetAsync((char*)x + r * f64, 0, f64, s));
            status[r] = GCR_OK;
            rel[r] = 0.0;
            done[r] = 1;
        }
    }
    auto not_done = [&]() {
        std::vector<char> m(n);
        for (int r = 0; r < n; ++r) m[r] = !done[r];
        return m;
    };
    auto true_residual = [&]() -> hipError_t {
        GCR_CHK(S.upload_mask(not_done()));
        GCR_CHK(launch_dslash(op, P_F64, P_F64, P_F64, false, w.r, x, rhs, n, s));
        BlasCtx bh = S.bc;
        bh.tail = w.host_tail;  // the norm lands in pinned slot 0
        // The smoother's copy is r / |r| with this norm, written once the
        // norm is known: a scale left in the scalars by the last iteration
        // would differ for a column that ran one queued-ahead iteration past
        // its stop, and the copy's rounding with it.
        GCR_CHK(blas_norm_to_scalars(bh, w.r, -1, nullptr, s));
        if (S.lo_prec() >= 0) GCR_CHK(blas_convert(S.bc, S.lo_prec(), w.rlo, P_F64, w.r, true, s));
        GCR_CHK(hipStreamSynchronize(s));
        for (int r = 0; r < n; ++r)
            if (!done[r]) rel[r] = std::sqrt(w.host_tail[r].rnorm2) / bnorm[r];
        return hipSuccess;
    };
    for (int r = 0; r < n; ++r)
        if (!done[r]) rel[r] = std::sqrt(w.host_tail[r].rnorm2) / bnorm[r];

    for (;;) {
        bool any = false;
        for (int r = 0; r < n; ++r) {
            if (done[r]) continue;
            if (!std::isfinite(rel[r])) { status[r] = GCR_NONFINITE; done[r] = 1; }
            else if (rel[r] <= p.tol) { status[r] = GCR_OK; done[r] = 1; }
            else if (iters[r] >= p.max_iter) { status[r] = GCR_NOT_CONVERGED; done[r] = 1; }
            else any = true;
        }
        if (!any) break;
        for (int r = 0; r < n; ++r) {
            cyc[r] = !done[r];
            k_used[r] = 0;
            brk[r] = 0;
            r_true[r] = rel[r] * bnorm[r];
        }
        GCR_CHK(S.upload_mask(cyc));
        // Iteration k + 1 is queued before the host reads the tails of k, so
        // the device does not idle through that round trip.  When every
        // active column is predicted to stop at k (its residual falling by
        // the last step's ratio once more), k + 1 is not queued ahead.  A
        // column that stops at k while k + 1 is already queued runs k + 1
        // once more; that iteration writes only its own slots (W, Z, column
        // k + 1 of R, c_{k+1}), the residual and its norm, which the back
        // substitution (first k_used directions) and the true residual below
        // (residual, norm and smoother copy recomputed from x) do not read.
        std::vector<double> rr_prev(n, 0.0), ratio(n, 1.0);
        for (int r = 0; r < n; ++r) rr_prev[r] = r_true[r];
        auto likely_last = [&](int k) {
            for (int r = 0; r < n; ++r) {
                if (!cyc[r]) continue;
                const double pred = rr_prev[r] * ratio[r];
                const bool stop = pred <= p.tol * bnorm[r] || iters[r] + 1 >= p.max_iter ||
                                  (p.reliable_delta > 0.0 && pred < p.reliable_delta * r_true[r]);
                if (!stop) return false;
            }
            (void)k;
            return true;
        };
        GCR_CHK(S.enqueue_iteration(0));
        for (int k = 0; k < p.restart; ++k) {
            // With the multigrid preconditioner nothing is queued ahead: its
            // coarse phase reads a stop flag on the host between chunks, so
            // queuing k + 1 would make the host wait for k + 1's coarse solve
            // before it could read the tails of k.
            const bool ahead = !p.mg && k + 1 < p.restart && !likely_last(k);
            if (ahead) GCR_CHK(S.enqueue_iteration(k + 1));
            hipError_t we;
            const GcrTail* tails = S.wait_tails(k, &we);
            if (we != hipSuccess) return we;
            bool changed = false, left = false;
            for (int r = 0; r < n; ++r) {
                if (!cyc[r]) continue;
                const GcrTail& t = tails[r];
                if (!(t.nu > 0.0)) {
                    brk[r] = 1;
                    cyc[r] = 0;
                    changed = true;
                    continue;
                }
                ++iters[r];
                k_used[r] = k + 1;
                const double rr = std::sqrt(t.rnorm2);
                if (!std::isfinite(rr) || rr <= p.tol * bnorm[r] || iters[r] >= p.max_iter ||
                    (p.reliable_delta > 0.0 && rr < p.reliable_delta * r_true[r])) {
                    cyc[r] = 0;
                    changed = true;
                }
                ratio[r] = rr_prev[r] > 0.0 ? std::min(1.0, rr / rr_prev[r]) : 1.0;
                rr_prev[r] = rr;
                left = left || cyc[r];
            }
            if (!left) break;
            if (changed) GCR_CHK(S.upload_mask(cyc));
            if (!ahead && k + 1 < p.restart) GCR_CHK(S.enqueue_iteration(k + 1));
        }
        // x += sum_k gamma_k z_k with R gamma = c over each column's first
        // k_used directions; the solution-update kernel solves the small
        // triangular system itself, reading k_used from pinned host memory
        // (nothing reads host_ku once the true residual below has been read)
        bool any_upd = false;
        for (int r = 0; r < n; ++r) {
            w.host_ku[r] = k_used[r];
            any_upd = any_upd || k_used[r] > 0;
        }
        if (any_upd) GCR_CHK(blas_gcr_solution_update(S.bc, p.inner, w.Z, w.zstride, x, w.host_ku, s));
        // reliable update: true FP64 residual
        GCR_CHK(true_residual());
        for (int r = 0; r < n; ++r) {
            if (done[r]) continue;
            ++cycles[r];
            if (brk[r]) {
                status[r] = rel[r] <= p.tol ? GCR_OK : GCR_BREAKDOWN;
                done[r] = 1;
            }
        }
    }
    if (dagger) {
        BlasCtx bc0 = S.bc;
        bc0.active = nullptr;
        GCR_CHK(blas_gamma5(bc0, x, x, s));
    }
    GCR_CHK(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int r = 0; r < n; ++r) {
        res[r].status = status[r];
        res[r].iters = iters[r];
        res[r].restarts = cycles[r];
        res[r].true_relres = rel[r];
        res[r].seconds = secs;
    }
    return hipSuccess;
}

}  // namespace cs
