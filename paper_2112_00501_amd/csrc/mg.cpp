// Two-level multigrid preconditioner (paper Section 3), host drivers.
//
// Setup: v_i = M_SAP eta_i (n_cy_setup SAP cycles from zero, all nv vectors
// in one batched launch per half-sweep); P = the local orthonormalisation of
// v_0 .. v_{nv-1} per aggregate and chirality; D_c = P^dag D P.  Each of the
// n_adapt adaptive passes replaces every v_i by M_MG v_i with the current P
// and D_c, then rebuilds P and D_c.
//
// Application z = M_MG r: r_c = P^dag r; e_c = coarse BiCGStab on D_c r_c
// (FP32 vectors, FP64 reductions, at most n_coarse iterations, stopping at a
// relative residual of tol_coarse, decided on the device); z = P e_c; then
// n_cy_post SAP cycles on D z = r started from z.  The coarse iterations run
// in chunks of MG_CHUNK; after each chunk the host reads the device's stop
// flag, so iterations after convergence are not launched.
#include <hip/hip_runtime.h>

#include <atomic>

#include "blas.hpp"
#include "mg.hpp"

namespace cs {

namespace {

#define MG_CHK(x)                            \
    do {                                     \
        hipError_t e_ = (x);                 \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

// n_cy SAP cycles on D x = b for nrhs FP32 fields; x0_zero: x starts at zero
hipError_t sap_cycles(const OpData& op, const LaunchCfg& cfg, int n_cy, int n_mr, bool x0_zero, void* x,
                      const void* b, int nrhs, hipStream_t s) {
    for (int cy = 0; cy < n_cy; ++cy)
        for (int col = 0; col < 2; ++col) {
            const int mode = (x0_zero && cy == 0) ? (col == 0 ? 1 : 2) : 0;
            MG_CHK(launch_sap_halfsweep(op, P_F32, col, n_mr, mode, x, b, nrhs, cfg, s, BLOCK_MR));
        }
    return hipSuccess;
}

hipError_t rebuild(const OpData& op, MgData& m, hipStream_t s) {
    MG_CHK(hipMemcpyAsync(m.P, m.V, m.field_bytes() * m.p.nv, hipMemcpyDeviceToDevice, s));
    MG_CHK(mg_orthonormalize(m.g, m.P, m.p.nv, s));
    MG_CHK(mg_assemble(op, m.P, m.p.nv, m.Dc, s));
    if (m.p.transfer_half) {
        const BlasCtx bc{m.g, m.p.nv, nullptr, nullptr, nullptr, nullptr};
        MG_CHK(blas_convert(bc, P_F16, m.P16, P_F32, m.P, false, s));
    }
    if (m.p.coarse_half) MG_CHK(mg_coarse_half(m.Dc, m.Dc16, m.dc_bytes() / sizeof(float2), s));
    return hipSuccess;
}

}  // namespace

size_t MgData::field_bytes() const { return spinor_bytes_per_site(P_F32) * g.V; }

void MgData::drop_graphs() const {
    for (Graphs& g : gr) {
        if (g.first) hipGraphExecDestroy(g.first);
        for (hipGraphExec_t e : g.chunk)
            if (e) hipGraphExecDestroy(e);
    }
    gr.clear();
}

void MgData::release() {
    drop_graphs();
    for (void** q : {&P, &P16, &V, &tmp, (void**)&Dc, &Dc16, (void**)&rc, (void**)&cv.x, (void**)&sc, (void**)&pa.A}) {
        if (*q) hipFree(*q);
        *q = nullptr;
    }
    if (host_flag) hipHostFree(host_flag);
    host_flag = nullptr;
    cv = CbVecs{};
    pa = CbPartials{};
}

hipError_t MgData::alloc(const Geom& g_, const MgParams& p_) {
    static std::atomic<unsigned long long> next_id{1};
    release();
    g = g_;
    p = p_;
    id = next_id++;
    MG_CHK(hipMalloc(&P, field_bytes() * p.nv));
    if (p.transfer_half) MG_CHK(hipMalloc(&P16, spinor_bytes_per_site(P_F16) * g.V * p.nv));
    MG_CHK(hipMalloc(&V, field_bytes() * p.nv));
    MG_CHK(hipMalloc(&tmp, field_bytes()));
    MG_CHK(hipMalloc((void**)&Dc, dc_bytes()));
    if (p.coarse_half) MG_CHK(hipMalloc(&Dc16, dc_bytes() / 2));
    MG_CHK(hipMalloc((void**)&rc, coarse_bytes()));
    // the nine coarse vectors and tau (4 vectors) in one allocation (cv.x owns it)
    float2* base = nullptr;
    MG_CHK(hipMalloc((void**)&base, coarse_bytes() * 13));
    const size_t n = (size_t)g.nblk * nc();
    cv.x = base;
    cv.r = base + n;
    cv.rh = base + 2 * n;
    cv.p[0] = base + 3 * n;
    cv.p[1] = base + 4 * n;
    cv.v[0] = base + 5 * n;
    cv.v[1] = base + 6 * n;
    cv.s = base + 7 * n;
    cv.t = base + 8 * n;
    cv.tau = base + 9 * n;
    MG_CHK(hipMalloc((void**)&sc, sizeof(CbScalars)));
    // partial sums, two complex values per workgroup (pa.A owns the allocation)
    const size_t na = 2 * (size_t)MG_ELEM_WG;
    double2* pb = nullptr;
    MG_CHK(hipMalloc((void**)&pb, sizeof(double2) * 3 * na));
    pa = CbPartials{pb, pb + na, pb + 2 * na};
    MG_CHK(hipHostMalloc((void**)&host_flag, sizeof(int), hipHostMallocDefault));
    return hipSuccess;
}

namespace {

// e_c = coarse BiCGStab on D_c from a given coarse right-hand side rc, left
// in cv.x; MG_CHUNK iterations between host reads of the stop flag
hipError_t coarse_solve_from(const MgData& m, const float2* rc, hipStream_t s) {
    const int cap = m.p.n_coarse;
    int done = cap < MG_CHUNK ? cap : MG_CHUNK;
    MG_CHK(mg_coarse_begin(m.g, m.nc(), rc, m.cv, m.sc, m.pa, m.p.tol_coarse, s));
    MG_CHK(mg_coarse_iters(m.g, m.coarse(), m.nc(), m.cv, m.sc, m.pa, 0, done, s));
    while (done < cap) {
        MG_CHK(hipMemcpyAsync(m.host_flag, &m.sc->stopped[done & 1], sizeof(int), hipMemcpyDeviceToHost, s));
        MG_CHK(hipStreamSynchronize(s));
        if (*m.host_flag) break;
        const int to = done + MG_CHUNK < cap ? done + MG_CHUNK : cap;
        MG_CHK(mg_coarse_iters(m.g, m.coarse(), m.nc(), m.cv, m.sc, m.pa, done, to, s));
        done = to;
    }
    return hipSuccess;
}

// One adaptive pass, v_i <- M_MG v_i for all null vectors at once: one
// restriction of all of them, the coarse solves one after another, one
// prolongation of all, and the post-smoothing as one batched SAP launch per
// half-sweep (the results are those of M_MG applied to each v_i in turn).
// W: nv FP32 fields, rcs and ecs: nv coarse vectors each.
hipError_t adaptive_pass(const OpData& op, MgData& m, void* W, float2* rcs, float2* ecs, hipStream_t s) {
    const size_t n = (size_t)m.g.nblk * m.nc();
    MG_CHK(mg_restrict_many(m.g, m.transfer(), m.p.nv, m.V, m.p.nv, rcs, s));
    for (int i = 0; i < m.p.nv; ++i) {
        MG_CHK(coarse_solve_from(m, rcs + (size_t)i * n, s));
        MG_CHK(hipMemcpyAsync(ecs + (size_t)i * n, m.cv.x, n * sizeof(float2), hipMemcpyDeviceToDevice, s));
    }
    MG_CHK(mg_prolong_many(m.g, m.transfer(), m.p.nv, ecs, m.p.nv, W, s));
    MG_CHK(sap_cycles(op, m.sap_cfg, m.p.n_cy_post, m.p.n_mr, false, W, m.V, m.p.nv, s));
    return hipMemcpyAsync(m.V, W, m.field_bytes() * m.p.nv, hipMemcpyDeviceToDevice, s);
}

}  // namespace

hipError_t mg_setup(const OpData& op, MgData& m, const void* etas, hipStream_t s) {
    MG_CHK(sap_cycles(op, m.sap_cfg, m.p.n_cy_setup, m.p.n_mr, true, m.V, etas, m.p.nv, s));
    MG_CHK(rebuild(op, m, s));
    if (m.p.n_adapt <= 0) return hipSuccess;
    // workspace of the batched passes, released once the passes are done
    void* W = nullptr;
    float2* cvs = nullptr;
    const size_t n = (size_t)m.g.nblk * m.nc();
    hipError_t e = hipMalloc(&W, m.field_bytes() * m.p.nv);
    if (e == hipSuccess) e = hipMalloc((void**)&cvs, 2 * n * m.p.nv * sizeof(float2));
    for (int pass = 0; e == hipSuccess && pass < m.p.n_adapt; ++pass) {
        e = adaptive_pass(op, m, W, cvs, cvs + n * m.p.nv, s);
        if (e == hipSuccess) e = rebuild(op, m, s);
    }
    // the frees wait for the queued work that uses the workspace
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (W) hipFree(W);
    if (cvs) hipFree(cvs);
    return e;
}

namespace {

// Run launch() directly, or as a graph captured into *exec on first use.
template <typename F>
hipError_t run_piece(hipGraphExec_t* exec, bool use_graph, hipStream_t s, F launch) {
    if (!use_graph) return launch();
    if (!*exec) {
        hipGraph_t graph;
        MG_CHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = launch();
        hipError_t e2 = hipStreamEndCapture(s, &graph);
        if (e != hipSuccess) return e;
        if (e2 != hipSuccess) return e2;
        e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
    }
    return hipGraphLaunch(*exec, s);
}

}  // namespace

hipError_t mg_coarse_phase(const MgData& m, const void* r, hipStream_t s, bool use_graph) {
    MgData::Graphs* gs = nullptr;
    if (use_graph) {
        for (MgData::Graphs& g : m.gr)
            if (g.r == r) gs = &g;
        if (!gs) {
            if (m.gr.size() >= 4) m.drop_graphs();  // a few input fields at a time
            m.gr.push_back(MgData::Graphs{});
            gs = &m.gr.back();
            gs->r = r;
        }
    }
    MgData::Graphs none;
    MgData::Graphs& G = gs ? *gs : none;
    const int cap = m.p.n_coarse;
    int done = cap < MG_CHUNK ? cap : MG_CHUNK;
    MG_CHK(run_piece(&G.first, use_graph, s, [&]() -> hipError_t {
        MG_CHK(mg_restrict(m.g, m.transfer(), m.p.nv, r, m.rc, s));
        MG_CHK(mg_coarse_begin(m.g, m.nc(), m.rc, m.cv, m.sc, m.pa, m.p.tol_coarse, s));
        return mg_coarse_iters(m.g, m.coarse(), m.nc(), m.cv, m.sc, m.pa, 0, done, s);
    }));
    for (int j = 0; done < cap; ++j) {
        // stopped[done & 1] was set by the stop test of iteration `done`
        MG_CHK(hipMemcpyAsync(m.host_flag, &m.sc->stopped[done & 1], sizeof(int), hipMemcpyDeviceToHost, s));
        MG_CHK(hipStreamSynchronize(s));
        if (*m.host_flag) break;
        const int to = done + MG_CHUNK < cap ? done + MG_CHUNK : cap;
        if ((int)G.chunk.size() <= j) G.chunk.resize(j + 1, nullptr);
        MG_CHK(run_piece(&G.chunk[j], use_graph, s, [&]() -> hipError_t {
            return mg_coarse_iters(m.g, m.coarse(), m.nc(), m.cv, m.sc, m.pa, done, to, s);
        }));
        done = to;
    }
    return hipSuccess;
}

hipError_t mg_finish(const OpData& op, const MgData& m, void* z, const void* r, hipStream_t s) {
    MG_CHK(mg_prolong(m.g, m.transfer(), m.p.nv, m.cv.x, z, s));
    return sap_cycles(op, m.sap_cfg, m.p.n_cy_post, m.p.n_mr, false, z, r, 1, s);
}

hipError_t mg_apply(const OpData& op, const MgData& m, void* z, const void* r, hipStream_t s) {
    MG_CHK(mg_coarse_phase(m, r, s, false));
    return mg_finish(op, m, z, r, s);
}

}  // namespace cs
