// Flexible GCR(m) outer solver with a SAP preconditioner (host driver).
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
//   z_k = SAP(r / |r|)                 inner precision
//   w_k = D z_k                        inner precision arithmetic
//   beta_jk = <w_j_hat, w_k>, j < k    classical Gram-Schmidt, FP64
//   w_k -= sum_j beta_jk w_j_hat; nu_k = |w_k|; c_k = <w_k_hat, r>
//   r -= c_k w_k_hat
// followed by one 24-byte device-to-host read of |r|^2 for the stopping
// test.  At the end of a cycle R gamma = c is solved on the host (R upper
// triangular, R_jk = beta_jk, R_kk = nu_k), x += sum_k gamma_k z_k, and the
// true residual r = b - D x is recomputed in FP64.  Convergence is only ever
// declared on that true residual.
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "blas.hpp"
#include "gcr.hpp"

namespace cs {

namespace {

int natural_out(int inner) { return inner == P_F64 ? P_F64 : P_F32; }
int link_for_w(int inner) { return inner == P_F64 ? P_F64 : P_F32; }

}  // namespace

void GcrWork::release() {
    for (void** p : {&r, &rlo, &Z, &W, &wtmp}) {
        if (*p) hipFree(*p);
        *p = nullptr;
    }
    if (partials) hipFree(partials);
    if (sc) hipFree(sc);
    if (host_sc) hipHostFree(host_sc);
    partials = nullptr;
    sc = nullptr;
    host_sc = nullptr;
    m = 0;
}

hipError_t GcrWork::ensure(const Geom& g, int m_, int inner_, int basis_) {
    if (m_ == m && inner_ == inner && basis_ == basis && W) return hipSuccess;
    release();
    m = m_;
    inner = inner_;
    basis = basis_;
    const size_t f64 = spinor_bytes_per_site(P_F64) * g.V;
    zstride = spinor_bytes_per_site(inner) * g.V;
    wstride = spinor_bytes_per_site(basis) * g.V;
    hipError_t e;
    if ((e = hipMalloc(&r, f64)) != hipSuccess) return e;
    if ((e = hipMalloc(&rlo, zstride)) != hipSuccess) return e;
    if ((e = hipMalloc(&Z, zstride * m)) != hipSuccess) return e;
    if ((e = hipMalloc(&W, wstride * m)) != hipSuccess) return e;
    if (natural_out(inner) != basis) {
        if ((e = hipMalloc(&wtmp, spinor_bytes_per_site(natural_out(inner)) * g.V)) != hipSuccess) return e;
    }
    if ((e = hipMalloc((void**)&partials, sizeof(double2) * BLAS_MAX_WG * (MULTIDOT_CHUNK + 2))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&sc, sizeof(GcrScalars))) != hipSuccess) return e;
    if ((e = hipHostMalloc((void**)&host_sc, sizeof(GcrScalars), hipHostMallocDefault)) != hipSuccess) return e;
    return hipSuccess;
}

#define GCR_CHK(x)                           \
    do {                                     \
        hipError_t e_ = (x);                 \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

// Read the three trailing scalars (rnorm2, inv_rnorm, nu).
static hipError_t read_tail(GcrWork& w, hipStream_t s) {
    const size_t off = offsetof(GcrScalars, rnorm2);
    GCR_CHK(hipMemcpyAsync((char*)w.host_sc + off, (char*)w.sc + off, 3 * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    return hipStreamSynchronize(s);
}

hipError_t gcr_solve_one(const OpData& op, const GcrParams& p, GcrWork& w, void* x, const void* b,
                         GcrResult* res, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const Geom& g = op.g;
    const BlasCtx bc{g, w.partials, w.sc};
    res->status = GCR_NOT_CONVERGED;
    res->iters = 0;
    res->restarts = 0;

    GCR_CHK(blas_norm_to_scalars(bc, b, s));
    GCR_CHK(read_tail(w, s));
    const double bnorm = std::sqrt(w.host_sc->rnorm2);
    if (!std::isfinite(bnorm)) {
        res->status = GCR_NONFINITE;
        res->true_relres = bnorm;
        return hipSuccess;
    }
    if (bnorm == 0.0) {  // D x = 0 has the unique solution x = 0
        GCR_CHK(hipMemsetAsync(x, 0, spinor_bytes_per_site(P_F64) * g.V, s));
        GCR_CHK(hipStreamSynchronize(s));
        res->status = GCR_OK;
        res->true_relres = 0.0;
        res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return hipSuccess;
    }
    // true residual r = b - D x
    GCR_CHK(launch_dslash(op, P_F64, P_F64, P_F64, false, w.r, x, b, 1, s));
    GCR_CHK(blas_norm_to_scalars(bc, w.r, s));
    GCR_CHK(read_tail(w, s));
    double rel = std::sqrt(w.host_sc->rnorm2) / bnorm;
    int iters = 0, cycles = 0;
    const int nout = natural_out(p.inner);

    for (;;) {
        if (!std::isfinite(rel)) { res->status = GCR_NONFINITE; break; }
        if (rel <= p.tol) { res->status = GCR_OK; break; }
        if (iters >= p.max_iter) { res->status = GCR_NOT_CONVERGED; break; }
        const double r_true = rel * bnorm;
        int k_used = 0;
        bool breakdown = false;
        for (int k = 0; k < p.restart; ++k) {
            char* zk = (char*)w.Z + (size_t)k * w.zstride;
            char* wk = (char*)w.W + (size_t)k * w.wstride;
            // z_k = SAP(r / |r|)
            if (p.n_cy > 0) {
                GCR_CHK(blas_convert(bc, p.inner, w.rlo, P_F64, w.r, &w.sc->inv_rnorm, s));
                for (int cy = 0; cy < p.n_cy; ++cy)
                    for (int col = 0; col < 2; ++col) {
                        const int mode = cy == 0 ? (col == 0 ? 1 : 2) : 0;
                        GCR_CHK(launch_sap_halfsweep(op, p.inner, col, p.n_mr, mode, zk, w.rlo, 1, s));
                    }
            } else {
                GCR_CHK(blas_convert(bc, p.inner, zk, P_F64, w.r, &w.sc->inv_rnorm, s));
            }
            // w_k = D z_k
            if (nout == w.basis) {
                GCR_CHK(launch_dslash(op, p.inner, nout, link_for_w(p.inner), false, wk, zk, nullptr, 1, s));
            } else {
                GCR_CHK(launch_dslash(op, p.inner, nout, link_for_w(p.inner), false, w.wtmp, zk, nullptr, 1, s));
                GCR_CHK(blas_convert(bc, w.basis, wk, nout, w.wtmp, nullptr, s));
            }
            if (k > 0) GCR_CHK(blas_gcr_project(bc, w.basis, w.W, w.wstride, k, s));
            GCR_CHK(blas_gcr_orthonormalise(bc, w.basis, w.W, w.wstride, k, w.r, s));
            GCR_CHK(blas_gcr_residual_update(bc, w.basis, wk, w.r, s));
            GCR_CHK(read_tail(w, s));
            if (!(w.host_sc->nu > 0.0)) {
                breakdown = true;
                break;
            }
            ++iters;
            k_used = k + 1;
            const double rr = std::sqrt(w.host_sc->rnorm2);
            if (!std::isfinite(rr)) break;
            if (rr <= p.tol * bnorm || iters >= p.max_iter) break;
            if (p.reliable_delta > 0.0 && rr < p.reliable_delta * r_true) break;
        }
        if (k_used > 0) {
            // back substitution R gamma = c on the host
            GCR_CHK(hipMemcpyAsync(w.host_sc, w.sc, sizeof(GcrScalars), hipMemcpyDeviceToHost, s));
            GCR_CHK(hipStreamSynchronize(s));
            GcrScalars& h = *w.host_sc;
            std::vector<std::complex<double>> gam(k_used);
            for (int k = k_used - 1; k >= 0; --k) {
                std::complex<double> acc(h.c[k].x, h.c[k].y);
                for (int j = k + 1; j < k_used; ++j)
                    acc -= std::complex<double>(h.R[k][j].x, h.R[k][j].y) * gam[j];
                gam[k] = acc / std::complex<double>(h.R[k][k].x, h.R[k][k].y);
            }
            for (int k = 0; k < k_used; ++k) h.gamma[k] = make_double2(gam[k].real(), gam[k].imag());
            const size_t goff = offsetof(GcrScalars, gamma);
            GCR_CHK(hipMemcpyAsync((char*)w.sc + goff, (char*)w.host_sc + goff,
                                   sizeof(double2) * k_used, hipMemcpyHostToDevice, s));
            GCR_CHK(blas_gcr_solution_update(bc, p.inner, w.Z, w.zstride, k_used, x, s));
        }
        // reliable update: true FP64 residual
        GCR_CHK(launch_dslash(op, P_F64, P_F64, P_F64, false, w.r, x, b, 1, s));
        GCR_CHK(blas_norm_to_scalars(bc, w.r, s));
        GCR_CHK(read_tail(w, s));
        rel = std::sqrt(w.host_sc->rnorm2) / bnorm;
        ++cycles;
        if (breakdown) {
            res->status = rel <= p.tol ? GCR_OK : GCR_BREAKDOWN;
            break;
        }
    }
    res->iters = iters;
    res->restarts = cycles;
    res->true_relres = rel;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return hipSuccess;
}

hipError_t gcr_solve_one_dag(const OpData& op, const GcrParams& p, GcrWork& w, void* x, const void* b,
                             void* tmp, GcrResult* res, hipStream_t s) {
    // D^dag = g5 D g5:  D^dag x = b  <=>  D (g5 x) = g5 b
    const BlasCtx bc{op.g, w.partials, w.sc};
    GCR_CHK(blas_gamma5(bc, tmp, b, s));
    GCR_CHK(blas_gamma5(bc, x, x, s));  // start vector g5 x0
    GCR_CHK(gcr_solve_one(op, p, w, x, tmp, res, s));
    return blas_gamma5(bc, x, x, s);
}

}  // namespace cs
