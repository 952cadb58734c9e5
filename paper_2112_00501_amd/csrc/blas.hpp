// Level-1 kernels of the flexible GCR outer solver.  All arithmetic and all
// reductions are FP64 whatever the storage precision of the operands.
// Reductions are deterministic: each workgroup writes its partial sums and a
// single-workgroup kernel adds them in a fixed order.
#pragma once

#include "cs_internal.hpp"

namespace cs {

constexpr int GCR_MAX_RESTART = 32;
constexpr int BLAS_MAX_WG = 1024;
constexpr int MULTIDOT_CHUNK = 16;

// Solver scalars kept on the device between kernels, so one GCR iteration
// needs a single device-to-host read (of `status`).
struct GcrScalars {
    double2 dots[MULTIDOT_CHUNK + 2];        // finalize output
    double2 R[GCR_MAX_RESTART][GCR_MAX_RESTART];  // R[j][k] = beta_jk (j < k), nu_k (j = k)
    double inv_nu[GCR_MAX_RESTART];
    double2 c[GCR_MAX_RESTART];
    double2 coef[GCR_MAX_RESTART];           // coefficients of the next update kernel
    double2 gamma[GCR_MAX_RESTART];          // back-substitution result (host -> device)
    double rnorm2;                           // |r|^2 of the current residual
    double inv_rnorm;                        // 1 / |r| (scale of the low-precision copy)
    double nu;                               // norm of the newest orthogonalised w
};

struct BlasCtx {
    Geom g;
    double2* partials;   // [BLAS_MAX_WG][MULTIDOT_CHUNK + 2]
    GcrScalars* sc;      // device
};

// dst = scale * src (scale: device pointer, or nullptr for 1)
hipError_t blas_convert(const BlasCtx& c, int dst_prec, void* dst, int src_prec, const void* src,
                        const double* scale, hipStream_t s);
// dst = gamma5 src (F64 fields; dst may equal src)
hipError_t blas_gamma5(const BlasCtx& c, void* dst, const void* src, hipStream_t s);
// |v|^2 -> sc->rnorm2 and sc->inv_rnorm (v is F64)
hipError_t blas_norm_to_scalars(const BlasCtx& c, const void* v, hipStream_t s);
// beta_jk = <w_j_hat, w_k> for j < k (W stored unnormalised, w_j_hat = W_j * inv_nu_j);
// sets R[j][k] = beta_jk and coef[j] = beta_jk * inv_nu_j.
hipError_t blas_gcr_project(const BlasCtx& c, int basis_prec, const void* W, size_t wstride, int k,
                            hipStream_t s);
// W_k -= sum_j coef_j W_j, then nu = |W_k|, c_k = <W_k, r> / nu, R[k][k] = nu,
// inv_nu[k] = 1/nu, coef[0] = c_k / nu.
hipError_t blas_gcr_orthonormalise(const BlasCtx& c, int basis_prec, void* W, size_t wstride, int k,
                                   const void* r, hipStream_t s);
// r -= coef[0] W_k, then |r|^2 -> rnorm2 / inv_rnorm.
hipError_t blas_gcr_residual_update(const BlasCtx& c, int basis_prec, const void* Wk, void* r,
                                    hipStream_t s);
// x += sum_{j < k} gamma_j Z_j
hipError_t blas_gcr_solution_update(const BlasCtx& c, int zprec, const void* Z, size_t zstride, int k,
                                    void* x, hipStream_t s);

}  // namespace cs
