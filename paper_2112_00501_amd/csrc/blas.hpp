// Level-1 kernels of the flexible GCR outer solver.  All arithmetic and all
// reductions are FP64 whatever the storage precision of the operands.
// Reductions are deterministic: each workgroup writes its partial sums and a
// later kernel adds them in a fixed order (a one-workgroup-per-right-hand-side
// finalize, or every workgroup of the consuming kernel).
//
// Every kernel works on nrhs right-hand sides at once (grid.y = right-hand
// side), each with its own solver scalars; right-hand sides whose entry in the
// device mask `active` is zero are skipped (no mask: all active).  Fields of
// one right-hand side are `stride` bytes apart; basis vectors are stored
// [k][rhs].
#pragma once

#include "cs_internal.hpp"

namespace cs {

constexpr int GCR_MAX_RESTART = 32;
constexpr int BLAS_MAX_WG = 1024;
constexpr int MULTIDOT_CHUNK = 16;

// Solver scalars of one right-hand side, kept on the device between kernels.
struct GcrScalars {
    double2 dots[MULTIDOT_CHUNK + 2];             // reduced sums of the last reduction
    double2 R[GCR_MAX_RESTART][GCR_MAX_RESTART];  // R[j][k] = beta_jk (j < k), nu_k (j = k)
    double inv_nu[GCR_MAX_RESTART];
    double2 c[GCR_MAX_RESTART];
    double2 coef[GCR_MAX_RESTART];                // coefficients of the next update kernel
    double rnorm2;                                // |r|^2 of the current residual
    double inv_rnorm;                             // 1 / |r| (0 when r = 0)
    double nu;                                    // norm of the newest orthogonalised w
};

// Compact per-right-hand-side results the host reads every iteration.
struct GcrTail {
    double rnorm2, nu;
};

struct BlasCtx {
    Geom g;
    int nrhs;
    const int* active;   // device mask [nrhs] or nullptr
    double2* partials;   // [nrhs][BLAS_MAX_WG][MULTIDOT_CHUNK + 2]
    GcrScalars* sc;      // device [nrhs]
    GcrTail* tail;       // device [nrhs]
};

// dst = scale * src per right-hand side; scale_from_sc: use sc[r].inv_rnorm,
// else 1.  dst / src strides follow their precisions.
hipError_t blas_convert(const BlasCtx& c, int dst_prec, void* dst, int src_prec, const void* src,
                        bool scale_from_sc, hipStream_t s);
// dst = gamma5 src (F64 fields; dst may equal src)
hipError_t blas_gamma5(const BlasCtx& c, void* dst, const void* src, hipStream_t s);
// |v|^2 -> sc[r].rnorm2, inv_rnorm and tail[r].rnorm2 (v is F64); with
// lo_prec >= 0 also writes v / |previous residual| in that precision to lo
// (scale 1 when no previous norm is set).
hipError_t blas_norm_to_scalars(const BlasCtx& c, const void* v, int lo_prec, void* lo, hipStream_t s);
// beta_jk = <w_j_hat, w_k> for j < k (W_j stored unnormalised, w_j_hat =
// W_j inv_nu_j); sets R[j][k] = beta_jk and coef[j] = beta_jk inv_nu_j.
hipError_t blas_gcr_project(const BlasCtx& c, int basis_prec, const void* W, size_t wstride, int k,
                            hipStream_t s);
// W_k -= sum_j coef_j W_j and the partial sums of |W_k|^2 and <W_k, r>; the
// scalars of this step are completed by blas_gcr_residual_update, which must
// follow it.
hipError_t blas_gcr_orthonormalise(const BlasCtx& c, int basis_prec, void* W, size_t wstride, int k,
                                   const void* r, hipStream_t s);
// nu = |W_k|, c_k = <W_k, r> / nu -> R[k][k] = nu, inv_nu[k] = 1/nu, c[k],
// tail.nu; then r -= (c_k / nu) W_k and |r|^2 -> rnorm2 / inv_rnorm / tail.
// With lo_prec >= 0 also writes the new r / |old r| in that precision to lo.
hipError_t blas_gcr_residual_update(const BlasCtx& c, int basis_prec, const void* W, size_t wstride,
                                    int k, void* r, int lo_prec, void* lo, hipStream_t s);
// x += sum_{j < nk} gamma_j Z_j, gamma solving R gamma = c over the first nk
// directions, nk = ku[r] for column r (ku may live in pinned host memory;
// columns with nk = 0 are left alone)
hipError_t blas_gcr_solution_update(const BlasCtx& c, int zprec, const void* Z, size_t zstride,
                                    void* x, const int* ku, hipStream_t s);
// Deterministic non-zero test pattern (for timing runs).
hipError_t blas_fill_pattern(const BlasCtx& c, int prec, void* dst, hipStream_t s);

// ---------------------------------------------------------------- BiCGStab
// Scalars of the flexible BiCGStab iteration (one right-hand side), kept on
// the device between kernels.
struct BiScalars {
    double2 rho;    // <rh, r> of the current residual
    double2 alpha, omega, beta;
    double rr;      // |r|^2
    int flag;       // 1: <rh, v> = 0 (iteration abandoned); 2: omega = 0
    int pad;
};

struct BiTail {
    double rr;
    int flag, pad;
};

// Fields of one BiCGStab solve: x, r, rh (shadow), p, v, s, t in the vector
// precision pv (F64, or F32 for the single-precision inner solve); plo / slo
// (smoother inputs) and zp / zs (smoother outputs) in the inner precision pi;
// w (the operator's output) in pw (F64 or F32).
struct BiFields {
    void *x, *r, *rh, *p, *v, *s, *t;
    void *plo, *slo, *zp, *zs, *w;
};

// p = r + beta (p - omega v), plo = p in precision pi
hipError_t bicg_update_p(const BlasCtx& c, const BiScalars* sc, const BiFields& f, int pv, int pi, hipStream_t s);
// v = w; alpha = rho / <rh, v> (flag 1 and alpha = 0 when <rh, v> = 0)
hipError_t bicg_alpha(const BlasCtx& c, BiScalars* sc, const BiFields& f, int pv, int pw, hipStream_t s);
// s = r - alpha v, slo = s in precision pi (nothing under flag 1)
hipError_t bicg_update_s(const BlasCtx& c, const BiScalars* sc, const BiFields& f, int pv, int pi, hipStream_t s);
// t = w; omega = <t, s> / <t, t> (0 and flag 2 when t = 0)
hipError_t bicg_omega(const BlasCtx& c, BiScalars* sc, const BiFields& f, int pv, int pw, hipStream_t s);
// x += alpha zp + omega zs, r = s - omega t; rho' = <rh, r>,
// beta = (rho' / rho)(alpha / omega), rho = rho', rr = |r|^2 -> tail
// (nothing under flag 1)
hipError_t bicg_update_xr(const BlasCtx& c, BiScalars* sc, BiTail* tail, const BiFields& f, int pv, int pi,
                          hipStream_t s);
// restart: rh = r, rho = rr = |r|^2, alpha = omega = 1, beta = 0, flag = 0 -> tail
hipError_t bicg_restart(const BlasCtx& c, BiScalars* sc, BiTail* tail, const BiFields& f, int pv, hipStream_t s);
// |v|^2 -> tail.rr (v in precision pv)
hipError_t bicg_norm2(const BlasCtx& c, BiScalars* sc, BiTail* tail, const void* v, int pv, hipStream_t s);
// dst32 = scale * src64;  x64 += scale * e32
hipError_t bicg_demote(const BlasCtx& c, const void* src64, void* dst32, double scale, hipStream_t s);
hipError_t bicg_promote_add(const BlasCtx& c, void* x64, const void* e32, double scale, hipStream_t s);

// dst = src for bytes (a multiple of 16; both 16-byte aligned): the plain
// copy kernel the field kernels' bandwidth is compared with.
hipError_t stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace cs
