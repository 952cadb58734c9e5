// Level-1 kernels of the flexible GCR outer solver (FP64 arithmetic and
// reductions on operands stored in any precision).  Each kernel walks the
// lattice block by block with one lane per site, so operands of different
// storage precisions line up site by site.
#include "blas.hpp"
#include "fields.hpp"

namespace cs {

namespace {

constexpr int NVS = MULTIDOT_CHUNK + 2;  // partial-sum slots per workgroup
constexpr int TPB = BLOCK_SITES;

enum Step { STEP_NONE = 0, STEP_PROJECT = 1, STEP_ORTHO = 2, STEP_NORM = 3 };

template <int P>
__device__ __forceinline__ void ld64(const void* base, int nblk, int blk, int l, cpx<double>* c) {
    using RS = typename SpinorIO<P>::R;
    cpx<RS> t[12];
    SpinorIO<P>::load(base, nblk, blk, l, t);
#pragma unroll
    for (int k = 0; k < 12; ++k) c[k] = {(double)t[k].re, (double)t[k].im};
}

template <int P>
__device__ __forceinline__ void st64(void* base, int nblk, int blk, int l, const cpx<double>* c) {
    using RS = typename SpinorIO<P>::R;
    cpx<RS> t[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) t[k] = {(RS)c[k].re, (RS)c[k].im};
    SpinorIO<P>::store(base, nblk, blk, l, t);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Reduce NV complex values over the workgroup; lane j < nv writes slot j of
// this workgroup's partials.
template <int NV>
__device__ __forceinline__ void wg_reduce_store(cpx<double>* acc, int nv, double2* out) {
    __shared__ double2 red[4][NV];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double re = wave_sum(acc[j].re), im = wave_sum(acc[j].im);
        if (lane == 0) red[wave][j] = make_double2(re, im);
    }
    __syncthreads();
    if ((int)threadIdx.x < nv) {
        const int j = threadIdx.x;
        double2 t;
        t.x = (red[0][j].x + red[1][j].x) + (red[2][j].x + red[3][j].x);
        t.y = (red[0][j].y + red[1][j].y) + (red[2][j].y + red[3][j].y);
        out[(size_t)blockIdx.x * NVS + j] = t;
    }
}

template <int PD, int PS>
__global__ __launch_bounds__(TPB) void k_convert(Geom g, void* dst, const void* src, const double* scale) {
    const double s = scale ? *scale : 1.0;
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> c[12];
        ld64<PS>(src, g.nblk, blk, threadIdx.x, c);
#pragma unroll
        for (int k = 0; k < 12; ++k) c[k] = s * c[k];
        st64<PD>(dst, g.nblk, blk, threadIdx.x, c);
    }
}

__global__ __launch_bounds__(TPB) void k_gamma5(Geom g, void* dst, const void* src) {
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> c[12];
        ld64<P_F64>(src, g.nblk, blk, threadIdx.x, c);
        negate_lower(c);
        st64<P_F64>(dst, g.nblk, blk, threadIdx.x, c);
    }
}

__global__ __launch_bounds__(TPB) void k_norm2_f64(Geom g, const void* v, double2* partials) {
    cpx<double> acc[1] = {{0.0, 0.0}};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> c[12];
        ld64<P_F64>(v, g.nblk, blk, threadIdx.x, c);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[0].re += c[k].re * c[k].re + c[k].im * c[k].im;
    }
    wg_reduce_store<1>(acc, 1, partials);
}

// partial <W_{j0 + j}, W_k> for j < n (n <= MULTIDOT_CHUNK)
template <int PB>
__global__ __launch_bounds__(TPB) void k_multidot(Geom g, const char* W, size_t ws, int j0, int n, int k,
                                                  double2* partials) {
    cpx<double> acc[MULTIDOT_CHUNK];
#pragma unroll
    for (int j = 0; j < MULTIDOT_CHUNK; ++j) acc[j] = {0.0, 0.0};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> v[12];
        ld64<PB>(W + (size_t)k * ws, g.nblk, blk, threadIdx.x, v);
#pragma unroll
        for (int j = 0; j < MULTIDOT_CHUNK; ++j) {
            if (j < n) {
                cpx<double> w[12];
                ld64<PB>(W + (size_t)(j0 + j) * ws, g.nblk, blk, threadIdx.x, w);
#pragma unroll
                for (int c = 0; c < 12; ++c) cmac_conj(acc[j], w[c], v[c]);
            }
        }
    }
    wg_reduce_store<MULTIDOT_CHUNK>(acc, n, partials);
}

// W_k -= sum_{j<k} coef_j W_j; partials |W_k|^2 and <W_k, r>
template <int PB>
__global__ __launch_bounds__(TPB) void k_ortho(Geom g, char* W, size_t ws, int k, const void* r,
                                               const GcrScalars* sc, double2* partials) {
    cpx<double> acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> v[12];
        ld64<PB>(W + (size_t)k * ws, g.nblk, blk, threadIdx.x, v);
        for (int j = 0; j < k; ++j) {
            const cpx<double> cf = {sc->coef[j].x, sc->coef[j].y};
            cpx<double> w[12];
            ld64<PB>(W + (size_t)j * ws, g.nblk, blk, threadIdx.x, w);
#pragma unroll
            for (int c = 0; c < 12; ++c) v[c] = v[c] - cf * w[c];
        }
        if (k > 0) st64<PB>(W + (size_t)k * ws, g.nblk, blk, threadIdx.x, v);
        cpx<double> rr[12];
        ld64<P_F64>(r, g.nblk, blk, threadIdx.x, rr);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            acc[0].re += v[c].re * v[c].re + v[c].im * v[c].im;
            cmac_conj(acc[1], v[c], rr[c]);
        }
    }
    wg_reduce_store<2>(acc, 2, partials);
}

// r -= coef[0] W_k; partial |r|^2
template <int PB>
__global__ __launch_bounds__(TPB) void k_residual_update(Geom g, const void* Wk, void* r,
                                                         const GcrScalars* sc, double2* partials) {
    const cpx<double> cf = {sc->coef[0].x, sc->coef[0].y};
    cpx<double> acc[1] = {{0.0, 0.0}};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> w[12], rr[12];
        ld64<PB>(Wk, g.nblk, blk, threadIdx.x, w);
        ld64<P_F64>(r, g.nblk, blk, threadIdx.x, rr);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            rr[c] = rr[c] - cf * w[c];
            acc[0].re += rr[c].re * rr[c].re + rr[c].im * rr[c].im;
        }
        st64<P_F64>(r, g.nblk, blk, threadIdx.x, rr);
    }
    wg_reduce_store<1>(acc, 1, partials);
}

// x += sum_{j<k} gamma_j Z_j
template <int PZ>
__global__ __launch_bounds__(TPB) void k_solution_update(Geom g, const char* Z, size_t zs, int k, void* x,
                                                         const GcrScalars* sc) {
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> xx[12];
        ld64<P_F64>(x, g.nblk, blk, threadIdx.x, xx);
        for (int j = 0; j < k; ++j) {
            const cpx<double> gm = {sc->gamma[j].x, sc->gamma[j].y};
            cpx<double> z[12];
            ld64<PZ>(Z + (size_t)j * zs, g.nblk, blk, threadIdx.x, z);
#pragma unroll
            for (int c = 0; c < 12; ++c) cmac(xx[c], gm, z[c]);
        }
        st64<P_F64>(x, g.nblk, blk, threadIdx.x, xx);
    }
}

// Sum the partials of nv values in a fixed order and apply one solver step.
__global__ __launch_bounds__(TPB) void k_finalize(const double2* partials, int nwg, int nv, GcrScalars* sc,
                                                  int step, int k, int j0) {
    __shared__ double2 red[TPB];
    const int t = threadIdx.x;
    for (int v = 0; v < nv; ++v) {
        double2 s = make_double2(0.0, 0.0);
        for (int i = t; i < nwg; i += TPB) {
            s.x += partials[(size_t)i * NVS + v].x;
            s.y += partials[(size_t)i * NVS + v].y;
        }
        red[t] = s;
        __syncthreads();
        for (int w = TPB / 2; w > 0; w >>= 1) {
            if (t < w) {
                red[t].x += red[t + w].x;
                red[t].y += red[t + w].y;
            }
            __syncthreads();
        }
        if (t == 0) sc->dots[v] = red[0];
        __syncthreads();
    }
    if (t != 0) return;
    if (step == STEP_PROJECT) {
        for (int j = 0; j < nv; ++j) {
            const double in = sc->inv_nu[j0 + j];
            const double2 beta = make_double2(sc->dots[j].x * in, sc->dots[j].y * in);
            sc->R[j0 + j][k] = beta;
            sc->coef[j0 + j] = make_double2(beta.x * in, beta.y * in);
        }
    } else if (step == STEP_ORTHO) {
        const double nu = sqrt(sc->dots[0].x);
        const double in = nu > 0.0 ? 1.0 / nu : 0.0;
        sc->nu = nu;
        sc->R[k][k] = make_double2(nu, 0.0);
        sc->inv_nu[k] = in;
        const double2 ck = make_double2(sc->dots[1].x * in, sc->dots[1].y * in);
        sc->c[k] = ck;
        sc->coef[0] = make_double2(ck.x * in, ck.y * in);
    } else if (step == STEP_NORM) {
        const double r2 = sc->dots[0].x;
        sc->rnorm2 = r2;
        sc->inv_rnorm = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
    }
}

int nwg_for(const Geom& g) { return g.nblk < BLAS_MAX_WG ? g.nblk : BLAS_MAX_WG; }

hipError_t finalize(const BlasCtx& c, int nv, int step, int k, int j0, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(TPB), 0, s, c.partials, nwg_for(c.g), nv, c.sc, step, k, j0);
    return hipGetLastError();
}

#define CS_DISPATCH_P(P, CALL)                       \
    switch (P) {                                     \
    case P_F64: { constexpr int PP = P_F64; CALL; } break; \
    case P_F32: { constexpr int PP = P_F32; CALL; } break; \
    case P_F16: { constexpr int PP = P_F16; CALL; } break; \
    case P_BF16: { constexpr int PP = P_BF16; CALL; } break; \
    default: return hipErrorInvalidValue;            \
    }

template <int PD>
hipError_t convert_from(const BlasCtx& c, void* dst, int src_prec, const void* src, const double* scale,
                        hipStream_t s) {
    const dim3 grid(nwg_for(c.g));
    CS_DISPATCH_P(src_prec, hipLaunchKernelGGL((k_convert<PD, PP>), grid, dim3(TPB), 0, s, c.g, dst, src, scale));
    return hipGetLastError();
}

}  // namespace

hipError_t blas_convert(const BlasCtx& c, int dst_prec, void* dst, int src_prec, const void* src,
                        const double* scale, hipStream_t s) {
    ProfScope ps("blas", s);
    switch (dst_prec) {
    case P_F64: return convert_from<P_F64>(c, dst, src_prec, src, scale, s);
    case P_F32: return convert_from<P_F32>(c, dst, src_prec, src, scale, s);
    case P_F16: return convert_from<P_F16>(c, dst, src_prec, src, scale, s);
    case P_BF16: return convert_from<P_BF16>(c, dst, src_prec, src, scale, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t blas_gamma5(const BlasCtx& c, void* dst, const void* src, hipStream_t s) {
    ProfScope ps("blas", s);
    hipLaunchKernelGGL(k_gamma5, dim3(nwg_for(c.g)), dim3(TPB), 0, s, c.g, dst, src);
    return hipGetLastError();
}

hipError_t blas_norm_to_scalars(const BlasCtx& c, const void* v, hipStream_t s) {
    ProfScope ps("blas", s);
    hipLaunchKernelGGL(k_norm2_f64, dim3(nwg_for(c.g)), dim3(TPB), 0, s, c.g, v, c.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(c, 1, STEP_NORM, 0, 0, s);
}

hipError_t blas_gcr_project(const BlasCtx& c, int pb, const void* W, size_t ws, int k, hipStream_t s) {
    ProfScope ps("blas", s);
    for (int j0 = 0; j0 < k; j0 += MULTIDOT_CHUNK) {
        const int n = k - j0 < MULTIDOT_CHUNK ? k - j0 : MULTIDOT_CHUNK;
        const dim3 grid(nwg_for(c.g));
        CS_DISPATCH_P(pb, hipLaunchKernelGGL((k_multidot<PP>), grid, dim3(TPB), 0, s, c.g, (const char*)W, ws, j0, n, k, c.partials));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = finalize(c, n, STEP_PROJECT, k, j0, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t blas_gcr_orthonormalise(const BlasCtx& c, int pb, void* W, size_t ws, int k, const void* r,
                                   hipStream_t s) {
    ProfScope ps("blas", s);
    const dim3 grid(nwg_for(c.g));
    CS_DISPATCH_P(pb, hipLaunchKernelGGL((k_ortho<PP>), grid, dim3(TPB), 0, s, c.g, (char*)W, ws, k, r, c.sc, c.partials));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(c, 2, STEP_ORTHO, k, 0, s);
}

hipError_t blas_gcr_residual_update(const BlasCtx& c, int pb, const void* Wk, void* r, hipStream_t s) {
    ProfScope ps("blas", s);
    const dim3 grid(nwg_for(c.g));
    CS_DISPATCH_P(pb, hipLaunchKernelGGL((k_residual_update<PP>), grid, dim3(TPB), 0, s, c.g, Wk, r, c.sc, c.partials));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(c, 1, STEP_NORM, 0, 0, s);
}

hipError_t blas_gcr_solution_update(const BlasCtx& c, int pz, const void* Z, size_t zs, int k, void* x,
                                    hipStream_t s) {
    ProfScope ps("blas", s);
    const dim3 grid(nwg_for(c.g));
    CS_DISPATCH_P(pz, hipLaunchKernelGGL((k_solution_update<PP>), grid, dim3(TPB), 0, s, c.g, (const char*)Z, zs, k, x, c.sc));
    return hipGetLastError();
}

}  // namespace cs
