// Level-1 kernels of the flexible GCR outer solver (FP64 arithmetic and
// reductions on operands stored in any precision).  Each kernel walks the
// lattice block by block with one lane per site, so operands of different
// storage precisions line up site by site; grid.y runs over right-hand sides.
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

__device__ __forceinline__ bool skip(const int* active) { return active && !active[blockIdx.y]; }

// Reduce NV complex values over the workgroup; lane j < nv writes slot j of
// this workgroup's partials of right-hand side blockIdx.y.
template <int NV>
__device__ __forceinline__ void wg_reduce_store(cpx<double>* acc, int nv, double2* partials) {
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
        partials[((size_t)blockIdx.y * BLAS_MAX_WG + blockIdx.x) * NVS + j] = t;
    }
}

template <int PD, int PS>
__global__ __launch_bounds__(TPB) void k_convert(Geom g, void* dst, size_t ds, const void* src, size_t ss,
                                                 const GcrScalars* sc, const int* active) {
    if (skip(active)) return;
    const double s = sc ? sc[blockIdx.y].inv_rnorm : 1.0;
    char* d = (char*)dst + blockIdx.y * ds;
    const char* q = (const char*)src + blockIdx.y * ss;
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> c[12];
        ld64<PS>(q, g.nblk, blk, threadIdx.x, c);
#pragma unroll
        for (int k = 0; k < 12; ++k) c[k] = s * c[k];
        st64<PD>(d, g.nblk, blk, threadIdx.x, c);
    }
}

__global__ __launch_bounds__(TPB) void k_gamma5(Geom g, void* dst, const void* src, size_t fs) {
    char* d = (char*)dst + blockIdx.y * fs;
    const char* q = (const char*)src + blockIdx.y * fs;
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> c[12];
        ld64<P_F64>(q, g.nblk, blk, threadIdx.x, c);
        negate_lower(c);
        st64<P_F64>(d, g.nblk, blk, threadIdx.x, c);
    }
}

template <int P>
__global__ __launch_bounds__(TPB) void k_fill(Geom g, void* dst, size_t fs) {
    char* d = (char*)dst + blockIdx.y * fs;
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> c[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            unsigned int h = (unsigned int)(((blk * 256 + threadIdx.x) * 12 + k) * 2654435761u + blockIdx.y * 97u);
            h ^= h >> 13;
            h *= 0x5bd1e995u;
            h ^= h >> 15;
            c[k] = {(double)(h & 0xffff) / 65536.0 - 0.5, (double)(h >> 16) / 65536.0 - 0.5};
        }
        st64<P>(d, g.nblk, blk, threadIdx.x, c);
    }
}

__global__ __launch_bounds__(TPB) void k_norm2_f64(Geom g, const void* v, size_t fs, const int* active,
                                                   double2* partials) {
    if (skip(active)) return;
    const char* q = (const char*)v + blockIdx.y * fs;
    cpx<double> acc[1] = {{0.0, 0.0}};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> c[12];
        ld64<P_F64>(q, g.nblk, blk, threadIdx.x, c);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[0].re += c[k].re * c[k].re + c[k].im * c[k].im;
    }
    wg_reduce_store<1>(acc, 1, partials);
}

// partial <W_{j0 + j}, W_k> for j < n (n <= MULTIDOT_CHUNK); W stored [k][rhs]
template <int PB>
__global__ __launch_bounds__(TPB) void k_multidot(Geom g, const char* W, size_t ws, int nrhs, int j0, int n,
                                                  int k, const int* active, double2* partials) {
    if (skip(active)) return;
    const int r = blockIdx.y;
    cpx<double> acc[MULTIDOT_CHUNK];
#pragma unroll
    for (int j = 0; j < MULTIDOT_CHUNK; ++j) acc[j] = {0.0, 0.0};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> v[12];
        ld64<PB>(W + ((size_t)k * nrhs + r) * ws, g.nblk, blk, threadIdx.x, v);
#pragma unroll
        for (int j = 0; j < MULTIDOT_CHUNK; ++j) {
            if (j < n) {
                cpx<double> w[12];
                ld64<PB>(W + ((size_t)(j0 + j) * nrhs + r) * ws, g.nblk, blk, threadIdx.x, w);
#pragma unroll
                for (int c = 0; c < 12; ++c) cmac_conj(acc[j], w[c], v[c]);
            }
        }
    }
    wg_reduce_store<MULTIDOT_CHUNK>(acc, n, partials);
}

// W_k -= sum_{j<k} coef_j W_j; partials |W_k|^2 and <W_k, r>
template <int PB>
__global__ __launch_bounds__(TPB) void k_ortho(Geom g, char* W, size_t ws, int nrhs, int k, const void* rv,
                                               size_t rs, const GcrScalars* sc, const int* active,
                                               double2* partials) {
    if (skip(active)) return;
    const int r = blockIdx.y;
    const GcrScalars* S = sc + r;
    const char* rr_base = (const char*)rv + r * rs;
    cpx<double> acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> v[12];
        ld64<PB>(W + ((size_t)k * nrhs + r) * ws, g.nblk, blk, threadIdx.x, v);
        for (int j = 0; j < k; ++j) {
            const cpx<double> cf = {S->coef[j].x, S->coef[j].y};
            cpx<double> w[12];
            ld64<PB>(W + ((size_t)j * nrhs + r) * ws, g.nblk, blk, threadIdx.x, w);
#pragma unroll
            for (int c = 0; c < 12; ++c) v[c] = v[c] - cf * w[c];
        }
        if (k > 0) st64<PB>(W + ((size_t)k * nrhs + r) * ws, g.nblk, blk, threadIdx.x, v);
        cpx<double> rr[12];
        ld64<P_F64>(rr_base, g.nblk, blk, threadIdx.x, rr);
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
__global__ __launch_bounds__(TPB) void k_residual_update(Geom g, const char* W, size_t ws, int nrhs, int k,
                                                         void* rv, size_t rs, const GcrScalars* sc,
                                                         const int* active, double2* partials) {
    if (skip(active)) return;
    const int r = blockIdx.y;
    const cpx<double> cf = {sc[r].coef[0].x, sc[r].coef[0].y};
    const char* wk = W + ((size_t)k * nrhs + r) * ws;
    char* rr_base = (char*)rv + r * rs;
    cpx<double> acc[1] = {{0.0, 0.0}};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> w[12], rr[12];
        ld64<PB>(wk, g.nblk, blk, threadIdx.x, w);
        ld64<P_F64>(rr_base, g.nblk, blk, threadIdx.x, rr);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            rr[c] = rr[c] - cf * w[c];
            acc[0].re += rr[c].re * rr[c].re + rr[c].im * rr[c].im;
        }
        st64<P_F64>(rr_base, g.nblk, blk, threadIdx.x, rr);
    }
    wg_reduce_store<1>(acc, 1, partials);
}

// x += sum_{j < nk} gamma_j Z_j
template <int PZ>
__global__ __launch_bounds__(TPB) void k_solution_update(Geom g, const char* Z, size_t zs, int nrhs, void* xv,
                                                         size_t xs, const GcrScalars* sc, const int* active) {
    if (skip(active)) return;
    const int r = blockIdx.y;
    const GcrScalars* S = sc + r;
    const int nk = S->nk;
    char* x_base = (char*)xv + r * xs;
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> xx[12];
        ld64<P_F64>(x_base, g.nblk, blk, threadIdx.x, xx);
        for (int j = 0; j < nk; ++j) {
            const cpx<double> gm = {S->gamma[j].x, S->gamma[j].y};
            cpx<double> z[12];
            ld64<PZ>(Z + ((size_t)j * nrhs + r) * zs, g.nblk, blk, threadIdx.x, z);
#pragma unroll
            for (int c = 0; c < 12; ++c) cmac(xx[c], gm, z[c]);
        }
        st64<P_F64>(x_base, g.nblk, blk, threadIdx.x, xx);
    }
}

// Sum the partials of nv values in a fixed order and apply one solver step
// (one workgroup per right-hand side).
__global__ __launch_bounds__(TPB) void k_finalize(const double2* partials, int nwg, int nv, GcrScalars* scs,
                                                  GcrTail* tails, const int* active, int step, int k, int j0) {
    const int r = blockIdx.x;
    if (active && !active[r]) return;
    GcrScalars* sc = scs + r;
    const double2* part = partials + (size_t)r * BLAS_MAX_WG * NVS;
    __shared__ double2 red[TPB];
    const int t = threadIdx.x;
    for (int v = 0; v < nv; ++v) {
        double2 s = make_double2(0.0, 0.0);
        for (int i = t; i < nwg; i += TPB) {
            s.x += part[(size_t)i * NVS + v].x;
            s.y += part[(size_t)i * NVS + v].y;
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
        tails[r].nu = nu;
        sc->R[k][k] = make_double2(nu, 0.0);
        sc->inv_nu[k] = in;
        const double2 ck = make_double2(sc->dots[1].x * in, sc->dots[1].y * in);
        sc->c[k] = ck;
        sc->coef[0] = make_double2(ck.x * in, ck.y * in);
    } else if (step == STEP_NORM) {
        const double r2 = sc->dots[0].x;
        sc->rnorm2 = r2;
        tails[r].rnorm2 = r2;
        sc->inv_rnorm = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
    }
}

int nwg_for(const Geom& g) { return g.nblk < BLAS_MAX_WG ? g.nblk : BLAS_MAX_WG; }

hipError_t finalize(const BlasCtx& c, int nv, int step, int k, int j0, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(c.nrhs), dim3(TPB), 0, s, c.partials, nwg_for(c.g), nv, c.sc, c.tail,
                       c.active, step, k, j0);
    return hipGetLastError();
}

#define CS_DISPATCH_P(P, CALL)                                   \
    switch (P) {                                                 \
    case P_F64: { constexpr int PP = P_F64; CALL; } break;       \
    case P_F32: { constexpr int PP = P_F32; CALL; } break;       \
    case P_F16: { constexpr int PP = P_F16; CALL; } break;       \
    case P_BF16: { constexpr int PP = P_BF16; CALL; } break;     \
    default: return hipErrorInvalidValue;                        \
    }

template <int PD>
hipError_t convert_from(const BlasCtx& c, void* dst, int src_prec, const void* src, bool scale, hipStream_t s) {
    const dim3 grid(nwg_for(c.g), c.nrhs);
    const size_t ds = spinor_bytes_per_site(PD) * c.g.V, ss = spinor_bytes_per_site(src_prec) * c.g.V;
    const GcrScalars* sc = scale ? c.sc : nullptr;
    CS_DISPATCH_P(src_prec, hipLaunchKernelGGL((k_convert<PD, PP>), grid, dim3(TPB), 0, s, c.g, dst, ds, src, ss, sc, c.active));
    return hipGetLastError();
}

size_t f64_stride(const Geom& g) { return spinor_bytes_per_site(P_F64) * g.V; }

}  // namespace

hipError_t blas_convert(const BlasCtx& c, int dst_prec, void* dst, int src_prec, const void* src,
                        bool scale_from_sc, hipStream_t s) {
    ProfScope ps("blas", s);
    switch (dst_prec) {
    case P_F64: return convert_from<P_F64>(c, dst, src_prec, src, scale_from_sc, s);
    case P_F32: return convert_from<P_F32>(c, dst, src_prec, src, scale_from_sc, s);
    case P_F16: return convert_from<P_F16>(c, dst, src_prec, src, scale_from_sc, s);
    case P_BF16: return convert_from<P_BF16>(c, dst, src_prec, src, scale_from_sc, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t blas_gamma5(const BlasCtx& c, void* dst, const void* src, hipStream_t s) {
    ProfScope ps("blas", s);
    hipLaunchKernelGGL(k_gamma5, dim3(nwg_for(c.g), c.nrhs), dim3(TPB), 0, s, c.g, dst, src, f64_stride(c.g));
    return hipGetLastError();
}

hipError_t blas_fill_pattern(const BlasCtx& c, int prec, void* dst, hipStream_t s) {
    const dim3 grid(nwg_for(c.g), c.nrhs);
    const size_t fs = spinor_bytes_per_site(prec) * c.g.V;
    CS_DISPATCH_P(prec, hipLaunchKernelGGL((k_fill<PP>), grid, dim3(TPB), 0, s, c.g, dst, fs));
    return hipGetLastError();
}

hipError_t blas_norm_to_scalars(const BlasCtx& c, const void* v, hipStream_t s) {
    ProfScope ps("blas", s);
    hipLaunchKernelGGL(k_norm2_f64, dim3(nwg_for(c.g), c.nrhs), dim3(TPB), 0, s, c.g, v, f64_stride(c.g),
                       c.active, c.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(c, 1, STEP_NORM, 0, 0, s);
}

hipError_t blas_gcr_project(const BlasCtx& c, int pb, const void* W, size_t ws, int k, hipStream_t s) {
    ProfScope ps("blas", s);
    for (int j0 = 0; j0 < k; j0 += MULTIDOT_CHUNK) {
        const int n = k - j0 < MULTIDOT_CHUNK ? k - j0 : MULTIDOT_CHUNK;
        const dim3 grid(nwg_for(c.g), c.nrhs);
        CS_DISPATCH_P(pb, hipLaunchKernelGGL((k_multidot<PP>), grid, dim3(TPB), 0, s, c.g, (const char*)W, ws, c.nrhs, j0, n, k, c.active, c.partials));
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
    const dim3 grid(nwg_for(c.g), c.nrhs);
    CS_DISPATCH_P(pb, hipLaunchKernelGGL((k_ortho<PP>), grid, dim3(TPB), 0, s, c.g, (char*)W, ws, c.nrhs, k, r, f64_stride(c.g), c.sc, c.active, c.partials));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(c, 2, STEP_ORTHO, k, 0, s);
}

hipError_t blas_gcr_residual_update(const BlasCtx& c, int pb, const void* W, size_t ws, int k, void* r,
                                    hipStream_t s) {
    ProfScope ps("blas", s);
    const dim3 grid(nwg_for(c.g), c.nrhs);
    CS_DISPATCH_P(pb, hipLaunchKernelGGL((k_residual_update<PP>), grid, dim3(TPB), 0, s, c.g, (const char*)W, ws, c.nrhs, k, r, f64_stride(c.g), c.sc, c.active, c.partials));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(c, 1, STEP_NORM, 0, 0, s);
}

hipError_t blas_gcr_solution_update(const BlasCtx& c, int pz, const void* Z, size_t zs, void* x, hipStream_t s) {
    ProfScope ps("blas", s);
    const dim3 grid(nwg_for(c.g), c.nrhs);
    CS_DISPATCH_P(pz, hipLaunchKernelGGL((k_solution_update<PP>), grid, dim3(TPB), 0, s, c.g, (const char*)Z, zs, c.nrhs, x, f64_stride(c.g), c.sc, c.active));
    return hipGetLastError();
}

}  // namespace cs
