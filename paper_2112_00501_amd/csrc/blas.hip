// Level-1 kernels of the flexible GCR outer solver (FP64 arithmetic and
// reductions on operands stored in any precision).  Each kernel walks the
// lattice block by block with one lane per site, so operands of different
// storage precisions line up site by site; grid.y runs over right-hand sides.
#include <type_traits>

#include "blas.hpp"
#include "fields.hpp"
#include "wave.hpp"

namespace cs {

namespace {

constexpr int NVS = MULTIDOT_CHUNK + 2;  // partial-sum slots per workgroup
constexpr int TPB = BLOCK_SITES;

enum Step { STEP_NONE = 0, STEP_PROJECT = 1, STEP_NORM = 2 };

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

__device__ __forceinline__ bool skip(const int* active) { return active && !active[blockIdx.y]; }

// Reduce NV complex values over the workgroup; lane j < nv writes slot v0 + j
// of this workgroup's partials of right-hand side blockIdx.y.
template <int NV>
__device__ __forceinline__ void wg_reduce_store(cpx<double>* acc, int nv, double2* partials, int v0 = 0) {
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
        partials[((size_t)blockIdx.y * BLAS_MAX_WG + blockIdx.x) * NVS + v0 + j] = t;
    }
}

// Sum slots v0 .. v0 + NVP - 1 of nwg workgroup partials (one right-hand side)
// in a fixed order with NT threads: lane t takes slot t % NVP and every
// (NT / NVP)-th workgroup from t / NVP in increasing order (loads issued eight
// at a time), then a fixed tree adds the chunks.  The total of slot v ends in
// red[v].  Any workgroup running this on the same partials gets bitwise the
// same sums.
template <int NVP, int NT>
__device__ __forceinline__ void sum_partials(const double2* part, int nwg, int v0, double2* red) {
    constexpr int G = NT / NVP;
    constexpr int U = 8;
    const int t = threadIdx.x, v = t % NVP, c = t / NVP;
    const double2* p = part + v0 + v;
    double2 s = make_double2(0.0, 0.0);
    int i = c;
    for (; i + (U - 1) * G < nwg; i += U * G) {
        double2 q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) q[u] = p[(size_t)(i + u * G) * NVS];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s.x += q[u].x;
            s.y += q[u].y;
        }
    }
    for (; i < nwg; i += G) {
        const double2 q = p[(size_t)i * NVS];
        s.x += q.x;
        s.y += q.y;
    }
    red[t] = s;
    __syncthreads();
#pragma unroll
    for (int w = G / 2; w > 0; w >>= 1) {
        if (c < w) {
            red[t].x += red[t + w * NVP].x;
            red[t].y += red[t + w * NVP].y;
        }
        __syncthreads();
    }
}

// GCR scalars of the orthonormalisation step from |W_k|^2 and <W_k, r>.
struct OrthoScalars {
    double nu, inv_nu;
    double2 ck, coef;
};

__device__ __forceinline__ OrthoScalars ortho_scalars(double2 ww, double2 wr) {
    OrthoScalars o;
    o.nu = sqrt(ww.x);
    o.inv_nu = o.nu > 0.0 ? 1.0 / o.nu : 0.0;
    o.ck = make_double2(wr.x * o.inv_nu, wr.y * o.inv_nu);
    o.coef = make_double2(o.ck.x * o.inv_nu, o.ck.y * o.inv_nu);
    return o;
}

// Slots of the partials: a projection uses 0 .. MULTIDOT_CHUNK - 1, the
// orthonormalisation 0 and 1 (|W_k|^2, <W_k, r>), a norm NORM_SLOT, so the
// residual update can read the orthonormalisation sums while it writes its own.
constexpr int NORM_SLOT = MULTIDOT_CHUNK;

// Sum the partials and apply one solver step (one workgroup per right-hand side).
constexpr int FIN_TPB = 1024;

template <int NVP>
__global__ __launch_bounds__(FIN_TPB) void k_finalize(const double2* partials, int nwg, int nv, int v0,
                                                      GcrScalars* scs, GcrTail* tails, const int* active, int step,
                                                      int k, int j0) {
    const int r = blockIdx.x;
    if (active && !active[r]) return;
    GcrScalars* sc = scs + r;
    __shared__ double2 red[FIN_TPB];
    sum_partials<NVP, FIN_TPB>(partials + (size_t)r * BLAS_MAX_WG * NVS, nwg, v0, red);
    if (threadIdx.x != 0) return;
    for (int v = 0; v < nv; ++v) sc->dots[v] = red[v];
    if (step == STEP_PROJECT) {
        for (int j = 0; j < nv; ++j) {
            const double in = sc->inv_nu[j0 + j];
            const double2 beta = make_double2(red[j].x * in, red[j].y * in);
            sc->R[j0 + j][k] = beta;
            sc->coef[j0 + j] = make_double2(beta.x * in, beta.y * in);
        }
    } else if (step == STEP_NORM) {
        const double r2 = red[0].x;
        sc->rnorm2 = r2;
        tails[r].rnorm2 = r2;
        sc->inv_rnorm = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
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

// Scale of the low-precision residual copy: 1 / |r| of the residual before
// this update (the preconditioner is homogeneous, so any positive scale gives
// the same direction; this one keeps the copy near unit norm).
__device__ __forceinline__ double lo_scale(const GcrScalars& S) {
    return S.inv_rnorm > 0.0 ? S.inv_rnorm : 1.0;
}

// |v|^2; optionally also writes lo_scale * v in precision PL to lo (PL < 0: no copy)
template <int PL>
__global__ __launch_bounds__(TPB) void k_norm2_f64(Geom g, const void* v, size_t fs, void* lo, size_t ls,
                                                   const GcrScalars* sc, const int* active, double2* partials) {
    if (skip(active)) return;
    const char* q = (const char*)v + blockIdx.y * fs;
    double sl = 1.0;
    if constexpr (PL >= 0) sl = lo_scale(sc[blockIdx.y]);
    cpx<double> acc[1] = {{0.0, 0.0}};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> c[12];
        ld64<P_F64>(q, g.nblk, blk, threadIdx.x, c);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[0].re += c[k].re * c[k].re + c[k].im * c[k].im;
        if constexpr (PL >= 0) {
#pragma unroll
            for (int k = 0; k < 12; ++k) c[k] = sl * c[k];
            st64<PL>((char*)lo + blockIdx.y * ls, g.nblk, blk, threadIdx.x, c);
        }
    }
    wg_reduce_store<1>(acc, 1, partials, NORM_SLOT);
}

// Basis vectors whose loads are issued together: enough to keep several
// loads of a lane in flight, few enough to stay in registers.
template <int P>
constexpr int load_group() {
    return sizeof(typename SpinorIO<P>::R) == 8 ? 2 : 4;
}

template <typename R>
__device__ __forceinline__ cpx<double> to64(cpx<R> a) {
    return {(double)a.re, (double)a.im};
}

// partial <W_{j0 + j}, W_k> for j < n (n <= MULTIDOT_CHUNK); W stored [k][rhs].
// The vectors are read in groups whose loads are all issued before any is
// used; inside the last group, indices past n repeat vector n - 1 and their
// sums are never stored.
// Dots handled by one multi-dot pass: MULTIDOT_CHUNK, or half of it for a
// 16-bit basis (whose pass keeps all of its vectors' packed words in flight)
template <int PB>
constexpr int multidot_chunk() {
    return PB == P_F16 || PB == P_BF16 ? MULTIDOT_CHUNK / 2 : MULTIDOT_CHUNK;
}

template <int PB>
__global__ __launch_bounds__(TPB) void k_multidot(Geom g, const char* W, size_t ws, int nrhs, int j0, int n,
                                                  int k, const int* active, double2* partials) {
    if (skip(active)) return;
    using RS = typename SpinorIO<PB>::R;
    constexpr int G = load_group<PB>();
    constexpr int CH = multidot_chunk<PB>();
    const int r = blockIdx.y;
    const char* base = W + (size_t)r * ws;
    const size_t vs = (size_t)nrhs * ws;  // from one basis vector to the next
    cpx<double> acc[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) acc[j] = {0.0, 0.0};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<RS> v[12];
        SpinorIO<PB>::load(base + (size_t)k * vs, g.nblk, blk, threadIdx.x, v);
        if constexpr (PB == P_F16 || PB == P_BF16) {
            // 16-bit basis: the packed words of all CH vectors in flight at
            // once (the bytes of four FP32 vectors), unpacked one at a time
            typename SpinorIO16<PB>::Raw raw[CH];
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const int j = q < n ? q : n - 1;
                SpinorIO16<PB>::load_raw(base + (size_t)(j0 + j) * vs, g.nblk, blk, threadIdx.x, raw[q]);
            }
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                if (q < n) {
                    cpx<float> t[12];
                    SpinorIO16<PB>::unpack(raw[q], t);
#pragma unroll
                    for (int c = 0; c < 12; ++c) cmac_conj(acc[q], to64(t[c]), to64(v[c]));
                }
            }
        } else {
#pragma unroll
            for (int jb = 0; jb < CH; jb += G) {
                if (jb < n) {
                    cpx<RS> t[G][12];
#pragma unroll
                    for (int q = 0; q < G; ++q) {
                        const int j = jb + q < n ? jb + q : n - 1;
                        SpinorIO<PB>::load(base + (size_t)(j0 + j) * vs, g.nblk, blk, threadIdx.x, t[q]);
                    }
#pragma unroll
                    for (int q = 0; q < G; ++q)
#pragma unroll
                        for (int c = 0; c < 12; ++c) cmac_conj(acc[jb + q], to64(t[q][c]), to64(v[c]));
                }
            }
        }
    }
    wg_reduce_store<CH>(acc, n, partials);
}

// W_k -= sum_{j<k} coef_j W_j (in increasing j, loads issued a group at a
// time); partials |W_k|^2 and <W_k, r>
template <int PB>
__global__ __launch_bounds__(TPB) void k_ortho(Geom g, char* W, size_t ws, int nrhs, int k, const void* rv,
                                               size_t rs, const GcrScalars* sc, const int* active,
                                               double2* partials) {
    if (skip(active)) return;
    using RS = typename SpinorIO<PB>::R;
    constexpr int G = load_group<PB>();
    const int r = blockIdx.y;
    const GcrScalars* S = sc + r;
    const char* rr_base = (const char*)rv + r * rs;
    char* base = W + (size_t)r * ws;
    const size_t vs = (size_t)nrhs * ws;
    cpx<double> acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> v[12], rr[12];
        ld64<PB>(base + (size_t)k * vs, g.nblk, blk, threadIdx.x, v);
        ld64<P_F64>(rr_base, g.nblk, blk, threadIdx.x, rr);
        for (int jb = 0; jb < k; jb += G) {
            cpx<RS> t[G][12];
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const int j = jb + q < k ? jb + q : k - 1;
                SpinorIO<PB>::load(base + (size_t)j * vs, g.nblk, blk, threadIdx.x, t[q]);
            }
#pragma unroll
            for (int q = 0; q < G; ++q) {
                if (jb + q < k) {
                    const cpx<double> cf = {S->coef[jb + q].x, S->coef[jb + q].y};
#pragma unroll
                    for (int c = 0; c < 12; ++c) v[c] = v[c] - cf * to64(t[q][c]);
                }
            }
        }
        if (k > 0) st64<PB>(base + (size_t)k * vs, g.nblk, blk, threadIdx.x, v);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            acc[0].re += v[c].re * v[c].re + v[c].im * v[c].im;
            cmac_conj(acc[1], v[c], rr[c]);
        }
    }
    wg_reduce_store<2>(acc, 2, partials);
}

// Completes the orthonormalisation step from its partials (every workgroup
// sums them in the same fixed order; workgroup 0 stores nu_k, c_k, R[k][k]),
// then r -= (c_k / nu_k) W_k, partial |r|^2 and optionally
// lo_scale * (new r) in precision PL to lo.
template <int PB, int PL>
__global__ __launch_bounds__(TPB) void k_residual_update(Geom g, const char* W, size_t ws, int nrhs, int k,
                                                         void* rv, size_t rs, void* lo, size_t los,
                                                         GcrScalars* sc, GcrTail* tails, const int* active,
                                                         double2* partials, int nwg) {
    if (skip(active)) return;
    const int r = blockIdx.y;
    __shared__ double2 red[TPB];
    sum_partials<2, TPB>(partials + (size_t)r * BLAS_MAX_WG * NVS, nwg, 0, red);
    const OrthoScalars o = ortho_scalars(red[0], red[1]);
    double sl = 1.0;
    if constexpr (PL >= 0) sl = lo_scale(sc[r]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        GcrScalars* S = sc + r;
        S->dots[0] = red[0];
        S->dots[1] = red[1];
        S->nu = o.nu;
        tails[r].nu = o.nu;
        S->R[k][k] = make_double2(o.nu, 0.0);
        S->inv_nu[k] = o.inv_nu;
        S->c[k] = o.ck;
        S->coef[0] = o.coef;
    }
    const cpx<double> cf = {o.coef.x, o.coef.y};
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
        if constexpr (PL >= 0) {
#pragma unroll
            for (int c = 0; c < 12; ++c) rr[c] = sl * rr[c];
            st64<PL>((char*)lo + r * los, g.nblk, blk, threadIdx.x, rr);
        }
    }
    wg_reduce_store<1>(acc, 1, partials, NORM_SLOT);
}

// x += sum_{j < nk} gamma_j Z_j
// x += sum_{j < nk} gamma_j Z_j.  Every workgroup first solves the
// triangular system R gamma = c over the first nk directions (R[k][k] = nu_k
// is real) in the same order, so all use the same gamma.
template <int PZ>
__global__ __launch_bounds__(TPB) void k_solution_update(Geom g, const char* Z, size_t zs, int nrhs, void* xv,
                                                         size_t xs, const GcrScalars* sc, const int* ku) {
    const int r = blockIdx.y;
    const GcrScalars* S = sc + r;
    __shared__ double2 gam[GCR_MAX_RESTART], cs[GCR_MAX_RESTART], Rs[GCR_MAX_RESTART][GCR_MAX_RESTART];
    __shared__ int nks;
    if (threadIdx.x == 0) nks = ku[r];
    __syncthreads();
    const int nk = nks;
    if (nk <= 0) return;
    // R and c to LDS with all lanes, then one lane solves from LDS
    for (int i = threadIdx.x; i < nk * nk; i += TPB) Rs[i / nk][i % nk] = S->R[i / nk][i % nk];
    if ((int)threadIdx.x < nk) cs[threadIdx.x] = S->c[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = nk - 1; k >= 0; --k) {
            double2 acc = cs[k];
            for (int j = k + 1; j < nk; ++j) {
                const double2 a = Rs[k][j], b = gam[j];
                acc.x -= a.x * b.x - a.y * b.y;
                acc.y -= a.x * b.y + a.y * b.x;
            }
            const double nu = Rs[k][k].x;
            gam[k] = make_double2(acc.x / nu, acc.y / nu);
        }
    }
    __syncthreads();
    char* x_base = (char*)xv + r * xs;
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> xx[12];
        ld64<P_F64>(x_base, g.nblk, blk, threadIdx.x, xx);
        for (int j = 0; j < nk; ++j) {
            const cpx<double> gm = {gam[j].x, gam[j].y};
            cpx<double> z[12];
            ld64<PZ>(Z + ((size_t)j * nrhs + r) * zs, g.nblk, blk, threadIdx.x, z);
#pragma unroll
            for (int c = 0; c < 12; ++c) cmac(xx[c], gm, z[c]);
        }
        st64<P_F64>(x_base, g.nblk, blk, threadIdx.x, xx);
    }
}


// ------------------------------------------------------------- BiCGStab

enum BiStep { BI_ALPHA = 1, BI_OMEGA = 2, BI_RHO = 3, BI_RESTART = 4, BI_NORM = 5 };

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Vectors of the iteration are stored in precision PV (FP64, or FP32 for
// the single-precision inner solve of the Richardson form); arithmetic and
// reductions are FP64 either way.
template <int PV, int PI>
__global__ __launch_bounds__(TPB) void k_bi_p(Geom g, const BiScalars* sc, BiFields f) {
    const cpx<double> beta = {sc->beta.x, sc->beta.y}, omega = {sc->omega.x, sc->omega.y};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> r[12], p[12], v[12];
        ld64<PV>(f.r, g.nblk, blk, threadIdx.x, r);
        ld64<PV>(f.p, g.nblk, blk, threadIdx.x, p);
        ld64<PV>(f.v, g.nblk, blk, threadIdx.x, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) p[k] = r[k] + beta * (p[k] - omega * v[k]);
        st64<PV>(f.p, g.nblk, blk, threadIdx.x, p);
        st64<PI>(f.plo, g.nblk, blk, threadIdx.x, p);
    }
}

// dst = w (precision PW) stored in PV; partials <a, dst> (slot 0) or, with
// TWO, <dst, b2> (slot 0) and |dst|^2 (slot 1)
template <int PW, bool TWO, int PV>
__global__ __launch_bounds__(TPB) void k_bi_take(Geom g, const BiScalars* sc, const void* w, void* dst,
                                                 const void* a, const void* b2, double2* partials) {
    if (sc->flag & 1) return;
    cpx<double> acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> v[12];
        ld64<PW>(w, g.nblk, blk, threadIdx.x, v);
        if constexpr (PV != PW) {
            st64<PV>(dst, g.nblk, blk, threadIdx.x, v);
            ld64<PV>(dst, g.nblk, blk, threadIdx.x, v);  // the value every later use sees
        } else {
            st64<PV>(dst, g.nblk, blk, threadIdx.x, v);
        }
        cpx<double> o[12];
        if (TWO) {
            ld64<PV>(b2, g.nblk, blk, threadIdx.x, o);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                cmac_conj(acc[0], v[k], o[k]);
                acc[1].re += v[k].re * v[k].re + v[k].im * v[k].im;
            }
        } else {
            ld64<PV>(a, g.nblk, blk, threadIdx.x, o);
#pragma unroll
            for (int k = 0; k < 12; ++k) cmac_conj(acc[0], o[k], v[k]);
        }
    }
    wg_reduce_store<2>(acc, TWO ? 2 : 1, partials);
}

template <int PV, int PI>
__global__ __launch_bounds__(TPB) void k_bi_s(Geom g, const BiScalars* sc, BiFields f) {
    if (sc->flag & 1) return;
    const cpx<double> alpha = {sc->alpha.x, sc->alpha.y};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> r[12], v[12];
        ld64<PV>(f.r, g.nblk, blk, threadIdx.x, r);
        ld64<PV>(f.v, g.nblk, blk, threadIdx.x, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) r[k] = r[k] - alpha * v[k];
        st64<PV>(f.s, g.nblk, blk, threadIdx.x, r);
        st64<PI>(f.slo, g.nblk, blk, threadIdx.x, r);
    }
}

template <int PV, int PI>
__global__ __launch_bounds__(TPB) void k_bi_xr(Geom g, const BiScalars* sc, BiFields f, double2* partials) {
    if (sc->flag & 1) return;
    const cpx<double> alpha = {sc->alpha.x, sc->alpha.y}, omega = {sc->omega.x, sc->omega.y};
    cpx<double> acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> x[12], zp[12], zs[12];
        ld64<PV>(f.x, g.nblk, blk, threadIdx.x, x);
        ld64<PI>(f.zp, g.nblk, blk, threadIdx.x, zp);
        ld64<PI>(f.zs, g.nblk, blk, threadIdx.x, zs);
#pragma unroll
        for (int k = 0; k < 12; ++k) x[k] = x[k] + alpha * zp[k] + omega * zs[k];
        st64<PV>(f.x, g.nblk, blk, threadIdx.x, x);
        cpx<double> s[12], t[12], rh[12];
        ld64<PV>(f.s, g.nblk, blk, threadIdx.x, s);
        ld64<PV>(f.t, g.nblk, blk, threadIdx.x, t);
        ld64<PV>(f.rh, g.nblk, blk, threadIdx.x, rh);
#pragma unroll
        for (int k = 0; k < 12; ++k) s[k] = s[k] - omega * t[k];
        st64<PV>(f.r, g.nblk, blk, threadIdx.x, s);
        if constexpr (PV != P_F64) ld64<PV>(f.r, g.nblk, blk, threadIdx.x, s);  // the stored residual
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            cmac_conj(acc[0], rh[k], s[k]);
            acc[1].re += s[k].re * s[k].re + s[k].im * s[k].im;
        }
    }
    wg_reduce_store<2>(acc, 2, partials);
}

// rh = r; partial |r|^2 (slot 0)
template <int PV>
__global__ __launch_bounds__(TPB) void k_bi_restart(Geom g, BiFields f, double2* partials) {
    cpx<double> acc[1] = {{0.0, 0.0}};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> r[12];
        ld64<PV>(f.r, g.nblk, blk, threadIdx.x, r);
        st64<PV>(f.rh, g.nblk, blk, threadIdx.x, r);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[0].re += r[k].re * r[k].re + r[k].im * r[k].im;
    }
    wg_reduce_store<1>(acc, 1, partials);
}

template <int PV>
__global__ __launch_bounds__(TPB) void k_bi_norm2(Geom g, const void* v, double2* partials) {
    cpx<double> acc[1] = {{0.0, 0.0}};
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> r[12];
        ld64<PV>(v, g.nblk, blk, threadIdx.x, r);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[0].re += r[k].re * r[k].re + r[k].im * r[k].im;
    }
    wg_reduce_store<1>(acc, 1, partials);
}

// dst (F32) = scale * src (F64)
__global__ __launch_bounds__(TPB) void k_bi_demote(Geom g, const void* src, void* dst, double scale) {
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> v[12];
        ld64<P_F64>(src, g.nblk, blk, threadIdx.x, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = scale * v[k];
        st64<P_F32>(dst, g.nblk, blk, threadIdx.x, v);
    }
}

// x (F64) += scale * e (F32)
__global__ __launch_bounds__(TPB) void k_bi_promote_add(Geom g, void* x, const void* e, double scale) {
    for (int blk = blockIdx.x; blk < g.nblk; blk += gridDim.x) {
        cpx<double> xv[12], ev[12];
        ld64<P_F64>(x, g.nblk, blk, threadIdx.x, xv);
        ld64<P_F32>(e, g.nblk, blk, threadIdx.x, ev);
#pragma unroll
        for (int k = 0; k < 12; ++k) xv[k] = xv[k] + scale * ev[k];
        st64<P_F64>(x, g.nblk, blk, threadIdx.x, xv);
    }
}

__global__ __launch_bounds__(FIN_TPB) void k_bi_finalize(const double2* partials, int nwg, BiScalars* sc,
                                                         BiTail* tail, int step) {
    if ((sc->flag & 1) && step != BI_RESTART && step != BI_NORM) {
        // an abandoned iteration: x and r are unchanged, the host restarts
        if (step == BI_RHO && threadIdx.x == 0) {
            tail->rr = sc->rr;
            tail->flag = sc->flag;
        }
        return;
    }
    __shared__ double2 red[FIN_TPB];
    sum_partials<2, FIN_TPB>(partials, nwg, 0, red);
    if (threadIdx.x != 0) return;
    const double2 d0 = red[0], d1 = red[1];
    if (step == BI_ALPHA) {
        if (d0.x == 0.0 && d0.y == 0.0) {
            sc->flag = 1;
            sc->alpha = make_double2(0.0, 0.0);
        } else {
            sc->alpha = cdiv(sc->rho, d0);
        }
    } else if (step == BI_OMEGA) {
        if (d1.x > 0.0) {
            sc->omega = make_double2(d0.x / d1.x, d0.y / d1.x);
        } else {
            sc->omega = make_double2(0.0, 0.0);
            sc->flag |= 2;
        }
        if (sc->omega.x == 0.0 && sc->omega.y == 0.0) sc->flag |= 2;
    } else if (step == BI_RHO) {
        const double2 rho_new = d0;
        if (sc->flag & 2) sc->beta = make_double2(0.0, 0.0);
        else sc->beta = cmul2(cdiv(rho_new, sc->rho), cdiv(sc->alpha, sc->omega));
        sc->rho = rho_new;
        sc->rr = d1.x;
        tail->rr = d1.x;
        tail->flag = sc->flag;
    } else if (step == BI_RESTART) {
        sc->rho = make_double2(d0.x, 0.0);
        sc->rr = d0.x;
        sc->alpha = sc->omega = make_double2(1.0, 0.0);
        sc->beta = make_double2(0.0, 0.0);
        sc->flag = 0;
        tail->rr = d0.x;
        tail->flag = 0;
    } else {  // BI_NORM
        tail->rr = d0.x;
        tail->flag = 0;
    }
}

int nwg_for(const Geom& g) { return g.nblk < BLAS_MAX_WG ? g.nblk : BLAS_MAX_WG; }

hipError_t finalize(const BlasCtx& c, int nv, int v0, int step, int k, int j0, hipStream_t s) {
    const int nwg = nwg_for(c.g);
    if (nv == 1)
        hipLaunchKernelGGL((k_finalize<1>), dim3(c.nrhs), dim3(FIN_TPB), 0, s, c.partials, nwg, nv, v0, c.sc,
                           c.tail, c.active, step, k, j0);
    else
        hipLaunchKernelGGL((k_finalize<MULTIDOT_CHUNK>), dim3(c.nrhs), dim3(FIN_TPB), 0, s, c.partials, nwg, nv,
                           v0, c.sc, c.tail, c.active, step, k, j0);
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

hipError_t blas_norm_to_scalars(const BlasCtx& c, const void* v, int lo_prec, void* lo, hipStream_t s) {
    ProfScope ps("blas", s);
    const dim3 grid(nwg_for(c.g), c.nrhs);
    const size_t ls = lo_prec >= 0 ? spinor_bytes_per_site(lo_prec) * c.g.V : 0;
    if (lo_prec < 0) {
        hipLaunchKernelGGL((k_norm2_f64<-1>), grid, dim3(TPB), 0, s, c.g, v, f64_stride(c.g), lo, ls, c.sc, c.active, c.partials);
    } else {
        CS_DISPATCH_P(lo_prec, hipLaunchKernelGGL((k_norm2_f64<PP>), grid, dim3(TPB), 0, s, c.g, v, f64_stride(c.g), lo, ls, c.sc, c.active, c.partials));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(c, 1, NORM_SLOT, STEP_NORM, 0, 0, s);
}

hipError_t blas_gcr_project(const BlasCtx& c, int pb, const void* W, size_t ws, int k, hipStream_t s) {
    ProfScope ps("blas", s);
    const int chunk = pb == P_F16 || pb == P_BF16 ? MULTIDOT_CHUNK / 2 : MULTIDOT_CHUNK;
    for (int j0 = 0; j0 < k; j0 += chunk) {
        const int n = k - j0 < chunk ? k - j0 : chunk;
        const dim3 grid(nwg_for(c.g), c.nrhs);
        CS_DISPATCH_P(pb, hipLaunchKernelGGL((k_multidot<PP>), grid, dim3(TPB), 0, s, c.g, (const char*)W, ws, c.nrhs, j0, n, k, c.active, c.partials));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = finalize(c, n, 0, STEP_PROJECT, k, j0, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t blas_gcr_orthonormalise(const BlasCtx& c, int pb, void* W, size_t ws, int k, const void* r,
                                   hipStream_t s) {
    ProfScope ps("blas", s);
    const dim3 grid(nwg_for(c.g), c.nrhs);
    CS_DISPATCH_P(pb, hipLaunchKernelGGL((k_ortho<PP>), grid, dim3(TPB), 0, s, c.g, (char*)W, ws, c.nrhs, k, r, f64_stride(c.g), c.sc, c.active, c.partials));
    return hipGetLastError();
}

hipError_t blas_gcr_residual_update(const BlasCtx& c, int pb, const void* W, size_t ws, int k, void* r,
                                    int lo_prec, void* lo, hipStream_t s) {
    ProfScope ps("blas", s);
    const dim3 grid(nwg_for(c.g), c.nrhs);
    const size_t los = lo_prec >= 0 ? spinor_bytes_per_site(lo_prec) * c.g.V : 0;
    hipError_t e = hipSuccess;
    auto go = [&](auto pbt, auto plt) {
        constexpr int PB = decltype(pbt)::value, PL = decltype(plt)::value;
        hipLaunchKernelGGL((k_residual_update<PB, PL>), grid, dim3(TPB), 0, s, c.g, (const char*)W, ws, c.nrhs, k, r,
                           f64_stride(c.g), lo, los, c.sc, c.tail, c.active, c.partials, nwg_for(c.g));
        e = hipGetLastError();
    };
    auto with_lo = [&](auto pbt) {
        switch (lo_prec) {
        case -1: go(pbt, std::integral_constant<int, -1>{}); break;
        case P_F64: go(pbt, std::integral_constant<int, P_F64>{}); break;
        case P_F32: go(pbt, std::integral_constant<int, P_F32>{}); break;
        case P_F16: go(pbt, std::integral_constant<int, P_F16>{}); break;
        case P_BF16: go(pbt, std::integral_constant<int, P_BF16>{}); break;
        default: e = hipErrorInvalidValue;
        }
    };
    switch (pb) {
    case P_F64: with_lo(std::integral_constant<int, P_F64>{}); break;
    case P_F32: with_lo(std::integral_constant<int, P_F32>{}); break;
    case P_F16: with_lo(std::integral_constant<int, P_F16>{}); break;
    case P_BF16: with_lo(std::integral_constant<int, P_BF16>{}); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return finalize(c, 1, NORM_SLOT, STEP_NORM, 0, 0, s);
}

hipError_t blas_gcr_solution_update(const BlasCtx& c, int pz, const void* Z, size_t zs, void* x, const int* ku,
                                    hipStream_t s) {
    ProfScope ps("blas", s);
    const dim3 grid(nwg_for(c.g), c.nrhs);
    CS_DISPATCH_P(pz, hipLaunchKernelGGL((k_solution_update<PP>), grid, dim3(TPB), 0, s, c.g, (const char*)Z, zs, c.nrhs, x, f64_stride(c.g), c.sc, ku));
    return hipGetLastError();
}


// ------------------------------------------------------------- BiCGStab

static hipError_t bi_fin(const BlasCtx& c, BiScalars* sc, BiTail* tail, int step, hipStream_t s) {
    hipLaunchKernelGGL(k_bi_finalize, dim3(1), dim3(FIN_TPB), 0, s, c.partials, nwg_for(c.g), sc, tail, step);
    return hipGetLastError();
}

// Calls f(integral_constant<PV>, integral_constant<PI>) for the supported
// vector precisions (F64, F32) and inner precisions.
template <class F>
static hipError_t with_pv_pi(int pv, int pi, F f) {
    auto inner = [&](auto pvt) -> hipError_t {
        switch (pi) {
        case P_F64: return f(pvt, std::integral_constant<int, P_F64>{});
        case P_F32: return f(pvt, std::integral_constant<int, P_F32>{});
        case P_F16: return f(pvt, std::integral_constant<int, P_F16>{});
        case P_BF16: return f(pvt, std::integral_constant<int, P_BF16>{});
        default: return hipErrorInvalidValue;
        }
    };
    switch (pv) {
    case P_F64: return inner(std::integral_constant<int, P_F64>{});
    case P_F32: return inner(std::integral_constant<int, P_F32>{});
    default: return hipErrorInvalidValue;
    }
}

template <class F>
static hipError_t with_pv(int pv, F f) {
    switch (pv) {
    case P_F64: return f(std::integral_constant<int, P_F64>{});
    case P_F32: return f(std::integral_constant<int, P_F32>{});
    default: return hipErrorInvalidValue;
    }
}

hipError_t bicg_update_p(const BlasCtx& c, const BiScalars* sc, const BiFields& f, int pv, int pi, hipStream_t s) {
    ProfScope ps("blas", s);
    return with_pv_pi(pv, pi, [&](auto a, auto b) {
        hipLaunchKernelGGL((k_bi_p<decltype(a)::value, decltype(b)::value>), dim3(nwg_for(c.g)), dim3(TPB), 0, s,
                           c.g, sc, f);
        return hipGetLastError();
    });
}

hipError_t bicg_alpha(const BlasCtx& c, BiScalars* sc, const BiFields& f, int pv, int pw, hipStream_t s) {
    ProfScope ps("blas", s);
    hipError_t e = with_pv_pi(pv, pw, [&](auto a, auto b) {
        constexpr int PV = decltype(a)::value, PW = decltype(b)::value;
        if constexpr (PW != P_F64 && PW != P_F32) {
            return hipErrorInvalidValue;
        } else {
            hipLaunchKernelGGL((k_bi_take<PW, false, PV>), dim3(nwg_for(c.g)), dim3(TPB), 0, s, c.g, sc, f.w, f.v,
                               f.rh, nullptr, c.partials);
            return hipGetLastError();
        }
    });
    if (e != hipSuccess) return e;
    return bi_fin(c, sc, nullptr, BI_ALPHA, s);
}

hipError_t bicg_update_s(const BlasCtx& c, const BiScalars* sc, const BiFields& f, int pv, int pi, hipStream_t s) {
    ProfScope ps("blas", s);
    return with_pv_pi(pv, pi, [&](auto a, auto b) {
        hipLaunchKernelGGL((k_bi_s<decltype(a)::value, decltype(b)::value>), dim3(nwg_for(c.g)), dim3(TPB), 0, s,
                           c.g, sc, f);
        return hipGetLastError();
    });
}

hipError_t bicg_omega(const BlasCtx& c, BiScalars* sc, const BiFields& f, int pv, int pw, hipStream_t s) {
    ProfScope ps("blas", s);
    hipError_t e = with_pv_pi(pv, pw, [&](auto a, auto b) {
        constexpr int PV = decltype(a)::value, PW = decltype(b)::value;
        if constexpr (PW != P_F64 && PW != P_F32) {
            return hipErrorInvalidValue;
        } else {
            hipLaunchKernelGGL((k_bi_take<PW, true, PV>), dim3(nwg_for(c.g)), dim3(TPB), 0, s, c.g, sc, f.w, f.t,
                               nullptr, f.s, c.partials);
            return hipGetLastError();
        }
    });
    if (e != hipSuccess) return e;
    return bi_fin(c, sc, nullptr, BI_OMEGA, s);
}

hipError_t bicg_update_xr(const BlasCtx& c, BiScalars* sc, BiTail* tail, const BiFields& f, int pv, int pi,
                          hipStream_t s) {
    ProfScope ps("blas", s);
    hipError_t e = with_pv_pi(pv, pi, [&](auto a, auto b) {
        hipLaunchKernelGGL((k_bi_xr<decltype(a)::value, decltype(b)::value>), dim3(nwg_for(c.g)), dim3(TPB), 0, s,
                           c.g, sc, f, c.partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    return bi_fin(c, sc, tail, BI_RHO, s);
}

hipError_t bicg_restart(const BlasCtx& c, BiScalars* sc, BiTail* tail, const BiFields& f, int pv, hipStream_t s) {
    ProfScope ps("blas", s);
    hipError_t e = with_pv(pv, [&](auto a) {
        hipLaunchKernelGGL((k_bi_restart<decltype(a)::value>), dim3(nwg_for(c.g)), dim3(TPB), 0, s, c.g, f,
                           c.partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    return bi_fin(c, sc, tail, BI_RESTART, s);
}

hipError_t bicg_norm2(const BlasCtx& c, BiScalars* sc, BiTail* tail, const void* v, int pv, hipStream_t s) {
    ProfScope ps("blas", s);
    hipError_t e = with_pv(pv, [&](auto a) {
        hipLaunchKernelGGL((k_bi_norm2<decltype(a)::value>), dim3(nwg_for(c.g)), dim3(TPB), 0, s, c.g, v,
                           c.partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    return bi_fin(c, sc, tail, BI_NORM, s);
}

hipError_t bicg_demote(const BlasCtx& c, const void* src64, void* dst32, double scale, hipStream_t s) {
    ProfScope ps("blas", s);
    hipLaunchKernelGGL(k_bi_demote, dim3(nwg_for(c.g)), dim3(TPB), 0, s, c.g, src64, dst32, scale);
    return hipGetLastError();
}

hipError_t bicg_promote_add(const BlasCtx& c, void* x64, const void* e32, double scale, hipStream_t s) {
    ProfScope ps("blas", s);
    hipLaunchKernelGGL(k_bi_promote_add, dim3(nwg_for(c.g)), dim3(TPB), 0, s, c.g, x64, e32, scale);
    return hipGetLastError();
}

// ------------------------------------------------------- bandwidth reference

// dst = src over n 16-byte words: a plain streaming copy, the measured
// bandwidth reference for the field kernels.  One word per lane and one
// launch-wide pass (no grid-stride loop): on MI355X this pattern copies
// faster than a persistent grid that keeps several loads in flight per lane.
__global__ __launch_bounds__(TPB) void k_stream_copy(float4* __restrict__ dst, const float4* __restrict__ src,
                                                     size_t n) {
    const size_t i = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
    ProfScope ps("copy", s);
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    const size_t wgs = (n + TPB - 1) / TPB;
    if (wgs > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)wgs), dim3(TPB), 0, s, (float4*)dst, (const float4*)src, n);
    return hipGetLastError();
}

}  // namespace cs
