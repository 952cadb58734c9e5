// Two-level multigrid pieces of the paper's Section 3 (FP32 storage and
// arithmetic; reductions in FP64 where a result feeds a solver scalar).
//
// Aggregates are the 4^4 SAP blocks (one workgroup, one lane per site).  A
// coarse site carries nc = 2 nv values, index c = chi * nv + i, chi the
// chirality (spins 0, 1 / spins 2, 3).  The prolongator P is stored as nv FP32
// spinor fields: field i holds p_{a,chi,i} on every aggregate a and chirality
// chi.  Coarse vectors are float2[nblk][nc]; the coarse operator
// D_c = P^dag D P is a 9-point stencil float2[nblk][9][nc (column)][nc (row)],
// direction d = 0 the aggregate itself, 1 + 2 mu its +mu neighbour, 2 + 2 mu
// its -mu neighbour (entries that reach the same aggregate through different
// faces stay separate, so the stencil is exact on any lattice).
#include "blas.hpp"
#include "dslash_core.hpp"
#include "mg.hpp"

namespace cs {

namespace {

constexpr int TPB = BLOCK_SITES;

__device__ __forceinline__ float wsum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sum N values over the workgroup; afterwards out[k] (LDS) holds total k.
template <int N>
__device__ __forceinline__ void block_sum(const float* v, float (*red)[N], float* out) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const float s = wsum(v[k]);
        if (lane == 0) red[wave][k] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < N) {
        const int k = threadIdx.x;
        out[k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
    }
    __syncthreads();
}

__device__ __forceinline__ void load_f32(const char* P, size_t fs, int i, int nblk, int blk, int l, cpx<float>* c) {
    SpinorIO<P_F32>::load(P + (size_t)i * fs, nblk, blk, l, c);
}

// Block index one step in direction mu (dir = +1 / -1) with periodic wrap.
__device__ __forceinline__ int block_step(const Geom& g, const BlockPos& p, int mu, int dir) {
    const int bc = mu == 0 ? p.bc[0] : mu == 1 ? p.bc[1] : mu == 2 ? p.bc[2] : p.bc[3];
    const int nb = mu == 0 ? g.NB[0] : mu == 1 ? g.NB[1] : mu == 2 ? g.NB[2] : g.NB[3];
    const int st = mu == 0 ? p.stride[0] : mu == 1 ? p.stride[1] : mu == 2 ? p.stride[2] : p.stride[3];
    if (dir > 0) return bc == nb - 1 ? p.blk - (nb - 1) * st : p.blk + st;
    return bc == 0 ? p.blk + (nb - 1) * st : p.blk - st;
}

// ---------------------------------------------------------------- setup

// Modified Gram-Schmidt of the nv fields per aggregate and chirality, in place.
__global__ __launch_bounds__(TPB) void k_mg_orthonormalize(Geom g, char* P, size_t fs, int nv) {
    const int blk = blockIdx.x, l = threadIdx.x;
    __shared__ float red[4][4];
    __shared__ float tot[4];
    for (int i = 0; i < nv; ++i) {
        cpx<float> v[12];
        load_f32(P, fs, i, g.nblk, blk, l, v);
        for (int j = 0; j < i; ++j) {
            cpx<float> q[12];
            load_f32(P, fs, j, g.nblk, blk, l, q);
            float d[4] = {0.f, 0.f, 0.f, 0.f};  // <q, v> per chirality (re, im)
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const int o = k < 6 ? 0 : 2;
                d[o] += q[k].re * v[k].re + q[k].im * v[k].im;
                d[o + 1] += q[k].re * v[k].im - q[k].im * v[k].re;
            }
            block_sum<4>(d, red, tot);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const int o = k < 6 ? 0 : 2;
                const cpx<float> c = {tot[o], tot[o + 1]};
                v[k] = v[k] - c * q[k];
            }
        }
        float n[2] = {0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 12; ++k) n[k < 6 ? 0 : 1] += v[k].re * v[k].re + v[k].im * v[k].im;
        float nn[4] = {n[0], n[1], 0.f, 0.f};
        block_sum<4>(nn, red, tot);
        const float s0 = tot[0] > 0.f ? 1.f / sqrtf(tot[0]) : 0.f, s1 = tot[1] > 0.f ? 1.f / sqrtf(tot[1]) : 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = (k < 6 ? s0 : s1) * v[k];
        SpinorIO<P_F32>::store(P + (size_t)i * fs, g.nblk, blk, l, v);
        __syncthreads();  // the next i reads the stored field
    }
}

// Column (chi_c, j) of P on one site: field j with the other chirality zeroed.
__device__ __forceinline__ void column_site(const char* P, size_t fs, int nv, int col, int nblk, int blk, int l,
                                            cpx<float>* c) {
    const int chi = col / nv, j = col % nv;
    load_f32(P, fs, j, nblk, blk, l, c);
#pragma unroll
    for (int k = 0; k < 12; ++k)
        if ((k < 6 ? 0 : 1) != chi) c[k] = {0.f, 0.f};
}

struct LdsColumn {  // in-block neighbours for the self term
    const cpx<float> (*s)[BLOCK_SITES];
    __device__ __forceinline__ bool want(bool inside) const { return inside; }
    template <typename R>
    __device__ __forceinline__ void load_nb(int, int l, bool, cpx<R>* c) const {
#pragma unroll
        for (int k = 0; k < 12; ++k) c[k] = s[k][l];
    }
};

// Hop term of direction MU, sign S (forward -1 / backward +1), for the lanes
// whose neighbour lies in the adjacent aggregate: acc += that hop of column col
// of P on the neighbouring aggregate.
template <int MU, int S>
__device__ __forceinline__ void face_term(const Geom& g, const BlockPos& p, int l, const void* links,
                                          const char* P, size_t fs, int nv, int col, cpx<float>* acc) {
    int nl;
    bool in;
    const int nb = neighbour(g, p, l, MU, S < 0 ? +1 : -1, &nl, &in);
    if (in) return;
    cpx<float> psi[12], u[9];
    column_site(P, fs, nv, col, g.nblk, nb, nl, psi);
    if (S < 0) load_link<P_F32, float, false>(links, p.blk, l, MU, u);  // U_mu(x)
    else load_link<P_F32, float, false>(links, nb, nl, MU, u);          // U_mu(x - mu)
    hop_term<MU, S>(u, psi, acc);
}

// D_c[a][d][col][row] = <p_{a,row}, D p_{n(a,d),col}> restricted to the
// terms of D that couple aggregate a to its neighbour in direction d.
__global__ __launch_bounds__(TPB) void k_mg_assemble(Geom g, const void* links, const void* clover, float kappa,
                                                     const char* P, size_t fs, int nv, float2* Dc) {
    const int blk = blockIdx.x, d = blockIdx.y, l = threadIdx.x, nc = 2 * nv;
    const BlockPos p = block_pos(g, blk);
    __shared__ cpx<float> s[12][BLOCK_SITES];
    __shared__ float red[4][8];
    __shared__ float tot[8];
    float cl[72];
    if (d == 0) CloverIO<float>::template load<false>(clover, blk, l, cl);
    for (int col = 0; col < nc; ++col) {
        cpx<float> w[12], acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {0.f, 0.f};
        if (d == 0) {
            cpx<float> c[12];
            column_site(P, fs, nv, col, g.nblk, blk, l, c);
            __syncthreads();  // the previous column's readers are done
#pragma unroll
            for (int k = 0; k < 12; ++k) s[k][l] = c[k];
            __syncthreads();
            LdsColumn ls{s};
            GlobalLinks<P_F32, false> lk{links};
            hopping_sum<float>(g, p, l, ls, lk, acc);
            clover_apply(cl, c, w);
#pragma unroll
            for (int k = 0; k < 12; ++k) w[k] = {w[k].re - kappa * acc[k].re, w[k].im - kappa * acc[k].im};
        } else {
            switch (d) {
            case 1: face_term<0, -1>(g, p, l, links, P, fs, nv, col, acc); break;
            case 2: face_term<0, +1>(g, p, l, links, P, fs, nv, col, acc); break;
            case 3: face_term<1, -1>(g, p, l, links, P, fs, nv, col, acc); break;
            case 4: face_term<1, +1>(g, p, l, links, P, fs, nv, col, acc); break;
            case 5: face_term<2, -1>(g, p, l, links, P, fs, nv, col, acc); break;
            case 6: face_term<2, +1>(g, p, l, links, P, fs, nv, col, acc); break;
            case 7: face_term<3, -1>(g, p, l, links, P, fs, nv, col, acc); break;
            default: face_term<3, +1>(g, p, l, links, P, fs, nv, col, acc); break;
            }
#pragma unroll
            for (int k = 0; k < 12; ++k) w[k] = {-kappa * acc[k].re, -kappa * acc[k].im};
        }
        // project onto the columns of this aggregate, two fields at a time
        for (int i0 = 0; i0 < nv; i0 += 2) {
            float dd[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (i0 + u < nv) {
                    cpx<float> q[12];
                    load_f32(P, fs, i0 + u, g.nblk, blk, l, q);
#pragma unroll
                    for (int k = 0; k < 12; ++k) {
                        const int o = 4 * u + (k < 6 ? 0 : 2);
                        dd[o] += q[k].re * w[k].re + q[k].im * w[k].im;
                        dd[o + 1] += q[k].re * w[k].im - q[k].im * w[k].re;
                    }
                }
            }
            block_sum<8>(dd, red, tot);
            if (l < 4) {
                const int u = l >> 1, chi = l & 1;
                const int i = i0 + u;
                if (i < nv) {
                    const int row = chi * nv + i;
                    Dc[(((size_t)blk * 9 + d) * nc + col) * nc + row] = make_float2(tot[4 * u + 2 * chi],
                                                                                    tot[4 * u + 2 * chi + 1]);
                }
            }
        }
    }
}

// --------------------------------------------------------------- transfer

// rc[a][chi * nv + i] = <p_{a,chi,i}, r> (r an FP32 field)
__global__ __launch_bounds__(TPB) void k_mg_restrict(Geom g, const char* P, size_t fs, int nv, const void* r,
                                                     float2* rc) {
    const int blk = blockIdx.x, l = threadIdx.x;
    __shared__ float red[4][8];
    __shared__ float tot[8];
    cpx<float> rv[12];
    SpinorIO<P_F32>::load(r, g.nblk, blk, l, rv);
    for (int i0 = 0; i0 < nv; i0 += 2) {
        float dd[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (i0 + u < nv) {
                cpx<float> q[12];
                load_f32(P, fs, i0 + u, g.nblk, blk, l, q);
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    const int o = 4 * u + (k < 6 ? 0 : 2);
                    dd[o] += q[k].re * rv[k].re + q[k].im * rv[k].im;
                    dd[o + 1] += q[k].re * rv[k].im - q[k].im * rv[k].re;
                }
            }
        }
        block_sum<8>(dd, red, tot);
        if (l < 4) {
            const int u = l >> 1, chi = l & 1, i = i0 + u;
            if (i < nv) rc[(size_t)blk * 2 * nv + chi * nv + i] = make_float2(tot[4 * u + 2 * chi], tot[4 * u + 2 * chi + 1]);
        }
    }
}

// z = P ec (an FP32 field)
__global__ __launch_bounds__(TPB) void k_mg_prolong(Geom g, const char* P, size_t fs, int nv, const float2* ec,
                                                    void* z) {
    const int blk = blockIdx.x, l = threadIdx.x;
    cpx<float> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = {0.f, 0.f};
    const float2* e = ec + (size_t)blk * 2 * nv;
    for (int i = 0; i < nv; ++i) {
        cpx<float> q[12];
        load_f32(P, fs, i, g.nblk, blk, l, q);
        const float2 e0 = e[i], e1 = e[nv + i];
        const cpx<float> c0 = {e0.x, e0.y}, c1 = {e1.x, e1.y};
#pragma unroll
        for (int k = 0; k < 12; ++k) cmac(o[k], k < 6 ? c0 : c1, q[k]);
    }
    SpinorIO<P_F32>::store(z, g.nblk, blk, l, o);
}

// ---------------------------------------------------------- coarse solver

// y = D_c x: one workgroup of 64 lanes per coarse site, lane = row.
__global__ __launch_bounds__(64) void k_mg_coarse_apply(Geom g, const float2* Dc, int nc, const float2* x,
                                                        float2* y, const CbScalars* sc) {
    if (sc && sc->stopped) return;
    const int a = blockIdx.x, row = threadIdx.x;
    if (row >= nc) return;
    const BlockPos p = block_pos(g, a);
    float re = 0.f, im = 0.f;
    for (int d = 0; d < 9; ++d) {
        const int nb = d == 0 ? a : block_step(g, p, (d - 1) >> 1, (d & 1) ? +1 : -1);
        const float2* m = Dc + ((size_t)a * 9 + d) * nc * nc + row;
        const float2* xv = x + (size_t)nb * nc;
        for (int c = 0; c < nc; ++c) {
            const float2 mm = m[(size_t)c * nc], xx = xv[c];
            re = fmaf(mm.x, xx.x, re);
            re = fmaf(-mm.y, xx.y, re);
            im = fmaf(mm.x, xx.y, im);
            im = fmaf(mm.y, xx.x, im);
        }
    }
    y[(size_t)a * nc + row] = make_float2(re, im);
}

__device__ __forceinline__ double2 cdiv2(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 cmul_d(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// FP64 wave/workgroup reduction of two complex values into partials slots
__device__ __forceinline__ void cb_partials(double a_re, double a_im, double b_re, double b_im, double2* partials) {
    __shared__ double red[4][4];
    double v[4] = {a_re, a_im, b_re, b_im};
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double s = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) red[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int k = threadIdx.x;
        partials[(size_t)blockIdx.x * 2 + k] = make_double2((red[0][2 * k] + red[1][2 * k]) + (red[2][2 * k] + red[3][2 * k]),
                                                            (red[0][2 * k + 1] + red[1][2 * k + 1]) +
                                                                (red[2][2 * k + 1] + red[3][2 * k + 1]));
    }
}

enum CbStep { CB_START = 0, CB_ALPHA = 1, CB_OMEGA = 2, CB_RHO = 3 };

// fixed-order sum of the partials (two complex slots per workgroup) and one step
__global__ __launch_bounds__(256) void k_cb_finalize(const double2* partials, int nwg, CbScalars* sc, int step,
                                                     double tol2) {
    if (step != CB_START && sc->stopped) return;
    __shared__ double2 red[2][256];
    const int t = threadIdx.x;
    double2 s0 = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
    for (int i = t; i < nwg; i += 256) {
        const double2 a = partials[(size_t)i * 2], b = partials[(size_t)i * 2 + 1];
        s0.x += a.x; s0.y += a.y; s1.x += b.x; s1.y += b.y;
    }
    red[0][t] = s0;
    red[1][t] = s1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t].x += red[0][t + w].x; red[0][t].y += red[0][t + w].y;
            red[1][t].x += red[1][t + w].x; red[1][t].y += red[1][t + w].y;
        }
        __syncthreads();
    }
    if (t != 0) return;
    const double2 d0 = red[0][0], d1 = red[1][0];
    if (step == CB_START) {  // d0.x = |r|^2
        sc->rho = make_double2(d0.x, 0.0);
        sc->rr = d0.x;
        sc->stop2 = tol2 * d0.x;
        sc->alpha = sc->omega = make_double2(1.0, 0.0);
        sc->beta = make_double2(0.0, 0.0);
        sc->stopped = d0.x > 0.0 ? 0 : 1;
    } else if (step == CB_ALPHA) {  // d0 = <rh, v>
        if (d0.x == 0.0 && d0.y == 0.0) sc->stopped = 1;  // before any update
        else sc->alpha = cdiv2(sc->rho, d0);
    } else if (step == CB_OMEGA) {  // d0 = <t, s>, d1.x = |t|^2
        sc->omega = d1.x > 0.0 ? make_double2(d0.x / d1.x, d0.y / d1.x) : make_double2(0.0, 0.0);
    } else {  // d0 = <rh, r>, d1.x = |r|^2 of the updated residual
        const bool w0 = sc->omega.x == 0.0 && sc->omega.y == 0.0;
        sc->beta = w0 ? make_double2(0.0, 0.0) : cmul_d(cdiv2(d0, sc->rho), cdiv2(sc->alpha, sc->omega));
        sc->rho = d0;
        sc->rr = d1.x;
        if (w0 || d1.x <= sc->stop2 || (d0.x == 0.0 && d0.y == 0.0)) sc->stopped = 1;
    }
}

// x = 0, r = rh = rc, p = v = 0, partial |r|^2
__global__ __launch_bounds__(256) void k_cb_init(int n, const float2* rc, CbVecs cv, double2* partials) {
    double s = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float2 r = rc[i];
        cv.x[i] = cv.p[i] = cv.v[i] = make_float2(0.f, 0.f);
        cv.r[i] = cv.rh[i] = r;
        s += (double)r.x * r.x + (double)r.y * r.y;
    }
    cb_partials(s, 0.0, 0.0, 0.0, partials);
}

__global__ __launch_bounds__(256) void k_cb_p(int n, const CbScalars* sc, CbVecs cv) {
    if (sc->stopped) return;
    const float br = (float)sc->beta.x, bi = (float)sc->beta.y, wr = (float)sc->omega.x, wi = (float)sc->omega.y;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float2 r = cv.r[i], p = cv.p[i], v = cv.v[i];
        // p = r + beta (p - omega v)
        const float tr = p.x - (wr * v.x - wi * v.y), ti = p.y - (wr * v.y + wi * v.x);
        cv.p[i] = make_float2(r.x + br * tr - bi * ti, r.y + br * ti + bi * tr);
    }
}

// partial <a, b> (slot 0) and, with TWO, |a|^2 (slot 1)
template <bool TWO>
__global__ __launch_bounds__(256) void k_cb_dot(int n, const CbScalars* sc, const float2* a, const float2* b,
                                                double2* partials) {
    if (sc->stopped) return;
    double re = 0.0, im = 0.0, aa = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float2 x = a[i], y = b[i];
        re += (double)x.x * y.x + (double)x.y * y.y;
        im += (double)x.x * y.y - (double)x.y * y.x;
        if (TWO) aa += (double)x.x * x.x + (double)x.y * x.y;
    }
    cb_partials(re, im, aa, 0.0, partials);
}

__global__ __launch_bounds__(256) void k_cb_s(int n, const CbScalars* sc, CbVecs cv) {
    if (sc->stopped) return;
    const float ar = (float)sc->alpha.x, ai = (float)sc->alpha.y;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float2 r = cv.r[i], v = cv.v[i];
        cv.s[i] = make_float2(r.x - (ar * v.x - ai * v.y), r.y - (ar * v.y + ai * v.x));
    }
}

// x += alpha p + omega s, r = s - omega t; partials <rh, r>, |r|^2
__global__ __launch_bounds__(256) void k_cb_xr(int n, const CbScalars* sc, CbVecs cv, double2* partials) {
    if (sc->stopped) return;
    const float ar = (float)sc->alpha.x, ai = (float)sc->alpha.y, wr = (float)sc->omega.x, wi = (float)sc->omega.y;
    double re = 0.0, im = 0.0, rr = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float2 x = cv.x[i], p = cv.p[i], s = cv.s[i], t = cv.t[i], h = cv.rh[i];
        cv.x[i] = make_float2(x.x + (ar * p.x - ai * p.y) + (wr * s.x - wi * s.y),
                              x.y + (ar * p.y + ai * p.x) + (wr * s.y + wi * s.x));
        const float2 r = make_float2(s.x - (wr * t.x - wi * t.y), s.y - (wr * t.y + wi * t.x));
        cv.r[i] = r;
        re += (double)h.x * r.x + (double)h.y * r.y;
        im += (double)h.x * r.y - (double)h.y * r.x;
        rr += (double)r.x * r.x + (double)r.y * r.y;
    }
    cb_partials(re, im, rr, 0.0, partials);
}

int cb_grid(int n) {
    const int b = (n + 255) / 256;
    return b < 1024 ? b : 1024;
}

}  // namespace

hipError_t mg_orthonormalize(const Geom& g, void* P, int nv, hipStream_t s) {
    ProfScope ps("mg", s);
    hipLaunchKernelGGL(k_mg_orthonormalize, dim3(g.nblk), dim3(TPB), 0, s, g, (char*)P,
                       spinor_bytes_per_site(P_F32) * g.V, nv);
    return hipGetLastError();
}

hipError_t mg_assemble(const OpData& op, const void* P, int nv, float2* Dc, hipStream_t s) {
    ProfScope ps("mg", s);
    hipLaunchKernelGGL(k_mg_assemble, dim3(op.g.nblk, 9), dim3(TPB), 0, s, op.g, op.links[P_F32], op.clover32,
                       (float)op.kappa, (const char*)P, spinor_bytes_per_site(P_F32) * op.g.V, nv, Dc);
    return hipGetLastError();
}

hipError_t mg_restrict(const Geom& g, const void* P, int nv, const void* r, float2* rc, hipStream_t s) {
    ProfScope ps("mg", s);
    hipLaunchKernelGGL(k_mg_restrict, dim3(g.nblk), dim3(TPB), 0, s, g, (const char*)P,
                       spinor_bytes_per_site(P_F32) * g.V, nv, r, rc);
    return hipGetLastError();
}

hipError_t mg_prolong(const Geom& g, const void* P, int nv, const float2* ec, void* z, hipStream_t s) {
    ProfScope ps("mg", s);
    hipLaunchKernelGGL(k_mg_prolong, dim3(g.nblk), dim3(TPB), 0, s, g, (const char*)P,
                       spinor_bytes_per_site(P_F32) * g.V, nv, ec, z);
    return hipGetLastError();
}

hipError_t mg_coarse_apply(const Geom& g, const float2* Dc, int nc, const float2* x, float2* y,
                           const CbScalars* sc, hipStream_t s) {
    ProfScope ps("mg", s);
    hipLaunchKernelGGL(k_mg_coarse_apply, dim3(g.nblk), dim3(64), 0, s, g, Dc, nc, x, y, sc);
    return hipGetLastError();
}

hipError_t mg_coarse_bicgstab(const Geom& g, const float2* Dc, int nc, const float2* rc, const CbVecs& cv,
                              CbScalars* sc, double2* partials, int max_iter, double tol, hipStream_t s) {
    ProfScope ps("mg", s);
    const int n = g.nblk * nc, grid = cb_grid(n);
#define CB_LAUNCH(...)                           \
    do {                                         \
        hipLaunchKernelGGL(__VA_ARGS__);         \
        hipError_t e_ = hipGetLastError();       \
        if (e_ != hipSuccess) return e_;         \
    } while (0)
    CB_LAUNCH(k_cb_init, dim3(grid), dim3(256), 0, s, n, rc, cv, partials);
    CB_LAUNCH(k_cb_finalize, dim3(1), dim3(256), 0, s, partials, grid, sc, (int)CB_START, tol * tol);
    for (int it = 0; it < max_iter; ++it) {
        CB_LAUNCH(k_cb_p, dim3(grid), dim3(256), 0, s, n, sc, cv);
        CB_LAUNCH(k_mg_coarse_apply, dim3(g.nblk), dim3(64), 0, s, g, Dc, nc, cv.p, cv.v, sc);
        CB_LAUNCH((k_cb_dot<false>), dim3(grid), dim3(256), 0, s, n, sc, cv.rh, cv.v, partials);
        CB_LAUNCH(k_cb_finalize, dim3(1), dim3(256), 0, s, partials, grid, sc, (int)CB_ALPHA, 0.0);
        CB_LAUNCH(k_cb_s, dim3(grid), dim3(256), 0, s, n, sc, cv);
        CB_LAUNCH(k_mg_coarse_apply, dim3(g.nblk), dim3(64), 0, s, g, Dc, nc, cv.s, cv.t, sc);
        CB_LAUNCH((k_cb_dot<true>), dim3(grid), dim3(256), 0, s, n, sc, cv.t, cv.s, partials);
        CB_LAUNCH(k_cb_finalize, dim3(1), dim3(256), 0, s, partials, grid, sc, (int)CB_OMEGA, 0.0);
        CB_LAUNCH(k_cb_xr, dim3(grid), dim3(256), 0, s, n, sc, cv, partials);
        CB_LAUNCH(k_cb_finalize, dim3(1), dim3(256), 0, s, partials, grid, sc, (int)CB_RHO, 0.0);
    }
#undef CB_LAUNCH
    return hipSuccess;
}

}  // namespace cs
