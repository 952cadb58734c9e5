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
#include <type_traits>

#include "blas.hpp"
#include "dslash_core.hpp"
#include "wave.hpp"
#include "mg.hpp"

namespace cs {

namespace {

constexpr int TPB = BLOCK_SITES;

// Sum N values over the workgroup; afterwards out[k] (LDS) holds total k.
template <int N>
__device__ __forceinline__ void block_sum(const float* v, float (*red)[N], float* out) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float t[N];
#pragma unroll
    for (int k = 0; k < N; ++k) t[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) red[wave][k] = t[k];
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
    const lds_cpx<float> (*s)[BLOCK_SITES];
    __device__ __forceinline__ bool want(bool inside) const { return inside; }
    template <typename R>
    __device__ __forceinline__ void load_nb(int, int l, bool, cpx<R>* c) const {
#pragma unroll
        for (int k = 0; k < 12; ++k) c[k] = s[k][l].get();
    }
};

// Assembly of D_c[a][d][col][row] = <p_{a,row}, D p_{n(a,d),col}> restricted
// to the terms of D that couple aggregate a to its neighbour in direction d.
// One workgroup per (aggregate, column), lane = site; the nc workgroups of an
// aggregate are consecutive on one XCD, so the aggregate's rows of P, links
// and clover term come from HBM once and from that XCD's L2 for the others.
// The column is applied once: the self term (clover and the in-aggregate
// hops of the column, staged in LDS) and the four -mu face terms (hops from
// the neighbouring aggregates) stay in registers while every row of P
// streams past; per row each lane
// forms 20 partial dot products (self term and four faces, two row
// chiralities, re and im), which are summed over the lanes through a
// lane-major LDS array in a fixed order.  The +mu blocks follow afterwards
// from gamma5-hermiticity (k_mg_assemble_fwd).
constexpr int ASM_R = 2;                 // rows per reduction round
constexpr int ASM_VALS = 20 * ASM_R;     // partial sums per lane and round
constexpr int ASM_LD = ASM_VALS + 1;     // padded row of the lane-major array

// y += conj(q) . x over the spins of each chirality: out[2 chi + (re, im)]
__device__ __forceinline__ void chi_dots(const cpx<float>* q, const cpx<float>* x, float* out) {
    float a[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const int o = k < 6 ? 0 : 2;
        a[o] += q[k].re * x[k].re + q[k].im * x[k].im;
        a[o + 1] += q[k].re * x[k].im - q[k].im * x[k].re;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = a[k];
}

// -kappa times the backward hop across the -MU face into lane l (zero on
// lanes not on that face)
template <int MU>
__device__ __forceinline__ void back_face(const Geom& g, const BlockPos& p, int l, const void* links,
                                          const char* P, size_t fs, int nv, int col, float kappa, cpx<float>* y) {
#pragma unroll
    for (int k = 0; k < 12; ++k) y[k] = {0.f, 0.f};
    if (((l >> (2 * MU)) & 3) != 0) return;
    int nl;
    bool in;
    const int nb = neighbour(g, p, l, MU, -1, &nl, &in);
    cpx<float> psi[12], u[9];
    column_site(P, fs, nv, col, g.nblk, nb, nl, psi);
    if (MU == 3) time_boundary_phase(g, wraps_time(g, p, MU, -1, in), &psi[0].re, 24);
    load_link<P_F32, float, false>(links, nb, nl, MU, u);  // U_mu(x - mu)
    hop_term<MU, +1>(u, psi, y);
#pragma unroll
    for (int k = 0; k < 12; ++k) y[k] = {-kappa * y[k].re, -kappa * y[k].im};
}

__global__ __launch_bounds__(TPB, 2) void k_mg_assemble(Geom g, const void* links, const void* clover, float kappa,
                                                     const char* P, size_t fs, int nv, float2* Dc) {
    const int l = threadIdx.x, nc = 2 * nv;
    const int w = xcd_remap(blockIdx.x, g.nblk * nc), blk = w / nc;
    const BlockPos p = block_pos(g, blk);
    __shared__ lds_cpx<float> s[12][BLOCK_SITES];
    __shared__ float red[BLOCK_SITES * ASM_LD];
    __shared__ float part[ASM_VALS][4];
    {
        const int col = w % nc;
        cpx<float> y0[12], yf[4][12];
        {
            cpx<float> c[12], acc[12];
            column_site(P, fs, nv, col, g.nblk, blk, l, c);
#pragma unroll
            for (int k = 0; k < 12; ++k) s[k][l].set(c[k]);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = {0.f, 0.f};
            LdsColumn ls{s};
            GlobalLinks<P_F32, false> lk{links};
            hopping_sum<float>(g, p, l, ls, lk, acc);
            float cl[72];
            CloverIO<float>::template load<false>(clover, blk, l, cl);
            clover_apply(cl, c, y0);
#pragma unroll
            for (int k = 0; k < 12; ++k) y0[k] = {y0[k].re - kappa * acc[k].re, y0[k].im - kappa * acc[k].im};
        }
        back_face<0>(g, p, l, links, P, fs, nv, col, kappa, yf[0]);
        back_face<1>(g, p, l, links, P, fs, nv, col, kappa, yf[1]);
        back_face<2>(g, p, l, links, P, fs, nv, col, kappa, yf[2]);
        back_face<3>(g, p, l, links, P, fs, nv, col, kappa, yf[3]);
        for (int i0 = 0; i0 < nv; i0 += ASM_R) {
            // partial sums of this lane: value 20 r + 4 e + 2 chi + (re, im),
            // e = 0 the self term, e = 1 + mu the -mu face
#pragma unroll
            for (int r = 0; r < ASM_R; ++r) {
                float v[20];
                if (i0 + r < nv) {
                    cpx<float> q[12];
                    load_f32(P, fs, i0 + r, g.nblk, blk, l, q);
                    chi_dots(q, y0, v);
#pragma unroll
                    for (int mu = 0; mu < 4; ++mu) chi_dots(q, yf[mu], v + 4 + 4 * mu);
                } else {
#pragma unroll
                    for (int k = 0; k < 20; ++k) v[k] = 0.f;
                }
#pragma unroll
                for (int k = 0; k < 20; ++k) red[l * ASM_LD + 20 * r + k] = v[k];
            }
            __syncthreads();
            // four partial sums of 64 lanes per value, then their fixed-order total
            for (int w = l; w < 4 * ASM_VALS; w += TPB) {
                const int val = w >> 2, seg = w & 3;
                float sum = 0.f;
                for (int j = 0; j < 64; ++j) sum += red[(seg * 64 + j) * ASM_LD + val];
                part[val][seg] = sum;
            }
            __syncthreads();
            for (int val = l; val < ASM_VALS; val += TPB) {
                const int r = val / 20, rem = val % 20, e = rem >> 2, chi = (rem >> 1) & 1;
                if ((rem & 1) == 0 && i0 + r < nv) {
                    const float re = (part[val][0] + part[val][1]) + (part[val][2] + part[val][3]);
                    const float im = (part[val + 1][0] + part[val + 1][1]) + (part[val + 1][2] + part[val + 1][3]);
                    const int row = chi * nv + i0 + r, d = e == 0 ? 0 : 2 * e;  // e = 1 + mu -> d = 2 + 2 mu
                    Dc[(((size_t)blk * 9 + d) * nc + col) * nc + row] = make_float2(re, im);
                }
            }
            __syncthreads();  // red and part are reused by the next round
        }
    }
}

// D_c[a][1 + 2 mu] from gamma5-hermiticity of D (P keeps chirality):
// D_c[a][+mu][col][row] = g5(col) g5(row) conj(D_c[b][-mu][row][col]) with
// b the +mu neighbour of a and g5 = +1 on chirality 0, -1 on chirality 1.
__global__ __launch_bounds__(TPB) void k_mg_assemble_fwd(Geom g, int nv, float2* Dc) {
    const int a = blockIdx.x, mu = blockIdx.y, nc = 2 * nv;
    const BlockPos p = block_pos(g, a);
    const int b = block_step(g, p, mu, +1);
    const float2* src = Dc + ((size_t)b * 9 + 2 + 2 * mu) * nc * nc;
    float2* dst = Dc + ((size_t)a * 9 + 1 + 2 * mu) * nc * nc;
    for (int idx = threadIdx.x; idx < nc * nc; idx += TPB) {
        const int col = idx / nc, row = idx % nc;
        const float sg = ((col < nv) == (row < nv)) ? 1.f : -1.f;
        const float2 v = src[(size_t)row * nc + col];
        dst[idx] = make_float2(sg * v.x, -sg * v.y);
    }
}

// --------------------------------------------------------------- transfer

// rc[a][chi * nv + i] = <p_{a,chi,i}, r> (r an FP32 field)
template <int PP>
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
                SpinorIO<PP>::load(P + (size_t)(i0 + u) * fs, g.nblk, blk, l, q);
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

// The restriction of nr FP32 fields r_j (stride rs) into nr coarse vectors
// (stride rcs), R fields per workgroup: each P row read serves all R, and
// every r_j gets the sums of k_mg_restrict (same terms, same order).
template <int PP, int R>
__global__ __launch_bounds__(TPB) void k_mg_restrict_many(Geom g, const char* P, size_t fs, int nv,
                                                          const char* rbase, size_t rs, int nr, float2* rcbase,
                                                          size_t rcs) {
    const int blk = blockIdx.x, l = threadIdx.x, j0 = blockIdx.y * R;
    __shared__ float red[4][8 * R];
    __shared__ float tot[8 * R];
    cpx<float> rv[R][12];
#pragma unroll
    for (int u = 0; u < R; ++u)
        SpinorIO<P_F32>::load(rbase + (size_t)(j0 + u < nr ? j0 + u : nr - 1) * rs, g.nblk, blk, l, rv[u]);
    for (int i0 = 0; i0 < nv; i0 += 2) {
        float dd[8 * R];
#pragma unroll
        for (int k = 0; k < 8 * R; ++k) dd[k] = 0.f;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (i0 + u < nv) {
                cpx<float> q[12];
                SpinorIO<PP>::load(P + (size_t)(i0 + u) * fs, g.nblk, blk, l, q);
#pragma unroll
                for (int j = 0; j < R; ++j)
#pragma unroll
                    for (int k = 0; k < 12; ++k) {
                        const int o = 8 * j + 4 * u + (k < 6 ? 0 : 2);
                        dd[o] += q[k].re * rv[j][k].re + q[k].im * rv[j][k].im;
                        dd[o + 1] += q[k].re * rv[j][k].im - q[k].im * rv[j][k].re;
                    }
            }
        }
        block_sum<8 * R>(dd, red, tot);
        if (l < 4 * R) {
            const int j = l >> 2, u = (l >> 1) & 1, chi = l & 1, i = i0 + u;
            if (i < nv && j0 + j < nr)
                rcbase[(size_t)(j0 + j) * rcs + (size_t)blk * 2 * nv + chi * nv + i] =
                    make_float2(tot[8 * j + 4 * u + 2 * chi], tot[8 * j + 4 * u + 2 * chi + 1]);
        }
    }
}

// z = P ec (an FP32 field)
template <int PP>
__global__ __launch_bounds__(TPB) void k_mg_prolong(Geom g, const char* P, size_t fs, int nv, const float2* ec,
                                                    void* z) {
    const int blk = blockIdx.x, l = threadIdx.x;
    cpx<float> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = {0.f, 0.f};
    const float2* e = ec + (size_t)blk * 2 * nv;
    for (int i = 0; i < nv; ++i) {
        cpx<float> q[12];
        SpinorIO<PP>::load(P + (size_t)i * fs, g.nblk, blk, l, q);
        const float2 e0 = e[i], e1 = e[nv + i];
        const cpx<float> c0 = {e0.x, e0.y}, c1 = {e1.x, e1.y};
#pragma unroll
        for (int k = 0; k < 12; ++k) cmac(o[k], k < 6 ? c0 : c1, q[k]);
    }
    SpinorIO<P_F32>::store(z, g.nblk, blk, l, o);
}

// The prolongation of nr coarse vectors (stride ecs) into nr FP32 fields
// (stride zs), R per workgroup: each P row read serves all R, every z_j
// gets the sums of k_mg_prolong (same terms, same order).
template <int PP, int R>
__global__ __launch_bounds__(TPB) void k_mg_prolong_many(Geom g, const char* P, size_t fs, int nv,
                                                         const float2* ecbase, size_t ecs, int nr, char* zbase,
                                                         size_t zs) {
    const int blk = blockIdx.x, l = threadIdx.x, j0 = blockIdx.y * R;
    cpx<float> o[R][12];
#pragma unroll
    for (int j = 0; j < R; ++j)
#pragma unroll
        for (int k = 0; k < 12; ++k) o[j][k] = {0.f, 0.f};
    for (int i = 0; i < nv; ++i) {
        cpx<float> q[12];
        SpinorIO<PP>::load(P + (size_t)i * fs, g.nblk, blk, l, q);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const float2* e = ecbase + (size_t)(j0 + j < nr ? j0 + j : nr - 1) * ecs + (size_t)blk * 2 * nv;
            const float2 e0 = e[i], e1 = e[nv + i];
            const cpx<float> c0 = {e0.x, e0.y}, c1 = {e1.x, e1.y};
#pragma unroll
            for (int k = 0; k < 12; ++k) cmac(o[j][k], k < 6 ? c0 : c1, q[k]);
        }
    }
#pragma unroll
    for (int j = 0; j < R; ++j)
        if (j0 + j < nr) SpinorIO<P_F32>::store(zbase + (size_t)(j0 + j) * zs, g.nblk, blk, l, o[j]);
}

// ---------------------------------------------------------- coarse solver
//
// Matrix-vector products with D_c read 5 of the 9 stencil blocks of every
// aggregate.  The +mu blocks are fixed by the -mu blocks of the neighbours
// through gamma5-hermiticity, D_c[b - mu][+mu] = G5 D_c[b][-mu]^dag G5 (G5 =
// +1 on chirality 0, -1 on chirality 1), so the product runs in two passes:
//   pass 1, one workgroup of 256 lanes per aggregate a: y_a = D_c[a][0] x_a
//     + sum_mu D_c[a][-mu] x_{a - mu}, and tau[a][mu] = G5 D_c[a][-mu]^dag G5
//     x_a, the +mu contribution of a to the aggregate a - mu;
//   pass 2, elementwise: y_a += sum_mu tau[a + mu][mu], mu in increasing order.
// Each -mu block is read from HBM once (its adjoint re-reads it from cache).
// In pass 1 the five blocks are one K5 x nc matrix M[k][row] (k = slot nc +
// col, slot 0 the aggregate itself, slot 1 + mu its -mu block, row fastest)
// applied to the gathered vector xg[k] = x_{n(a, slot), col} staged in LDS.
// Lane t owns row t % nc and the column chunk t / nc (every (256 / nc)-th
// k), so a wave reads whole consecutive rows of M (coalesced) and each lane
// keeps several independent loads in flight; the chunks are then added in a
// fixed order.  The adjoints give lane t the outputs o = t, t + 256, ... of
// the 4 nc values tau[a][mu][i] (o = mu nc + i), each a sum over the nc
// entries of one stored column.

constexpr int CMV_TPB = 256;
constexpr int CMV_KMAX = 5 * 2 * MG_MAX_NV;

__device__ __forceinline__ int coarse_nb(const Geom& g, const BlockPos& p, int d) {
    return d == 0 ? p.blk : block_step(g, p, (d - 1) >> 1, (d & 1) ? +1 : -1);
}

// stencil direction of gather slot sl: the aggregate itself, then -mu
__device__ __forceinline__ int slot_dir(int sl) { return sl == 0 ? 0 : 2 * sl; }

// Entry i of the coarse matrices, FP32 or FP16 storage
template <bool HALF>
__device__ __forceinline__ float2 cm_load(const void* M, size_t i) {
    if (HALF) {
        float a, b;
        unpack2<P_F16>(((const unsigned int*)M)[i], a, b);
        return make_float2(a, b);
    }
    return ((const float2*)M)[i];
}

// y_row = sum over the self and -mu blocks of aggregate a of M[k][row] xs[k];
// valid in lanes t < nc (others return 0)
template <bool HALF>
__device__ __forceinline__ float2 cmv_rows5(const void* __restrict__ Dc, int a, int nc, const float2* xs,
                                            float2* red) {
    const int t = threadIdx.x, kch = CMV_TPB / nc, row = t % nc, kc = t / nc, K5 = 5 * nc;
    const size_t base = (size_t)a * 9 * nc * nc + row;
    float re = 0.f, im = 0.f, re2 = 0.f, im2 = 0.f;
    if (kc < kch) {
        int k = kc;
        for (; k + kch < K5; k += 2 * kch) {
            const int k1 = k + kch;
            const float2 m0 = cm_load<HALF>(Dc, base + (size_t)(slot_dir(k / nc) * nc + k % nc) * nc);
            const float2 m1 = cm_load<HALF>(Dc, base + (size_t)(slot_dir(k1 / nc) * nc + k1 % nc) * nc);
            const float2 x0 = xs[k], x1 = xs[k1];
            re = fmaf(m0.x, x0.x, re); re = fmaf(-m0.y, x0.y, re);
            im = fmaf(m0.x, x0.y, im); im = fmaf(m0.y, x0.x, im);
            re2 = fmaf(m1.x, x1.x, re2); re2 = fmaf(-m1.y, x1.y, re2);
            im2 = fmaf(m1.x, x1.y, im2); im2 = fmaf(m1.y, x1.x, im2);
        }
        if (k < K5) {
            const float2 m0 = cm_load<HALF>(Dc, base + (size_t)(slot_dir(k / nc) * nc + k % nc) * nc), x0 = xs[k];
            re = fmaf(m0.x, x0.x, re); re = fmaf(-m0.y, x0.y, re);
            im = fmaf(m0.x, x0.y, im); im = fmaf(m0.y, x0.x, im);
        }
    }
    red[t] = make_float2(re + re2, im + im2);
    __syncthreads();
    float2 y = make_float2(0.f, 0.f);
    if (t < nc)
        for (int c = 0; c < kch; ++c) {
            const float2 v = red[c * nc + t];
            y.x += v.x;
            y.y += v.y;
        }
    return y;
}

// tau[a][mu][i] = sum_c g5(i) g5(c) conj(D_c[a][-mu][col i][row c]) xa[c],
// xa the aggregate's own entries (LDS)
template <bool HALF>
__device__ __forceinline__ void cmv_adjoint4(const void* __restrict__ Dc, int a, int nc, const float2* xa,
                                             float2* __restrict__ tau) {
    const int nv = nc / 2;
    for (int o = threadIdx.x; o < 4 * nc; o += CMV_TPB) {
        const int mu = o / nc, i = o % nc;
        const size_t base = (((size_t)a * 9 + 2 + 2 * mu) * nc + i) * nc;
        float re = 0.f, im = 0.f;
        for (int c = 0; c < nc; ++c) {
            const float2 m = cm_load<HALF>(Dc, base + c);
            const float2 x = xa[c];
            const float sg = (i < nv) == (c < nv) ? 1.f : -1.f;
            // conj(m) x
            re = fmaf(sg * m.x, x.x, re); re = fmaf(sg * m.y, x.y, re);
            im = fmaf(sg * m.x, x.y, im); im = fmaf(-sg * m.y, x.x, im);
        }
        tau[((size_t)a * 4 + mu) * nc + i] = make_float2(re, im);
    }
}

// Sum over aligned groups of G = 16, 32 or 64 lanes (a row of the wave, a
// half or the whole wave); every lane of the group receives the total.
template <int G>
__device__ __forceinline__ float group_sum(float v) {
    using namespace wave_detail;
    v += dpp_move<DPP_XOR1>(v);
    v += dpp_move<DPP_XOR2>(v);
    v += dpp_move<DPP_HALF_MIRROR>(v);
    v += dpp_move<DPP_MIRROR>(v);
    if constexpr (G >= 32) v = cross_add<16>(v);
    if constexpr (G >= 64) v = cross_add<32>(v);
    return v;
}

// Pass 1 of the product for nc = NC in {16, 32, 64}: the adjoint terms come
// from the same loads as the forward ones.  The NC lanes of the group kc
// all hold entry k of one stored column (rows 0..NC-1), so each lane forms
// g5(col) g5(row) conj(M[k][row]) xa[row] and a group sum gives
// tau[a][mu][col] for the -mu slots (it is formed, and dropped, for the
// self slot too, so that every lane takes part in every exchange).  The
// loads of a lane are issued in batches (5 FP32 or 10 FP16 entries) before
// their arithmetic, and the sums are stored after the loop, so no store
// sits between loads.
// The forward chunks are reduced as in cmv_rows5.
template <bool HALF, int NC>
__device__ __forceinline__ float2 cmv5_fused(const void* __restrict__ Dc, int a, const float2* xs, float2* red,
                                             float2* __restrict__ tau) {
    constexpr int KCH = CMV_TPB / NC, NJ = 5 * NC / KCH, NV = NC / 2;
    // loads issued together before their arithmetic (NJ is 5, 20 or 80)
    constexpr int CH = NJ < (HALF ? 10 : 5) ? NJ : (HALF ? 10 : 5);
    static_assert(NJ % CH == 0 && NJ <= 2 * NC, "batches cover the loop; a lane keeps at most two sums");
    const int t = threadIdx.x, row = t % NC, kc = t / NC;
    const size_t base = (size_t)a * 9 * NC * NC + row;
    const float2 xa = xs[row];
    float re = 0.f, im = 0.f;
    // the adjoint sums this lane stores: j = row and j = row + NC
    float2 keep0 = make_float2(0.f, 0.f), keep1 = make_float2(0.f, 0.f);
#pragma unroll 1
    for (int j0 = 0; j0 < NJ; j0 += CH) {
        float2 m[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int k = kc + (j0 + c) * KCH;
            m[c] = cm_load<HALF>(Dc, base + (size_t)(slot_dir(k / NC) * NC + k % NC) * NC);
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int j = j0 + c, k = kc + j * KCH, col = k % NC;
            const float2 x = xs[k];
            re = fmaf(m[c].x, x.x, re);
            re = fmaf(-m[c].y, x.y, re);
            im = fmaf(m[c].x, x.y, im);
            im = fmaf(m[c].y, x.x, im);
            const float sg = (col < NV) == (row < NV) ? 1.f : -1.f;
            float ar = sg * fmaf(m[c].x, xa.x, m[c].y * xa.y), ai = sg * fmaf(m[c].x, xa.y, -m[c].y * xa.x);
            ar = group_sum<NC>(ar);
            ai = group_sum<NC>(ai);
            if (j == row) keep0 = make_float2(ar, ai);
            if (j == row + NC) keep1 = make_float2(ar, ai);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int j = i * NC + row;
        if (j < NJ) {
            const int k = kc + j * KCH, sl = k / NC;
            if (sl > 0) tau[((size_t)a * 4 + sl - 1) * NC + k % NC] = i ? keep1 : keep0;
        }
    }
    red[t] = make_float2(re, im);
    __syncthreads();
    float2 y = make_float2(0.f, 0.f);
    if (t < NC)
        for (int c = 0; c < KCH; ++c) {
            const float2 v = red[c * NC + t];
            y.x += v.x;
            y.y += v.y;
        }
    return y;
}

// Pass 1 for any nc: NC = 0 takes the two-step form
template <bool HALF, int NC>
__device__ __forceinline__ float2 cmv5(const void* __restrict__ Dc, int a, int nc, const float2* xs, float2* red,
                                       float2* __restrict__ tau) {
    if constexpr (NC > 0) {
        return cmv5_fused<HALF, NC>(Dc, a, xs, red, tau);
    } else {
        const float2 y = cmv_rows5<HALF>(Dc, a, nc, xs, red);
        cmv_adjoint4<HALF>(Dc, a, nc, xs, tau);
        return y;
    }
}

// Gather of slot sl's entries of x for aggregate p (n(a, slot))
__device__ __forceinline__ size_t gather_index(const Geom& g, const BlockPos& p, int nc, int k) {
    return (size_t)coarse_nb(g, p, slot_dir(k / nc)) * nc + k % nc;
}

// Pass 2 for entry i = a nc + row: the +mu contributions of the four +mu
// neighbours, in increasing mu
__device__ __forceinline__ float2 tau_sum(const Geom& g, int nc, const float2* __restrict__ tau, size_t i) {
    const int a = (int)(i / nc), row = (int)(i % nc);
    const BlockPos p = block_pos(g, a);
    float2 s = make_float2(0.f, 0.f);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int b = block_step(g, p, mu, +1);
        const float2 v = tau[((size_t)b * 4 + mu) * nc + row];
        s.x += v.x;
        s.y += v.y;
    }
    return s;
}

__device__ __forceinline__ double2 cdot_d(float2 a, float2 b) {  // conj(a) b
    return make_double2((double)a.x * b.x + (double)a.y * b.y, (double)a.x * b.y - (double)a.y * b.x);
}

// y = D_c x, pass 1 (y holds the self and -mu terms afterwards, tau the
// adjoint terms)
template <bool HALF, int NC>
__global__ __launch_bounds__(CMV_TPB) void k_mg_coarse_apply(Geom g, const void* __restrict__ Dc, int nc,
                                                             const float2* __restrict__ x, float2* __restrict__ y,
                                                             float2* __restrict__ tau) {
    __shared__ float2 xs[CMV_KMAX];
    __shared__ float2 red[CMV_TPB];
    const int a = blockIdx.x, K5 = 5 * nc;
    const BlockPos p = block_pos(g, a);
    for (int k = threadIdx.x; k < K5; k += CMV_TPB) xs[k] = x[gather_index(g, p, nc, k)];
    __syncthreads();
    const float2 v = cmv5<HALF, NC>(Dc, a, nc, xs, red, tau);
    if ((int)threadIdx.x < nc) y[(size_t)a * nc + threadIdx.x] = v;
}

// y = D_c x, pass 2
__global__ __launch_bounds__(256) void k_mg_coarse_complete(Geom g, int nc, float2* __restrict__ y,
                                                            const float2* __restrict__ tau) {
    const size_t n = (size_t)g.nblk * nc;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float2 t = tau_sum(g, nc, tau, i);
        const float2 v = y[i];
        y[i] = make_float2(v.x + t.x, v.y + t.y);
    }
}

__device__ __forceinline__ double2 cdiv2(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 cmul_d(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Coarse BiCGStab.  The start (x = 0, r = rh = r_c) is followed by the stop
// test F1 of iteration 0; iteration it (parity q = it & 1) is then eight
// launches, the last of which is the stop test of iteration it + 1:
//   M1  p = r + beta (p_prev - omega v_prev) formed while gathering, pass 1
//       of v = D_c p
//   C1  pass 2 of v = D_c p, partials B = <rh, v>
//   F2  alpha = rho_new / <rh, v> (a zero denominator ends the solve)
//   M2  s = r - alpha v formed while gathering, pass 1 of t = D_c s
//   C2  pass 2 of t = D_c s, partials C = <t, s>, |t|^2
//   F3  omega = <t, s> / |t|^2 (0 when t = 0)
//   U   x += alpha p + omega s, r = s - omega t, partials A
//   F1  rho_new = <rh, r>, |r|^2 from the partials A; stop before the next
//       iteration when rho_new = 0, omega = 0, |r| <= tol |r_0| or an earlier
//       stop; beta = (rho_new / rho_old) (alpha / omega)
// p and v alternate between two buffers by parity, so the gathers of M1 read
// the previous iteration's values while its own entries are written.  A
// kernel reads only scalars written by earlier kernels (slots by parity
// where a kernel would otherwise read what it writes), and every later
// kernel returns at once after a stop, so a fixed number of iterations can be
// launched or captured; stopped[it & 1] tells whether iteration it runs.

// Fixed-order sum of the first three reals (re, im of slot 0; re of slot 1)
// of nwg two-slot partials by one workgroup of 1024 lanes; valid in lane 0.
__device__ __forceinline__ void sum3_partials(const double2* partials, int nwg, double* out) {
    __shared__ double red[3][1024];
    const int t = threadIdx.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int i = t; i < nwg; i += 1024) {
        const double2 a = partials[(size_t)i * 2], b = partials[(size_t)i * 2 + 1];
        s0 += a.x;
        s1 += a.y;
        s2 += b.x;
    }
    red[0][t] = s0;
    red[1][t] = s1;
    red[2][t] = s2;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] += red[0][t + w];
            red[1][t] += red[1][t + w];
            red[2][t] += red[2][t + w];
        }
        __syncthreads();
    }
    out[0] = red[0][0];
    out[1] = red[1][0];
    out[2] = red[2][0];
}

__global__ __launch_bounds__(1024) void k_cb_f1(const double2* partials, int nwg, CbScalars* sc, int it,
                                                double tol2) {
    const int q = it & 1;
    double tot[3];
    sum3_partials(partials, nwg, tot);
    if (threadIdx.x != 0) return;
    const double2 rho = make_double2(tot[0], tot[1]);
    const double rr = tot[2];
    int stop;
    if (it == 0) {
        sc->stop2 = tol2 * rr;
        sc->alpha = sc->omega = make_double2(1.0, 0.0);
        sc->beta[q] = make_double2(0.0, 0.0);
        stop = 0;
    } else {
        const bool w0 = sc->omega.x == 0.0 && sc->omega.y == 0.0;
        stop = sc->stopped[q ^ 1] || sc->brk[q ^ 1] || w0 || rr <= sc->stop2;
        sc->beta[q] = stop ? make_double2(0.0, 0.0) : cmul_d(cdiv2(rho, sc->rho[q ^ 1]), cdiv2(sc->alpha, sc->omega));
    }
    if (rho.x == 0.0 && rho.y == 0.0) stop = 1;
    sc->rho[q] = rho;
    sc->rr = rr;
    sc->stopped[q] = stop;
}

// Workgroup partials (a, b) over 256-entry chunks: partials A of <rh, r>,
// |r|^2, B of <rh, v> and C of <t, s>, |t|^2
__device__ __forceinline__ void chunk_partials(double2 a, double b, double2* partials) {
    __shared__ double red[3][4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    a = make_double2(wave_sum(a.x), wave_sum(a.y));
    b = wave_sum(b);
    if (lane == 0) {
        red[0][wave] = a.x;
        red[1][wave] = a.y;
        red[2][wave] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[(size_t)blockIdx.x * 2] = make_double2((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]),
                                                        (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
        partials[(size_t)blockIdx.x * 2 + 1] =
            make_double2((red[2][0] + red[2][1]) + (red[2][2] + red[2][3]), 0.0);
    }
}

template <bool HALF, int NC>
__global__ __launch_bounds__(CMV_TPB) void k_cb_m1(Geom g, const void* __restrict__ Dc, int nc, CbVecs cv,
                                                   const CbScalars* sc, int q) {
    if (sc->stopped[q]) return;
    __shared__ float2 xs[CMV_KMAX];
    __shared__ float2 red[CMV_TPB];
    const int a = blockIdx.x, K5 = 5 * nc;
    const BlockPos p = block_pos(g, a);
    const float br = (float)sc->beta[q].x, bi = (float)sc->beta[q].y;
    const float wr = (float)sc->omega.x, wi = (float)sc->omega.y;
    const float2 *pp = cv.p[q ^ 1], *vp = cv.v[q ^ 1];
    float2* pn = cv.p[q];
    for (int k = threadIdx.x; k < K5; k += CMV_TPB) {
        const size_t i = gather_index(g, p, nc, k);
        const float2 r = cv.r[i], po = pp[i], vo = vp[i];
        const float tr = po.x - (wr * vo.x - wi * vo.y), ti = po.y - (wr * vo.y + wi * vo.x);
        const float2 pv = make_float2(r.x + (br * tr - bi * ti), r.y + (br * ti + bi * tr));
        xs[k] = pv;
        if (k < nc) pn[i] = pv;
    }
    __syncthreads();
    const float2 v = cmv5<HALF, NC>(Dc, a, nc, xs, red, cv.tau);
    if ((int)threadIdx.x < nc) cv.v[q][(size_t)a * nc + threadIdx.x] = v;
}

// v += the +mu terms, partials B of <rh, v>
__global__ __launch_bounds__(256) void k_cb_c1(Geom g, int nc, CbVecs cv, const CbScalars* sc, int q,
                                               double2* partials) {
    if (sc->stopped[q]) return;
    const size_t n = (size_t)g.nblk * nc;
    float2* vq = cv.v[q];
    double2 d = make_double2(0.0, 0.0);
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float2 t = tau_sum(g, nc, cv.tau, i), v0 = vq[i];
        const float2 v = make_float2(v0.x + t.x, v0.y + t.y);
        vq[i] = v;
        const double2 hv = cdot_d(cv.rh[i], v);
        d.x += hv.x;
        d.y += hv.y;
    }
    chunk_partials(d, 0.0, partials);
}

__global__ __launch_bounds__(1024) void k_cb_f2(const double2* partials, int nwg, CbScalars* sc, int q) {
    if (sc->stopped[q]) return;
    double tot[3];
    sum3_partials(partials, nwg, tot);
    if (threadIdx.x != 0) return;
    const double2 rv = make_double2(tot[0], tot[1]);
    const bool brk = rv.x == 0.0 && rv.y == 0.0;
    sc->brk[q] = brk;
    if (!brk) sc->alpha = cdiv2(sc->rho[q], rv);
}

template <bool HALF, int NC>
__global__ __launch_bounds__(CMV_TPB) void k_cb_m2(Geom g, const void* __restrict__ Dc, int nc, CbVecs cv,
                                                   const CbScalars* sc, int q) {
    if (sc->stopped[q] || sc->brk[q]) return;
    __shared__ float2 xs[CMV_KMAX];
    __shared__ float2 red[CMV_TPB];
    const int a = blockIdx.x, K5 = 5 * nc;
    const BlockPos p = block_pos(g, a);
    const float ar = (float)sc->alpha.x, ai = (float)sc->alpha.y;
    const float2* vq = cv.v[q];
    for (int k = threadIdx.x; k < K5; k += CMV_TPB) {
        const size_t i = gather_index(g, p, nc, k);
        const float2 r = cv.r[i], v = vq[i];
        const float2 sv = make_float2(r.x - (ar * v.x - ai * v.y), r.y - (ar * v.y + ai * v.x));
        xs[k] = sv;
        if (k < nc) cv.s[i] = sv;
    }
    __syncthreads();
    const float2 tv = cmv5<HALF, NC>(Dc, a, nc, xs, red, cv.tau);
    if ((int)threadIdx.x < nc) cv.t[(size_t)a * nc + threadIdx.x] = tv;
}

// t += the +mu terms, partials C of <t, s>, |t|^2
__global__ __launch_bounds__(256) void k_cb_c2(Geom g, int nc, CbVecs cv, const CbScalars* sc, int q,
                                               double2* partials) {
    if (sc->stopped[q] || sc->brk[q]) return;
    const size_t n = (size_t)g.nblk * nc;
    double2 ts = make_double2(0.0, 0.0);
    double tt = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float2 u = tau_sum(g, nc, cv.tau, i), t0 = cv.t[i];
        const float2 t = make_float2(t0.x + u.x, t0.y + u.y);
        cv.t[i] = t;
        const double2 d = cdot_d(t, cv.s[i]);
        ts.x += d.x;
        ts.y += d.y;
        tt += (double)t.x * t.x + (double)t.y * t.y;
    }
    chunk_partials(ts, tt, partials);
}

__global__ __launch_bounds__(1024) void k_cb_f3(const double2* partials, int nwg, CbScalars* sc, int q) {
    if (sc->stopped[q] || sc->brk[q]) return;
    double tot[3];
    sum3_partials(partials, nwg, tot);
    if (threadIdx.x != 0) return;
    const double tt = tot[2];
    sc->omega = tt > 0.0 ? make_double2(tot[0] / tt, tot[1] / tt) : make_double2(0.0, 0.0);
}

// x = 0, r = rh = rc, p_prev = v_prev = 0 (slot 1), partials A
__global__ __launch_bounds__(256) void k_cb_init(int n, const float2* rc, CbVecs cv, double2* partials) {
    double2 a = make_double2(0.0, 0.0);
    double b = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float2 r = rc[i];
        cv.x[i] = cv.p[1][i] = cv.v[1][i] = make_float2(0.f, 0.f);
        cv.r[i] = cv.rh[i] = r;
        const double rr = (double)r.x * r.x + (double)r.y * r.y;
        a.x += rr;
        b += rr;
    }
    chunk_partials(a, b, partials);
}

__global__ __launch_bounds__(256) void k_cb_update(int n, const CbScalars* sc, int q, CbVecs cv,
                                                   double2* partials) {
    if (sc->stopped[q] || sc->brk[q]) return;
    const float ar = (float)sc->alpha.x, ai = (float)sc->alpha.y, wr = (float)sc->omega.x, wi = (float)sc->omega.y;
    const float2* pq = cv.p[q];
    double2 a = make_double2(0.0, 0.0);
    double b = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float2 x = cv.x[i], p = pq[i], s = cv.s[i], t = cv.t[i], h = cv.rh[i];
        cv.x[i] = make_float2(x.x + (ar * p.x - ai * p.y) + (wr * s.x - wi * s.y),
                              x.y + (ar * p.y + ai * p.x) + (wr * s.y + wi * s.x));
        const float2 r = make_float2(s.x - (wr * t.x - wi * t.y), s.y - (wr * t.y + wi * t.x));
        cv.r[i] = r;
        const double2 hr = cdot_d(h, r);
        a.x += hr.x;
        a.y += hr.y;
        b += (double)r.x * r.x + (double)r.y * r.y;
    }
    chunk_partials(a, b, partials);
}

// FP16 copy of the FP32 coarse matrices
__global__ __launch_bounds__(256) void k_mg_dc_half(const float2* __restrict__ src, unsigned int* __restrict__ dst,
                                                    size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float2 v = src[i];
        dst[i] = pack2<P_F16>(v.x, v.y);
    }
}

int cb_grid(int n) {
    const int b = (n + 255) / 256;
    return b < MG_ELEM_WG ? b : MG_ELEM_WG;
}

// f(half, nc) with the storage flag and the product's nc as compile-time
// constants: 16, 32 and 64 take the fused pass 1, other sizes NC = 0
template <typename F>
void with_nc(int nc, bool half, F&& f) {
    auto go = [&](auto h) {
        switch (nc) {
        case 16: f(h, std::integral_constant<int, 16>{}); break;
        case 32: f(h, std::integral_constant<int, 32>{}); break;
        case 64: f(h, std::integral_constant<int, 64>{}); break;
        default: f(h, std::integral_constant<int, 0>{}); break;
        }
    };
    if (half) go(std::true_type{});
    else go(std::false_type{});
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
    hipLaunchKernelGGL(k_mg_assemble, dim3(op.g.nblk * 2 * nv), dim3(TPB), 0, s, op.g, op.links[P_F32], op.clover32,
                       (float)op.kappa, (const char*)P, spinor_bytes_per_site(P_F32) * op.g.V, nv, Dc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mg_assemble_fwd, dim3(op.g.nblk, 4), dim3(TPB), 0, s, op.g, nv, Dc);
    return hipGetLastError();
}

hipError_t mg_restrict(const Geom& g, Transfer T, int nv, const void* r, float2* rc, hipStream_t s) {
    ProfScope ps("mg", s);
    const size_t fs = spinor_bytes_per_site(T.prec) * g.V;
    if (T.prec == P_F16)
        hipLaunchKernelGGL(k_mg_restrict<P_F16>, dim3(g.nblk), dim3(TPB), 0, s, g, (const char*)T.P, fs, nv, r, rc);
    else
        hipLaunchKernelGGL(k_mg_restrict<P_F32>, dim3(g.nblk), dim3(TPB), 0, s, g, (const char*)T.P, fs, nv, r, rc);
    return hipGetLastError();
}

hipError_t mg_prolong(const Geom& g, Transfer T, int nv, const float2* ec, void* z, hipStream_t s) {
    ProfScope ps("mg", s);
    const size_t fs = spinor_bytes_per_site(T.prec) * g.V;
    if (T.prec == P_F16)
        hipLaunchKernelGGL(k_mg_prolong<P_F16>, dim3(g.nblk), dim3(TPB), 0, s, g, (const char*)T.P, fs, nv, ec, z);
    else
        hipLaunchKernelGGL(k_mg_prolong<P_F32>, dim3(g.nblk), dim3(TPB), 0, s, g, (const char*)T.P, fs, nv, ec, z);
    return hipGetLastError();
}

hipError_t mg_restrict_many(const Geom& g, Transfer T, int nv, const void* r, int nr, float2* rc,
                            hipStream_t s) {
    ProfScope ps("mg", s);
    constexpr int R = 4;
    const size_t fs = spinor_bytes_per_site(T.prec) * g.V, rs = spinor_bytes_per_site(P_F32) * g.V;
    const size_t rcs = (size_t)g.nblk * 2 * nv;
    const dim3 grid(g.nblk, (nr + R - 1) / R);
    if (T.prec == P_F16)
        hipLaunchKernelGGL((k_mg_restrict_many<P_F16, R>), grid, dim3(TPB), 0, s, g, (const char*)T.P, fs, nv,
                           (const char*)r, rs, nr, rc, rcs);
    else
        hipLaunchKernelGGL((k_mg_restrict_many<P_F32, R>), grid, dim3(TPB), 0, s, g, (const char*)T.P, fs, nv,
                           (const char*)r, rs, nr, rc, rcs);
    return hipGetLastError();
}

hipError_t mg_prolong_many(const Geom& g, Transfer T, int nv, const float2* ec, int nr, void* z, hipStream_t s) {
    ProfScope ps("mg", s);
    constexpr int R = 4;
    const size_t fs = spinor_bytes_per_site(T.prec) * g.V, zs = spinor_bytes_per_site(P_F32) * g.V;
    const size_t ecs = (size_t)g.nblk * 2 * nv;
    const dim3 grid(g.nblk, (nr + R - 1) / R);
    if (T.prec == P_F16)
        hipLaunchKernelGGL((k_mg_prolong_many<P_F16, R>), grid, dim3(TPB), 0, s, g, (const char*)T.P, fs, nv, ec,
                           ecs, nr, (char*)z, zs);
    else
        hipLaunchKernelGGL((k_mg_prolong_many<P_F32, R>), grid, dim3(TPB), 0, s, g, (const char*)T.P, fs, nv, ec,
                           ecs, nr, (char*)z, zs);
    return hipGetLastError();
}

hipError_t mg_coarse_half(const float2* Dc, void* Dc16, size_t n, hipStream_t s) {
    ProfScope ps("mg", s);
    const size_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_mg_dc_half, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(256), 0, s, Dc, (unsigned int*)Dc16,
                       n);
    return hipGetLastError();
}

hipError_t mg_coarse_apply(const Geom& g, CoarseMat M, int nc, const float2* x, float2* y, float2* tau,
                           hipStream_t s) {
    ProfScope ps("mg", s);
    with_nc(nc, M.half, [&](auto half, auto ncc) {
        hipLaunchKernelGGL((k_mg_coarse_apply<decltype(half)::value, decltype(ncc)::value>), dim3(g.nblk),
                           dim3(CMV_TPB), 0, s, g, M.m, nc, x, y, tau);
    });
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mg_coarse_complete, dim3(cb_grid(g.nblk * nc)), dim3(256), 0, s, g, nc, y, tau);
    return hipGetLastError();
}

#define CB_CHECK()                               \
    do {                                         \
        hipError_t e_ = hipGetLastError();       \
        if (e_ != hipSuccess) return e_;         \
    } while (0)
#define CB_LAUNCH(...)                           \
    do {                                         \
        hipLaunchKernelGGL(__VA_ARGS__);         \
        CB_CHECK();                              \
    } while (0)

hipError_t mg_coarse_begin(const Geom& g, int nc, const float2* rc, const CbVecs& cv, CbScalars* sc,
                           const CbPartials& pa, double tol, hipStream_t s) {
    ProfScope ps("mg", s);
    const int n = g.nblk * nc, grid = cb_grid(n);
    CB_LAUNCH(k_cb_init, dim3(grid), dim3(256), 0, s, n, rc, cv, pa.A);
    CB_LAUNCH(k_cb_f1, dim3(1), dim3(1024), 0, s, pa.A, grid, sc, 0, tol * tol);
    return hipSuccess;
}

hipError_t mg_coarse_iters(const Geom& g, CoarseMat M, int nc, const CbVecs& cv, CbScalars* sc,
                           const CbPartials& pa, int it0, int it1, hipStream_t s) {
    ProfScope ps("mg", s);
    const int n = g.nblk * nc, grid = cb_grid(n);
    for (int it = it0; it < it1; ++it) {
        const int q = it & 1;
        with_nc(nc, M.half, [&](auto half, auto ncc) {
            hipLaunchKernelGGL((k_cb_m1<decltype(half)::value, decltype(ncc)::value>), dim3(g.nblk), dim3(CMV_TPB),
                               0, s, g, M.m, nc, cv, sc, q);
        });
        CB_CHECK();
        CB_LAUNCH(k_cb_c1, dim3(grid), dim3(256), 0, s, g, nc, cv, sc, q, pa.B);
        CB_LAUNCH(k_cb_f2, dim3(1), dim3(1024), 0, s, pa.B, grid, sc, q);
        with_nc(nc, M.half, [&](auto half, auto ncc) {
            hipLaunchKernelGGL((k_cb_m2<decltype(half)::value, decltype(ncc)::value>), dim3(g.nblk), dim3(CMV_TPB),
                               0, s, g, M.m, nc, cv, sc, q);
        });
        CB_CHECK();
        CB_LAUNCH(k_cb_c2, dim3(grid), dim3(256), 0, s, g, nc, cv, sc, q, pa.C);
        CB_LAUNCH(k_cb_f3, dim3(1), dim3(1024), 0, s, pa.C, grid, sc, q);
        CB_LAUNCH(k_cb_update, dim3(grid), dim3(256), 0, s, n, sc, q, cv, pa.A);
        CB_LAUNCH(k_cb_f1, dim3(1), dim3(1024), 0, s, pa.A, grid, sc, it + 1, 0.0);
    }
    return hipSuccess;
}

#undef CB_LAUNCH
#undef CB_CHECK

hipError_t mg_coarse_bicgstab(const Geom& g, CoarseMat M, int nc, const float2* rc, const CbVecs& cv,
                              CbScalars* sc, const CbPartials& pa, int max_iter, double tol, hipStream_t s) {
    hipError_t e = mg_coarse_begin(g, nc, rc, cv, sc, pa, tol, s);
    if (e != hipSuccess) return e;
    return mg_coarse_iters(g, M, nc, cv, sc, pa, 0, max_iter, s);
}

}  // namespace cs
