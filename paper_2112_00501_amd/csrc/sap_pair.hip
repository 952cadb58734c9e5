// SAP half-sweep with two lanes per site (FP32 arithmetic; FP32, FP16 or
// BF16 storage).  The visit of a block is the one of the one-lane kernel in
// sap.hip (block residual from the full operator, n_mr minimal-residual steps
// on the Dirichlet block operator out of LDS, x_B += delta); the work of a
// site is split over a lane pair so that a block has twice the lanes and each
// lane half the dependent arithmetic:
//   * lanes l and l ^ 32 of a wave hold the same site; lane half h = 0 sums
//     the four forward hops (1 - gamma_mu) U_mu(x) psi(x + mu), h = 1 the four
//     backward hops (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu).  The two
//     differ only in the sign S of (1 + S gamma_mu) and in U against U^dag,
//     so both halves of a wave run one instruction stream;
//   * the partners then exchange half-spinors: h = 0 keeps the upper
//     chirality (spins 0, 1), h = 1 the lower one, applies that chirality's
//     6x6 block of the clover term (the term is block diagonal in chirality),
//     and holds that half of rho, q and delta.
#include "dslash_core.hpp"
#include "wave.hpp"

namespace cs {

namespace {

constexpr int PAIR_TPB = 2 * BLOCK_SITES;

struct PairLane {
    int l;     // site in the block
    int h;     // 0: forward hops, upper chirality; 1: backward hops, lower chirality
    float sg;  // S of (1 + S gamma_mu): -1 forward, +1 backward
};

__device__ __forceinline__ PairLane pair_lane() {
    const int t = threadIdx.x, lane = t & 63;
    PairLane q;
    q.h = lane >> 5;
    q.l = (t >> 6) * 32 + (lane & 31);
    q.sg = q.h ? 1.f : -1.f;
    return q;
}

// LDS of one block.  rho rows have RHO_STRIDE sites so that row offsets stay
// multiples of 512 bytes (one immediate offset pairs two rows); site
// ZERO_SITE of every row holds zero and is never written, so a lane whose
// neighbour lies outside the block reads zeros instead of branching.  The
// links are kept whole (all three rows), rebuilt once when staged.
constexpr int RHO_STRIDE = BLOCK_SITES + 64;
constexpr int ZERO_SITE = BLOCK_SITES;

struct PairSmem {
    lds_cpx<float> rho[12][RHO_STRIDE];      // rho (or the staged x) of the whole block
    lds_cpx<float> u[4][9][BLOCK_SITES];     // the block's links
    float red[3][PAIR_TPB / 64];
};

// Neighbour of site l in direction MU: forward for h = 0, backward for h = 1.
template <int MU>
__device__ __forceinline__ void pair_neighbour(const Geom& g, const BlockPos& p, const PairLane& q, int* nb,
                                               int* nl, bool* in) {
    constexpr int sh = 2 * MU;
    const int lc = (q.l >> sh) & 3;
    const bool fwd = q.h == 0;
    const bool inside = fwd ? lc < 3 : lc > 0;
    *in = inside;
    *nl = inside ? (fwd ? q.l + (1 << sh) : q.l - (1 << sh)) : (fwd ? q.l - (3 << sh) : q.l + (3 << sh));
    const int up = p.bc[MU] == g.NB[MU] - 1 ? p.blk - (g.NB[MU] - 1) * p.stride[MU] : p.blk + p.stride[MU];
    const int dn = p.bc[MU] == 0 ? p.blk + (g.NB[MU] - 1) * p.stride[MU] : p.blk - p.stride[MU];
    *nb = inside ? p.blk : (fwd ? up : dn);
}

// acc += (1 + S gamma_mu) M psi with M = U (h = 0) or U^dag (h = 1) and S the
// lane's sign; u holds the full 3x3 link.  Chiral basis, gamma_mu =
// [[0, A],[A^dag, 0]] with A_x = -i s1, A_y = -i s2, A_z = -i s3, A_t = 1:
// the upper half of (1 + S gamma_mu) psi is hh = psi_up + S A psi_lo and the
// lower half is S A^dag hh.
// FIRST: acc holds nothing yet and is set rather than added to.
template <int MU, bool FIRST = false>
__device__ __forceinline__ void pair_hop(const cpx<float>* u, int h, float sg, const cpx<float>* psi,
                                         cpx<float>* acc) {
    cpx<float> hh[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cpx<float> s0 = psi[a], s1 = psi[3 + a], s2 = psi[6 + a], s3 = psi[9 + a];
        cpx<float> a0, a1;  // A psi_lo
        if (MU == 0) { a0 = mul_mi(s3); a1 = mul_mi(s2); }
        else if (MU == 1) { a0 = {-s3.re, -s3.im}; a1 = s2; }
        else if (MU == 2) { a0 = mul_mi(s2); a1 = mul_i(s3); }
        else { a0 = s2; a1 = s3; }
        hh[a] = {fmaf(sg, a0.re, s0.re), fmaf(sg, a0.im, s0.im)};
        hh[3 + a] = {fmaf(sg, a1.re, s1.re), fmaf(sg, a1.im, s1.im)};
    }
    cpx<float> v[6];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cpx<float> t = {0.f, 0.f};
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                // M[a][b] = U[a][b] or conj(U[b][a]), chosen per lane
                const cpx<float> d = u[a * 3 + b], e = u[b * 3 + a];
                const cpx<float> m = {h ? e.re : d.re, h ? -e.im : d.im};
                cmac(t, m, hh[3 * s + b]);
            }
            v[3 * s + a] = t;
        }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cpx<float> v0 = v[a], v1 = v[3 + a];
        cpx<float> b0, b1;  // A^dag v
        if (MU == 0) { b0 = mul_i(v1); b1 = mul_i(v0); }
        else if (MU == 1) { b0 = v1; b1 = {-v0.re, -v0.im}; }
        else if (MU == 2) { b0 = mul_i(v0); b1 = mul_mi(v1); }
        else { b0 = v0; b1 = v1; }
        if constexpr (FIRST) {
            acc[a] = v0;
            acc[3 + a] = v1;
            acc[6 + a] = {sg * b0.re, sg * b0.im};
            acc[9 + a] = {sg * b1.re, sg * b1.im};
        } else {
            acc[a] = acc[a] + v0;
            acc[3 + a] = acc[3 + a] + v1;
            acc[6 + a] = {fmaf(sg, b0.re, acc[6 + a].re), fmaf(sg, b0.im, acc[6 + a].im)};
            acc[9 + a] = {fmaf(sg, b1.re, acc[9 + a].re), fmaf(sg, b1.im, acc[9 + a].im)};
        }
    }
}

// Hop in direction MU inside the block: psi from LDS, the link from LDS
// (U_mu(x) for forward lanes, U_mu(x - mu) at the neighbour for backward
// ones).  A lane whose neighbour is outside the block reads the zero site and
// adds nothing; no lane branches.
template <int MU, bool FIRST = false>
__device__ __forceinline__ void pair_hop_lds(const Geom& g, const BlockPos& p, const PairLane& q,
                                             const PairSmem& sm, cpx<float>* acc) {
    int nb, nl;
    bool in;
    pair_neighbour<MU>(g, p, q, &nb, &nl, &in);
    const int sl = in ? nl : ZERO_SITE;
    cpx<float> psi[12], u[9];
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k] = sm.rho[k][sl].get();
    const int li = q.h ? nl : q.l;
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = sm.u[MU][k][li].get();
    pair_hop<MU, FIRST>(u, q.h, q.sg, psi, acc);
}

// The four hops inside the block, acc set by the first.
__device__ __forceinline__ void pair_hops_lds(const Geom& g, const BlockPos& p, const PairLane& q,
                                              const PairSmem& sm, cpx<float>* acc) {
    pair_hop_lds<0, true>(g, p, q, sm, acc);
    pair_hop_lds<1>(g, p, q, sm, acc);
    pair_hop_lds<2>(g, p, q, sm, acc);
    pair_hop_lds<3>(g, p, q, sm, acc);
}

// Hops in directions MA and MB that leave the block, from global memory (the
// neighbouring blocks have the other colour and are not written by this
// launch).  Every lane issues the loads of both directions before either is
// applied; lanes without a face neighbour read their own site, which is
// cached.  A forward lane reads its own link U_mu(x), a backward one the
// neighbour block's U_mu(x - mu).
template <int MU, int P, int PLINK>
__device__ __forceinline__ void pair_face_load(const Geom& g, const BlockPos& p, const PairLane& q,
                                               const void* xr, const void* links, cpx<float>* psi,
                                               cpx<float>* u, bool* face) {
    int nb, nl;
    bool in;
    pair_neighbour<MU>(g, p, q, &nb, &nl, &in);
    *face = !in;
    const int sb = in ? p.blk : nb, sl = in ? q.l : nl;
    using RS = typename SpinorIO<P>::R;
    cpx<RS> t[12];
    SpinorIO<P>::load(xr, g.nblk, sb, sl, t);
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k] = {(float)t[k].re, (float)t[k].im};
    if (MU == 3)
        time_boundary_phase(g, !in && (q.h == 0 ? p.bc[3] == g.NB[3] - 1 : p.bc[3] == 0), &psi[0].re, 24);
    const bool nbr_link = !in && q.h == 1;
    load_link<PLINK, float, false>(links, nbr_link ? nb : p.blk, nbr_link ? nl : q.l, MU, u);
}

template <int MA, int MB, int P, int PLINK>
__device__ __forceinline__ void pair_faces(const Geom& g, const BlockPos& p, const PairLane& q, const void* xr,
                                           const void* links, cpx<float>* acc) {
    cpx<float> pa[12], ua[9], pb[12], ub[9];
    bool fa, fb;
    pair_face_load<MA, P, PLINK>(g, p, q, xr, links, pa, ua, &fa);
    pair_face_load<MB, P, PLINK>(g, p, q, xr, links, pb, ub, &fb);
    if (fa) pair_hop<MA>(ua, q.h, q.sg, pa, acc);
    if (fb) pair_hop<MB>(ub, q.h, q.sg, pb, acc);
}

// The hop sum of the site: own chirality half of (this lane's sum + the
// partner's sum).  Every lane of the wave must call it.
__device__ __forceinline__ void pair_combine(const cpx<float>* acc, cpx<float>* mine) {
#pragma unroll
    for (int i = 0; i < 6; ++i)
        mine[i] = {pair_split_sum(acc[i].re, acc[6 + i].re), pair_split_sum(acc[i].im, acc[6 + i].im)};
}

// Full spinor of the site from the two halves.  Every lane of the wave must call it.
__device__ __forceinline__ void pair_gather(const cpx<float>* half, cpx<float>* full) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        pair_share(half[i].re, full[i].re, full[6 + i].re);
        pair_share(half[i].im, full[i].im, full[6 + i].im);
    }
}

// Own chirality half of a stored spinor.
template <int P>
__device__ __forceinline__ void load_half(const void* base, int nblk, int blk, const PairLane& q, cpx<float>* v) {
    if constexpr (P == P_F32) {
        const float4* p = (const float4*)base + ((size_t)blk * 6 + 3 * q.h) * BLOCK_SITES + q.l;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float4 t = p[k * BLOCK_SITES];
            v[2 * k] = {t.x, t.y};
            v[2 * k + 1] = {t.z, t.w};
        }
    } else {
        cpx<float> t[12];
        SpinorIO<P>::load(base, nblk, blk, q.l, t);
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] = q.h ? t[6 + i] : t[i];
    }
}

// x_B = (add: x_B +) delta, delta given as this lane's chirality half; x_B
// is read again here rather than kept in registers through the block solve.
// Every lane of the wave must call it.
template <int P>
__device__ __forceinline__ void store_update(void* base, int nblk, int blk, const PairLane& q, bool add,
                                             const cpx<float>* delta) {
    if constexpr (P == P_F32) {
        cpx<float> o[6];
        if (add) {
            load_half<P>(base, nblk, blk, q, o);
#pragma unroll
            for (int i = 0; i < 6; ++i) o[i] = o[i] + delta[i];
        } else {
#pragma unroll
            for (int i = 0; i < 6; ++i) o[i] = delta[i];
        }
        float4* p = (float4*)base + ((size_t)blk * 6 + 3 * q.h) * BLOCK_SITES + q.l;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            p[k * BLOCK_SITES] = make_float4(o[2 * k].re, o[2 * k].im, o[2 * k + 1].re, o[2 * k + 1].im);
    } else {
        // the per-site scale covers all 24 reals: lane half 0 writes the site
        cpx<float> full[12];
        pair_gather(delta, full);
        if (q.h == 0) {
            if (add) {
                cpx<float> t[12];
                SpinorIO<P>::load(base, nblk, blk, q.l, t);
#pragma unroll
                for (int k = 0; k < 12; ++k) full[k] = full[k] + t[k];
            }
            SpinorIO<P>::store(base, nblk, blk, q.l, full);
        }
    }
}

// Chirality block h of 1 + T: 6 diagonal reals, then the 15 upper entries.
__device__ __forceinline__ void load_clover_half(const void* base, int blk, const PairLane& q, float* c) {
    const float4* p = (const float4*)base + ((size_t)blk * 18 + 9 * q.h) * BLOCK_SITES + q.l;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const float4 v = p[k * BLOCK_SITES];
        c[4 * k] = v.x;
        c[4 * k + 1] = v.y;
        c[4 * k + 2] = v.z;
        c[4 * k + 3] = v.w;
    }
}

__device__ __forceinline__ void clover_apply_half(const float* d, const cpx<float>* v, cpx<float>* o) {
    const float* up = d + 6;
#pragma unroll
    for (int i = 0; i < 6; ++i) o[i] = d[i] * v[i];
    int k = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j, ++k) {
            const cpx<float> a = {up[2 * k], up[2 * k + 1]};
            cmac(o[i], a, v[j]);       // upper entry (i, j)
            cmac_conj(o[j], a, v[i]);  // its mirror (j, i) = conj
        }
}

// Sum of three values over the workgroup; every lane receives the same total.
__device__ __forceinline__ void pair_sum3(float& a, float& b, float& c, float (*red)[PAIR_TPB / 64]) {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wave] = a;
        red[1][wave] = b;
        red[2][wave] = c;
    }
    __syncthreads();
    a = ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3])) + ((red[0][4] + red[0][5]) + (red[0][6] + red[0][7]));
    b = ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3])) + ((red[1][4] + red[1][5]) + (red[1][6] + red[1][7]));
    c = ((red[2][0] + red[2][1]) + (red[2][2] + red[2][3])) + ((red[2][4] + red[2][5]) + (red[2][6] + red[2][7]));
}

// BS = BLOCK_JACOBI: the Jacobi form for A = C^-1 D (see k_sap_halfsweep);
// `clover` is then (1 + T)^-1.
template <int P, int PLINK, int BS>
__global__ __launch_bounds__(PAIR_TPB) void k_sap_pair(Geom g, const void* __restrict__ links,
                                                       const void* __restrict__ clover, double kappa_d, int colour,
                                                       int n_mr, int mode, void* __restrict__ x,
                                                       const void* __restrict__ b, size_t stride, int nrhs,
                                                       int tile, int nitems) {
    __shared__ PairSmem sm;
    const PairLane q = pair_lane();
    const int ncb = g.nblk / 2;
    const float kappa = (float)kappa_d;

    if (threadIdx.x < 12) sm.rho[threadIdx.x][ZERO_SITE].set({0.f, 0.f});  // read after the barrier below

    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int w = xcd_remap(item, nitems);
        const int blk = colour_block(g, colour, w % ncb);
        const int r0 = (w / ncb) * tile;
        const int r1 = r0 + tile < nrhs ? r0 + tile : nrhs;
        const BlockPos p = block_pos(g, blk);

        // every global load of the item that does not depend on the
        // right-hand side is issued before the barrier: lane half h stages
        // the links of directions 2h and 2h + 1
        cpx<typename LinkIO<PLINK>::R> lw[2][6];
#pragma unroll
        for (int j = 0; j < 2; ++j) LinkIO<PLINK>::load6(links, blk, q.l, 2 * q.h + j, lw[j]);
        float cl[36];
        load_clover_half(clover, blk, q, cl);
        // keep the clover loads here, in flight with the link loads, rather
        // than sunk towards their first use
#pragma unroll
        for (int k = 0; k < 36; ++k) asm volatile("" ::"v"(cl[k]));
        __syncthreads();  // the previous item's readers of the staged links are done
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            cpx<float> u[9];
#pragma unroll
            for (int k = 0; k < 6; ++k) u[k] = {(float)lw[j][k].re, (float)lw[j][k].im};
            su3_row2(u);
#pragma unroll
            for (int k = 0; k < 9; ++k) sm.u[2 * q.h + j][k][q.l].set(u[k]);
        }

        for (int r = r0; r < r1; ++r) {
            char* xr = (char*)x + (size_t)r * stride;
            const char* br = (const char*)b + (size_t)r * stride;

            // ---- block residual r_B = b_B - (D x)_B
            cpx<float> rho[6], xh[6];
            if (mode == 0) load_half<P>(xr, g.nblk, blk, q, xh);
            {
                cpx<float> hop[6], cx[6];
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    hop[i] = {0.f, 0.f};
                    cx[i] = {0.f, 0.f};
                }
                if (mode != 1) {
                    cpx<float> acc[12];
#pragma unroll
                    for (int k = 0; k < 12; ++k) acc[k] = {0.f, 0.f};
                    if (mode == 0) {  // own x staged in LDS for the hops inside the block
                        __syncthreads();  // the previous right-hand side's readers of rho are done
#pragma unroll
                        for (int i = 0; i < 6; ++i) sm.rho[6 * q.h + i][q.l].set(xh[i]);
                        __syncthreads();
                        pair_hops_lds(g, p, q, sm, acc);
                        if constexpr (BS == BLOCK_MR) clover_apply_half(cl, xh, cx);
                    }
                    pair_faces<0, 1, P, PLINK>(g, p, q, xr, links, acc);
                    pair_faces<2, 3, P, PLINK>(g, p, q, xr, links, acc);
                    pair_combine(acc, hop);
                }
                cpx<float> bh[6];
                load_half<P>(br, g.nblk, blk, q, bh);
                if constexpr (BS == BLOCK_MR) {
#pragma unroll
                    for (int i = 0; i < 6; ++i)
                        rho[i] = {bh[i].re - (cx[i].re - kappa * hop[i].re), bh[i].im - (cx[i].im - kappa * hop[i].im)};
                } else {
                    // rho = C^-1 (b + kappa hop) - x; own x is still staged in LDS
#pragma unroll
                    for (int i = 0; i < 6; ++i) bh[i] = {bh[i].re + kappa * hop[i].re, bh[i].im + kappa * hop[i].im};
                    clover_apply_half(cl, bh, rho);
                    if (mode == 0) {
#pragma unroll
                        for (int i = 0; i < 6; ++i) rho[i] = rho[i] - sm.rho[6 * q.h + i][q.l].get();
                    }
                }
                __syncthreads();  // every lane has read x (or the previous rho) from LDS
#pragma unroll
                for (int i = 0; i < 6; ++i) sm.rho[6 * q.h + i][q.l].set(rho[i]);
            }

            cpx<float> delta[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) delta[i] = {0.f, 0.f};
            if constexpr (BS == BLOCK_JACOBI) {
                // ---- Jacobi steps on A_BB = (C^-1 D)_BB
                if (n_mr > 0) {
#pragma unroll
                    for (int i = 0; i < 6; ++i) delta[i] = rho[i];
                }
                for (int it = 1; it < n_mr; ++it) {
                    __syncthreads();  // delta of the whole block is in LDS
                    cpx<float> acc[12];
                    pair_hops_lds(g, p, q, sm, acc);
                    cpx<float> hop[6];
                    pair_combine(acc, hop);
                    clover_apply_half(cl, hop, delta);
#pragma unroll
                    for (int i = 0; i < 6; ++i)
                        delta[i] = {rho[i].re + kappa * delta[i].re, rho[i].im + kappa * delta[i].im};
                    __syncthreads();  // every lane has read the previous delta
#pragma unroll
                    for (int i = 0; i < 6; ++i) sm.rho[6 * q.h + i][q.l].set(delta[i]);
                }
            }
            // ---- MR on the Dirichlet block operator
            for (int it = 0; BS == BLOCK_MR && it < n_mr; ++it) {
                __syncthreads();  // rho of the whole block is in LDS
                cpx<float> qv[6];
                {
                    cpx<float> acc[12];
                    pair_hops_lds(g, p, q, sm, acc);
                    cpx<float> hop[6];
                    pair_combine(acc, hop);
                    clover_apply_half(cl, rho, qv);
#pragma unroll
                    for (int i = 0; i < 6; ++i)
                        qv[i] = {qv[i].re - kappa * hop[i].re, qv[i].im - kappa * hop[i].im};
                }
                float qq = 0.f, qr_re = 0.f, qr_im = 0.f;
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    qq = fmaf(qv[i].re, qv[i].re, qq);
                    qq = fmaf(qv[i].im, qv[i].im, qq);
                    // conj(q) * rho
                    qr_re = fmaf(qv[i].re, rho[i].re, qr_re);
                    qr_re = fmaf(qv[i].im, rho[i].im, qr_re);
                    qr_im = fmaf(qv[i].re, rho[i].im, qr_im);
                    qr_im = fmaf(-qv[i].im, rho[i].re, qr_im);
                }
                pair_sum3(qq, qr_re, qr_im, sm.red);  // also: every lane is done reading rho
                if (qq == 0.f) break;                 // rho = 0: the block is solved (uniform branch)
                const float inv = 1.f / qq;
                const cpx<float> alpha = {qr_re * inv, qr_im * inv};
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    cmac(delta[i], alpha, rho[i]);
                    cpx<float> t = rho[i];
                    t.re = fmaf(-alpha.re, qv[i].re, t.re);
                    t.re = fmaf(alpha.im, qv[i].im, t.re);
                    t.im = fmaf(-alpha.re, qv[i].im, t.im);
                    t.im = fmaf(-alpha.im, qv[i].re, t.im);
                    rho[i] = t;
                    sm.rho[6 * q.h + i][q.l].set(t);
                }
            }

            // ---- x_B (+)= delta; own block only, which no other lane reads from HBM
            store_update<P>(xr, g.nblk, blk, q, mode == 0, delta);
        }
    }
}

template <int P, int PLINK>
hipError_t launch_pair(const OpData& op, int colour, int n_mr, int mode, void* x, const void* b, int nrhs,
                       const LaunchCfg& cfg, hipStream_t s, int bs) {
    const int tile = cfg.rhs_tile < 1 ? 1 : (cfg.rhs_tile > nrhs ? nrhs : cfg.rhs_tile);
    const int nitems = (op.g.nblk / 2) * ((nrhs + tile - 1) / tile);
    const int grid = cfg.persistent_wgs > 0 && cfg.persistent_wgs < nitems ? cfg.persistent_wgs : nitems;
    const size_t stride = spinor_bytes_per_site(P) * op.g.V;
    if (bs == BLOCK_JACOBI)
        hipLaunchKernelGGL((k_sap_pair<P, PLINK, BLOCK_JACOBI>), dim3(grid), dim3(PAIR_TPB), 0, s, op.g,
                           op.links[PLINK], op.cinv32, op.kappa, colour, n_mr, mode, x, b, stride, nrhs, tile, nitems);
    else
        hipLaunchKernelGGL((k_sap_pair<P, PLINK, BLOCK_MR>), dim3(grid), dim3(PAIR_TPB), 0, s, op.g,
                           op.links[PLINK], op.clover32, op.kappa, colour, n_mr, mode, x, b, stride, nrhs, tile,
                           nitems);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sap_pair(const OpData& op, int prec, int colour, int n_mr, int mode, void* x, const void* b,
                           int nrhs, const LaunchCfg& cfg, hipStream_t s, int bs) {
    switch (prec) {
    case P_F32: return launch_pair<P_F32, P_F32>(op, colour, n_mr, mode, x, b, nrhs, cfg, s, bs);
    case P_F16: return launch_pair<P_F16, P_F16>(op, colour, n_mr, mode, x, b, nrhs, cfg, s, bs);
    case P_BF16: return launch_pair<P_BF16, P_BF16>(op, colour, n_mr, mode, x, b, nrhs, cfg, s, bs);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace cs
