// One half-sweep of the multiplicative red/black Schwarz smoother (paper
// Section 2: domains are updated in turn, each with a fixed number of
// block-solver iterations).  One workgroup owns one 4^4 block of the current
// colour; one lane owns one site.  Per block:
//   r_B = b_B - (D x)_B          full operator; the neighbouring blocks all
//                                have the other colour, so they are not being
//                                written by this launch (no races, no atomics)
//   delta = 0, rho = r_B
//   n_mr times:  q = D_BB rho    Dirichlet block operator, rho and the links
//                                read from LDS, the clover term from registers
//                alpha = <q, rho> / <q, q>   (workgroup reductions)
//                delta += alpha rho,  rho -= alpha q
//   x_B += delta
// HBM traffic per site: b, x, the face neighbours of x, the links and the
// clover term once, and x once written.  All MR iterations run out of LDS
// and registers.
#include <type_traits>

#include "dslash_core.hpp"
#include "wave.hpp"

namespace cs {

namespace {

// Rows 0 and 1 of the block's links, kept in LDS in float for the MR loop.
template <bool ON>
struct LinkSmem { lds_cpx<float> u[4][6][BLOCK_SITES]; };
template <>
struct LinkSmem<false> { lds_cpx<float> u[1][1][1]; };

template <typename R>
struct LdsSpinor {  // in-block neighbours of the Dirichlet operator
    lds_cpx<R> (*s)[BLOCK_SITES];
    __device__ __forceinline__ bool want(bool inside) const { return inside; }
    template <typename RR>
    __device__ __forceinline__ void load_nb(int, int l, bool, cpx<RR>* c) const {
#pragma unroll
        for (int k = 0; k < 12; ++k) c[k] = {(RR)s[k][l].re, (RR)s[k][l].im};
    }
};

// Row 2 of the site's own four links, rebuilt once per work item from the
// staged rows and kept in registers: every forward hop inside the block
// uses the own link U_mu(x), so only the backward hops rebuild a row.
struct OwnRow2 {
    cpx<float> r[4][3];
};

// acc += the two hops of direction MU that stay inside the block (Dirichlet
// block operator), neighbours and links read from LDS; the same terms in the
// same order as the general hopping sum
template <int MU, typename R>
__device__ __forceinline__ void block_hop_dir(int l, const LdsSpinor<R>& ls, const LinkSmem<true>& sm,
                                              const OwnRow2& own, cpx<R>* acc) {
    constexpr int sh = 2 * MU;
    const int lc = (l >> sh) & 3;
    if (lc < 3) {  // forward neighbour, own link U_mu(x)
        cpx<R> psi[12], u[9];
        ls.load_nb(0, l + (1 << sh), true, psi);
#pragma unroll
        for (int k = 0; k < 6; ++k) u[k] = {(R)sm.u[MU][k][l].re, (R)sm.u[MU][k][l].im};
#pragma unroll
        for (int k = 0; k < 3; ++k) u[6 + k] = {(R)own.r[MU][k].re, (R)own.r[MU][k].im};
        hop_term<MU, -1>(u, psi, acc);
    }
    if (lc > 0) {  // backward neighbour, its link U_mu(x - mu)
        const int nl = l - (1 << sh);
        cpx<R> psi[12], u[9];
        ls.load_nb(0, nl, true, psi);
#pragma unroll
        for (int k = 0; k < 6; ++k) u[k] = {(R)sm.u[MU][k][nl].re, (R)sm.u[MU][k][nl].im};
        su3_row2(u);
        hop_term<MU, +1>(u, psi, acc);
    }
}

template <typename R>
__device__ __forceinline__ void block_hops(int l, const LdsSpinor<R>& ls, const LinkSmem<true>& sm,
                                           const OwnRow2& own, cpx<R>* acc) {
    block_hop_dir<0>(l, ls, sm, own, acc);
    block_hop_dir<1>(l, ls, sm, own, acc);
    block_hop_dir<2>(l, ls, sm, own, acc);
    block_hop_dir<3>(l, ls, sm, own, acc);
}

// x is zero on the blocks of the current colour: only hops that leave the
// block contribute to D x.
template <int P>
struct OutsideSpinor {
    const void* base;
    int nblk;
    __device__ __forceinline__ bool want(bool inside) const { return !inside; }
    template <typename R>
    __device__ __forceinline__ void load_nb(int blk, int l, bool, cpx<R>* c) const {
        using RS = typename SpinorIO<P>::R;
        cpx<RS> t[12];
        SpinorIO<P>::load(base, nblk, blk, l, t);
#pragma unroll
        for (int k = 0; k < 12; ++k) c[k] = {(R)t[k].re, (R)t[k].im};
    }
};

// Hops that leave the block, for the directions MU0 and MU1 together (a lane
// has at most one face neighbour per direction).  All lanes issue the loads
// (lanes without a face neighbour read their own site, which is in cache) so
// that the loads of both directions are in flight at once.  Only a backward
// hop needs a link from the neighbour block, U_mu(x - mu); the other lanes
// point their link load at their own link, which the block has just staged
// (a cache hit), so no unused link crosses from HBM.
template <int MU, int P, typename R>
__device__ __forceinline__ void face_load(const Geom& g, const BlockPos& p, int l, const void* xr,
                                          const void* links, cpx<R>* psi, cpx<R>* ug, int* kind) {
    const int sh = 2 * MU;
    const int lc = (l >> sh) & 3;
    int nb = p.blk, nl = l;
    *kind = 0;
    if (lc == 3) {
        *kind = 1;
        nl = l - (3 << sh);
        nb = p.bc[MU] == g.NB[MU] - 1 ? p.blk - (g.NB[MU] - 1) * p.stride[MU] : p.blk + p.stride[MU];
    } else if (lc == 0) {
        *kind = 2;
        nl = l + (3 << sh);
        nb = p.bc[MU] == 0 ? p.blk + (g.NB[MU] - 1) * p.stride[MU] : p.blk - p.stride[MU];
    }
    using RS = typename SpinorIO<P>::R;
    cpx<RS> t[12];
    SpinorIO<P>::load(xr, g.nblk, nb, nl, t);
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k] = {(R)t[k].re, (R)t[k].im};
    if (MU == 3)
        time_boundary_phase(g, *kind == 1 ? p.bc[3] == g.NB[3] - 1 : (*kind == 2 && p.bc[3] == 0), &psi[0].re, 24);
    const bool back = *kind == 2;
    load_link<P, R, false>(links, back ? nb : p.blk, back ? nl : l, MU, ug);
}

// acc += the hop across a face of direction MU for a lane on it: the forward
// hop (kind 1) with the lane's own link, the backward hop (kind 2) with
// U_mu(x - mu); ug holds the link face_load fetched.  Used for t, whose faces
// are whole waves.
template <int MU, typename R>
__device__ __forceinline__ void face_apply(int kind, const cpx<R>* psi, const cpx<R>* ug, cpx<R>* acc) {
    if (kind == 1) hop_term<MU, -1>(ug, psi, acc);
    else if (kind == 2) hop_term<MU, +1>(ug, psi, acc);
}

// acc += (1 + S gamma_mu) U' psi with the sign S and the link U' chosen per
// lane: a lane on the +MU face (kind 1) takes the forward hop (S = -1, U),
// a lane on the -MU face (kind 2) the backward hop (S = +1, U^dag), in one
// pass.  For x, y and z a quarter of the lanes of every wave lies on each
// face, so one merged pass replaces two passes at a quarter occupancy each.
// The spin algebra is that of spin_project and spin_reconstruct_add with S
// as a factor.
template <int MU, typename R>
__device__ __forceinline__ void face_apply_merged(int kind, const cpx<R>* psi, const cpx<R>* ug, cpx<R>* acc) {
    if (kind == 0) return;
    const bool fwd = kind == 1;
    const R S = fwd ? (R)-1 : (R)1;
    cpx<R> u[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const cpx<R> t = ug[b * 3 + a];
            u[a * 3 + b] = fwd ? ug[a * 3 + b] : cpx<R>{t.re, -t.im};
        }
    auto axpy = [](cpx<R> y, R a, cpx<R> x) { return cpx<R>{(R)fma(a, x.re, y.re), (R)fma(a, x.im, y.im)}; };
    cpx<R> h[6], v[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cpx<R> s0 = psi[a], s1 = psi[3 + a], s2 = psi[6 + a], s3 = psi[9 + a];
        if (MU == 0) {
            h[a] = axpy(s0, S, mul_mi(s3));
            h[3 + a] = axpy(s1, S, mul_mi(s2));
        } else if (MU == 1) {
            h[a] = axpy(s0, -S, s3);
            h[3 + a] = axpy(s1, S, s2);
        } else if (MU == 2) {
            h[a] = axpy(s0, S, mul_mi(s2));
            h[3 + a] = axpy(s1, S, mul_i(s3));
        } else {
            h[a] = axpy(s0, S, s2);
            h[3 + a] = axpy(s1, S, s3);
        }
    }
    su3_mul_half<false>(u, h, v);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cpx<R> v0 = v[a], v1 = v[3 + a];
        acc[a] = acc[a] + v0;
        acc[3 + a] = acc[3 + a] + v1;
        if (MU == 0) {
            acc[6 + a] = axpy(acc[6 + a], S, mul_i(v1));
            acc[9 + a] = axpy(acc[9 + a], S, mul_i(v0));
        } else if (MU == 1) {
            acc[6 + a] = axpy(acc[6 + a], S, v1);
            acc[9 + a] = axpy(acc[9 + a], -S, v0);
        } else if (MU == 2) {
            acc[6 + a] = axpy(acc[6 + a], S, mul_i(v0));
            acc[9 + a] = axpy(acc[9 + a], S, mul_mi(v1));
        } else {
            acc[6 + a] = axpy(acc[6 + a], S, v0);
            acc[9 + a] = axpy(acc[9 + a], S, v1);
        }
    }
}

template <int MA, int MB, int P, typename R>
__device__ __forceinline__ void face_pair(const Geom& g, const BlockPos& p, int l, const void* xr,
                                          const void* links, cpx<R>* acc) {
    cpx<R> pa[12], ua[9], pb[12], ub[9];
    int ka, kb;
    face_load<MA, P>(g, p, l, xr, links, pa, ua, &ka);
    face_load<MB, P>(g, p, l, xr, links, pb, ub, &kb);
    face_apply_merged<MA>(ka, pa, ua, acc);
    if (MB == 3) face_apply<MB>(kb, pb, ub, acc);
    else face_apply_merged<MB>(kb, pb, ub, acc);
}

// out = M in for a packed clover-format matrix M read from global memory one
// chirality block at a time (36 reals live instead of 72).
template <typename R>
__device__ __forceinline__ void clover_apply_by_chirality(const void* m, int blk, int l, const cpx<R>* in,
                                                          cpx<R>* out) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        R d[36];
        if constexpr (std::is_same<R, double>::value) {
            const double2* p = (const double2*)m + ((size_t)blk * 36 + 18 * h) * BLOCK_SITES + l;
#pragma unroll
            for (int k = 0; k < 18; ++k) {
                const double2 v = p[k * BLOCK_SITES];
                d[2 * k] = v.x;
                d[2 * k + 1] = v.y;
            }
        } else {
            const float4* p = (const float4*)m + ((size_t)blk * 18 + 9 * h) * BLOCK_SITES + l;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const float4 v = p[k * BLOCK_SITES];
                d[4 * k] = v.x;
                d[4 * k + 1] = v.y;
                d[4 * k + 2] = v.z;
                d[4 * k + 3] = v.w;
            }
        }
        const R* up = d + 6;
        const cpx<R>* v = in + 6 * h;
        cpx<R> o[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) o[i] = d[i] * v[i];
        int k = 0;
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i + 1; j < 6; ++j, ++k) {
                const cpx<R> a = {up[2 * k], up[2 * k + 1]};
                cmac(o[i], a, v[j]);
                cmac_conj(o[j], a, v[i]);
            }
#pragma unroll
        for (int i = 0; i < 6; ++i) out[6 * h + i] = o[i];
    }
}

// Site of lane t when the lanes are ordered by parity: lanes 0..127 take the
// even sites of a 4^4 block, 128..255 the odd ones, each in increasing site
// order.  Every x-row of four sites (row m = ly + 4 lz + 16 lt) holds two
// sites of each parity, at lx = q and q + 2 with q = (parity of m) xor the
// wanted parity.
__device__ __forceinline__ int eo_site(int t) {
    const int par = t >> 7, i = t & 127, m = i >> 1, j = i & 1;
    const int q = (((m & 3) + ((m >> 2) & 3) + (m >> 4)) & 1) ^ par;
    return 4 * m + q + 2 * j;
}

// Sum of three values over the 256 lanes; every lane receives the same total.
template <typename R>
__device__ __forceinline__ void block_sum3(R& a, R& b, R& c, R (*red)[4]) {
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
    a = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    b = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    c = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
}

// Work item = (block of the current colour, tile of right-hand sides).  One
// workgroup stages the block's links in LDS and loads its clover term once,
// then runs the visit for each right-hand side of the tile, so links and
// clover are read from HBM once per tile instead of once per right-hand side.
// With gridDim.x < nitems the launch is persistent: workgroups stride over
// the work items.
//
// BS = BLOCK_EO: the same block system D_BB delta = r_B, solved by MR on its
// Schur complement S = C_e - kappa^2 H_eo C_o^-1 H_oe over the even sites of
// the block (right-hand side r_e + kappa H_eo C_o^-1 r_o), then delta_o =
// C_o^-1 (r_o + kappa H_oe delta_e); `cinv` is (1 + T)^-1.  Even and odd
// lanes take turns (hops join opposite parities), and a step costs about two
// hopping sums.
//
// BS = BLOCK_JACOBI: the block system of A = C^-1 D is solved instead, by
// Jacobi steps (A_BB has the identity on its diagonal); `clover` is then
// (1 + T)^-1 and the visit is
//   rho = C^-1 (b + kappa hop(x)) - x_B      (= C^-1 (b - D x)_B)
//   delta = rho;  n_mr - 1 times: delta = rho + kappa C^-1 hop_BB(delta)
//   x_B += delta
// (hop = the hopping sum, D = C - kappa hop), with no reductions.
//
// GEN: the general visit (mode 0, x nonzero everywhere), compiled on its own
// so that its launches carry their own name in a kernel trace; the two
// half-sweeps of a cycle that start from x = 0 (modes 1 and 2) share the
// other instantiation.
template <int P, int PLINK, int BS, bool GEN>
__global__ CS_SAP_BOUNDS void k_sap_halfsweep(Geom g, const void* __restrict__ links,
                                              const void* __restrict__ clover,
                                              const void* __restrict__ cinv, double kappa_d,
                                              int colour, int n_mr, int mode_in, void* __restrict__ x,
                                              const void* __restrict__ b, size_t stride, int nrhs,
                                              int tile, int nitems) {
    using R = typename Arith<P>::R;
    constexpr bool F32PATH = std::is_same<R, float>::value;
    __shared__ lds_cpx<R> s_rho[12][BLOCK_SITES];
    // FP64 Jacobi keeps the block residual in LDS instead of registers (the
    // FP64 kernel runs one workgroup per compute unit either way)
    constexpr bool RHO_LDS = BS == BLOCK_JACOBI && !F32PATH;
    __shared__ lds_cpx<R> s_rho0[RHO_LDS ? 12 : 1][RHO_LDS ? BLOCK_SITES : 1];
    __shared__ LinkSmem<F32PATH> s_lk;
    __shared__ R s_red[3][4];

    // lane -> site; the even-odd solver puts the block's 128 even sites on
    // lanes 0..127 and its odd sites on 128..255, so that its parity phases
    // run on whole waves
    const int l = BS == BLOCK_EO ? eo_site(threadIdx.x) : (int)threadIdx.x;
    const int ncb = g.nblk / 2;
    const R kappa = (R)kappa_d;
    const int mode = GEN ? 0 : mode_in;
    LdsSpinor<R> ls{s_rho};

    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int w = xcd_remap(item, nitems);
        const int blk = colour_block(g, colour, w % ncb);
        const int r0 = (w / ncb) * tile;
        const int r1 = r0 + tile < nrhs ? r0 + tile : nrhs;
        const BlockPos p = block_pos(g, blk);

        __syncthreads();  // the previous item's readers of s_lk are done
#if CS_SAP_PRIO
        // raised wave priority while the visit's loads are issued, so that
        // they go out ahead of the block-solver arithmetic of the other
        // workgroup resident on the compute unit
        __builtin_amdgcn_s_setprio(1);
#endif
        OwnRow2 own;
        if constexpr (F32PATH) {
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                cpx<typename LinkIO<PLINK>::R> u[6];
                LinkIO<PLINK>::load6(links, blk, l, mu, u);
                cpx<float> uf[9];
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    uf[k] = {(float)u[k].re, (float)u[k].im};
                    s_lk.u[mu][k][l].set(uf[k]);
                }
                su3_row2(uf);
#pragma unroll
                for (int k = 0; k < 3; ++k) own.r[mu][k] = uf[6 + k];
            }
        }
        // The FP32 path keeps the clover term in registers for the whole
        // tile; the FP64 one re-reads it (it would not fit next to the MR
        // state).
        R cl[F32PATH ? 72 : 1];
        if constexpr (F32PATH) CloverIO<R>::load(clover, blk, l, cl);

        for (int r = r0; r < r1; ++r) {
            char* xr = (char*)x + (size_t)r * stride;
            const char* br = (const char*)b + (size_t)r * stride;

            // ---- block residual r_B = b_B - (D x)_B (Jacobi: C^-1 r_B), stored as rho in LDS
            cpx<R> rho0[12];
            if constexpr (F32PATH && CS_SAP_LDS_RESIDUAL) {
                // own x staged in LDS: the hops inside the block read it (and
                // the links) from LDS; the face hops read HBM two directions
                // at a time
                cpx<R> acc[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[k] = {(R)0, (R)0};
                if (mode == 0) {
                    using RS = typename SpinorIO<P>::R;
                    cpx<RS> t[12];
                    SpinorIO<P>::load(xr, g.nblk, blk, l, t);
                    __syncthreads();  // the previous right-hand side's readers of rho are done
#pragma unroll
                    for (int k = 0; k < 12; ++k) s_rho[k][l] = {(R)t[k].re, (R)t[k].im};
                    __syncthreads();
                    block_hops<R>(l, ls, s_lk, own, acc);
                }
                if (mode != 1) {
                    face_pair<0, 1, P, R>(g, p, l, xr, links, acc);
                    face_pair<2, 3, P, R>(g, p, l, xr, links, acc);
                }
                cpx<R> cx[12];
                cpx<R> self[12];
                if (mode == 0) {
                    ls.load_nb(0, l, true, self);
                    if constexpr (BS != BLOCK_JACOBI) clover_apply(cl, self, cx);
                } else {
#pragma unroll
                    for (int k = 0; k < 12; ++k) cx[k] = self[k] = {(R)0, (R)0};
                }
                using RS = typename SpinorIO<P>::R;
                cpx<RS> t[12];
                SpinorIO<P>::load(br, g.nblk, blk, l, t);
                if constexpr (BS != BLOCK_JACOBI) {
#pragma unroll
                    for (int k = 0; k < 12; ++k)
                        rho0[k] = {(R)t[k].re - (cx[k].re - kappa * acc[k].re),
                                   (R)t[k].im - (cx[k].im - kappa * acc[k].im)};
                } else {
                    cpx<R> u[12];
#pragma unroll
                    for (int k = 0; k < 12; ++k)
                        u[k] = {(R)t[k].re + kappa * acc[k].re, (R)t[k].im + kappa * acc[k].im};
                    clover_apply(cl, u, rho0);
#pragma unroll
                    for (int k = 0; k < 12; ++k) rho0[k] = rho0[k] - self[k];
                }
                __syncthreads();  // every lane has read x from rho
#pragma unroll
                for (int k = 0; k < 12; ++k) s_rho[k][l].set(rho0[k]);
            } else if constexpr (BS != BLOCK_JACOBI) {
                cpx<R> acc[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[k] = {(R)0, (R)0};
                if (mode != 1) {
                    GlobalLinks<PLINK> glk{links};
                    if (mode == 0) {
                        GlobalSpinor<P, false> gs{xr, g.nblk};
                        hopping_sum_rolled<R>(g, p, l, gs, glk, acc);
                        cpx<R> self[12], cx[12];
                        gs.load(blk, l, self);
                        if constexpr (F32PATH) {
                            clover_apply(cl, self, cx);
                        } else {
                            R c2[72];
                            CloverIO<R>::template load<false>(clover, blk, l, c2);
                            clover_apply(c2, self, cx);
                        }
#pragma unroll
                        for (int k = 0; k < 12; ++k) acc[k] = {cx[k].re - kappa * acc[k].re, cx[k].im - kappa * acc[k].im};
                    } else {
                        OutsideSpinor<P> os{xr, g.nblk};
                        hopping_sum_rolled<R>(g, p, l, os, glk, acc);
#pragma unroll
                        for (int k = 0; k < 12; ++k) acc[k] = {-kappa * acc[k].re, -kappa * acc[k].im};
                    }
                }
                using RS = typename SpinorIO<P>::R;
                cpx<RS> t[12];
                SpinorIO<P>::load(br, g.nblk, blk, l, t);
#pragma unroll
                for (int k = 0; k < 12; ++k) rho0[k] = {(R)t[k].re - acc[k].re, (R)t[k].im - acc[k].im};
                __syncthreads();  // the previous right-hand side's readers of rho are done
#pragma unroll
                for (int k = 0; k < 12; ++k) s_rho[k][l].set(rho0[k]);
            } else {
                // Jacobi: rho = C^-1 (b + kappa hop) - x
                cpx<R> acc[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[k] = {(R)0, (R)0};
                if (mode != 1) {
                    GlobalLinks<PLINK> glk{links};
                    if (mode == 0) {
                        GlobalSpinor<P, false> gs{xr, g.nblk};
                        hopping_sum_rolled<R>(g, p, l, gs, glk, acc);
                    } else {
                        OutsideSpinor<P> os{xr, g.nblk};
                        hopping_sum_rolled<R>(g, p, l, os, glk, acc);
                    }
                }
                using RS = typename SpinorIO<P>::R;
                cpx<RS> t[12];
                SpinorIO<P>::load(br, g.nblk, blk, l, t);
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    acc[k] = {(R)t[k].re + kappa * acc[k].re, (R)t[k].im + kappa * acc[k].im};
                if constexpr (F32PATH) clover_apply(cl, acc, rho0);
                else clover_apply_by_chirality<R>(clover, blk, l, acc, rho0);
                if (mode == 0) {
                    using RS = typename SpinorIO<P>::R;
                    cpx<RS> xs[12];
                    SpinorIO<P>::load(xr, g.nblk, blk, l, xs);
#pragma unroll
                    for (int k = 0; k < 12; ++k) rho0[k] = {rho0[k].re - (R)xs[k].re, rho0[k].im - (R)xs[k].im};
                }
                __syncthreads();  // the previous right-hand side's readers of rho are done
#pragma unroll
                for (int k = 0; k < 12; ++k) s_rho[k][l].set(rho0[k]);
            }

            cpx<R> delta[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) delta[k] = {(R)0, (R)0};
            if constexpr (BS == BLOCK_JACOBI) {
                // ---- Jacobi steps on A_BB; the current delta lives in LDS
                if (n_mr > 0) {
#pragma unroll
                    for (int k = 0; k < 12; ++k) delta[k] = rho0[k];
                }
                if constexpr (RHO_LDS) {
#pragma unroll
                    for (int k = 0; k < 12; ++k) s_rho0[k][l].set(rho0[k]);
                }
                for (int it = 1; it < n_mr; ++it) {
                    __syncthreads();  // delta of every site is in LDS
                    cpx<R> acc[12];
#pragma unroll
                    for (int k = 0; k < 12; ++k) acc[k] = {(R)0, (R)0};
                    if constexpr (F32PATH) {
                        block_hops<R>(l, ls, s_lk, own, acc);
                        clover_apply(cl, acc, delta);
                    } else {
                        GlobalLinks<PLINK, false> lk{links};
                        hopping_sum_rolled<R>(g, p, l, ls, lk, acc);
                        clover_apply_by_chirality<R>(clover, blk, l, acc, delta);
                    }
#pragma unroll
                    for (int k = 0; k < 12; ++k) {
                        const cpx<R> r0 = RHO_LDS ? s_rho0[k][l].get() : rho0[k];
                        delta[k] = {r0.re + kappa * delta[k].re, r0.im + kappa * delta[k].im};
                    }
                    __syncthreads();  // every lane has read the previous delta
#pragma unroll
                    for (int k = 0; k < 12; ++k) s_rho[k][l].set(delta[k]);
                }
            }
#if CS_SAP_PRIO
            __builtin_amdgcn_s_setprio(0);
#endif
            // ---- MR on the Dirichlet block operator; rho lives in LDS only
            for (int it = 0; BS == BLOCK_MR && it < n_mr; ++it) {
                __syncthreads();
                cpx<R> q[12];
                {
                    cpx<R> acc[12];
#pragma unroll
                    for (int k = 0; k < 12; ++k) acc[k] = {(R)0, (R)0};
                    if constexpr (F32PATH) {
                        block_hops<R>(l, ls, s_lk, own, acc);
                    } else {
                        GlobalLinks<PLINK, false> lk{links};
                        hopping_sum_rolled<R>(g, p, l, ls, lk, acc);
                    }
                    cpx<R> rho[12];
                    ls.load_nb(0, l, true, rho);
                    if constexpr (F32PATH) {
                        clover_apply(cl, rho, q);
                    } else {
                        R c2[72];
                        CloverIO<R>::template load<false>(clover, blk, l, c2);
                        clover_apply(c2, rho, q);
                    }
#pragma unroll
                    for (int k = 0; k < 12; ++k) q[k] = {q[k].re - kappa * acc[k].re, q[k].im - kappa * acc[k].im};
                }
                cpx<R> rho[12];
                ls.load_nb(0, l, true, rho);
                R qq = 0, qr_re = 0, qr_im = 0;
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    qq = fma(q[k].re, q[k].re, qq);
                    qq = fma(q[k].im, q[k].im, qq);
                    // conj(q) * rho
                    qr_re = fma(q[k].re, rho[k].re, qr_re);
                    qr_re = fma(q[k].im, rho[k].im, qr_re);
                    qr_im = fma(q[k].re, rho[k].im, qr_im);
                    qr_im = fma(-q[k].im, rho[k].re, qr_im);
                }
                block_sum3(qq, qr_re, qr_im, s_red);
                if (qq == (R)0) break;  // rho = 0: the block is solved (uniform branch)
                const R inv = (R)1 / qq;
                const cpx<R> alpha = {qr_re * inv, qr_im * inv};
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    cmac(delta[k], alpha, rho[k]);
                    cpx<R> t = rho[k];
                    t.re = fma(-alpha.re, q[k].re, t.re);
                    t.re = fma(alpha.im, q[k].im, t.re);
                    t.im = fma(-alpha.re, q[k].im, t.im);
                    t.im = fma(-alpha.im, q[k].re, t.im);
                    s_rho[k][l].set(t);
                }
            }

            if constexpr (BS == BLOCK_EO) {
                // ---- even-odd preconditioned MR: S = C_e - kappa^2 H_eo C_o^-1 H_oe on
                // the even sites, then the odd sites by back-substitution.  s_rho
                // holds r_B; rho0 keeps it in registers for the odd lanes.
                const bool odd = threadIdx.x >= BLOCK_SITES / 2;  // wave-uniform
                auto hop_lds = [&](cpx<R>* acc) {  // in-block hopping sum from s_rho
#pragma unroll
                    for (int k = 0; k < 12; ++k) acc[k] = {(R)0, (R)0};
                    if constexpr (F32PATH) {
                        block_hops<R>(l, ls, s_lk, own, acc);
                    } else {
                        GlobalLinks<PLINK, false> lk{links};
                        hopping_sum_rolled<R>(g, p, l, ls, lk, acc);
                    }
                };
                if (odd) {  // C_o^-1 r_o on the odd sites
                    cpx<R> t[12];
                    clover_apply_by_chirality<R>(cinv, blk, l, rho0, t);
#pragma unroll
                    for (int k = 0; k < 12; ++k) s_rho[k][l].set(t[k]);
                }
                __syncthreads();
                cpx<R> rr[12];
                if (!odd) {  // rhat_e = r_e + kappa H_eo C_o^-1 r_o
                    cpx<R> acc[12];
                    hop_lds(acc);
#pragma unroll
                    for (int k = 0; k < 12; ++k) rr[k] = {rho0[k].re + kappa * acc[k].re, rho0[k].im + kappa * acc[k].im};
                }
                __syncthreads();  // every even lane has read the odd entries
                if (!odd) {
#pragma unroll
                    for (int k = 0; k < 12; ++k) s_rho[k][l].set(rr[k]);
                }
                for (int it = 0; it < n_mr; ++it) {
                    __syncthreads();  // the even residual is in LDS
                    if (odd) {  // t_o = kappa C_o^-1 H_oe r_e
                        cpx<R> acc[12], t[12];
                        hop_lds(acc);
                        clover_apply_by_chirality<R>(cinv, blk, l, acc, t);
#pragma unroll
                        for (int k = 0; k < 12; ++k) s_rho[k][l] = {kappa * t[k].re, kappa * t[k].im};
                    }
                    __syncthreads();
                    cpx<R> q[12];
                    R qq = 0, qr_re = 0, qr_im = 0;
                    if (!odd) {  // q_e = C_e r_e - kappa H_eo t_o
                        cpx<R> acc[12];
                        hop_lds(acc);
                        ls.load_nb(0, l, true, rr);
                        if constexpr (F32PATH) {
                            clover_apply(cl, rr, q);
                        } else {
                            R c2[72];
                            CloverIO<R>::template load<false>(clover, blk, l, c2);
                            clover_apply(c2, rr, q);
                        }
#pragma unroll
                        for (int k = 0; k < 12; ++k) {
                            q[k] = {q[k].re - kappa * acc[k].re, q[k].im - kappa * acc[k].im};
                            qq = fma(q[k].re, q[k].re, qq);
                            qq = fma(q[k].im, q[k].im, qq);
                            qr_re = fma(q[k].re, rr[k].re, qr_re);
                            qr_re = fma(q[k].im, rr[k].im, qr_re);
                            qr_im = fma(q[k].re, rr[k].im, qr_im);
                            qr_im = fma(-q[k].im, rr[k].re, qr_im);
                        }
                    }
                    block_sum3(qq, qr_re, qr_im, s_red);
                    if (qq == (R)0) break;  // the even residual is zero (uniform branch)
                    const R inv = (R)1 / qq;
                    const cpx<R> alpha = {qr_re * inv, qr_im * inv};
                    if (!odd) {
#pragma unroll
                        for (int k = 0; k < 12; ++k) {
                            cmac(delta[k], alpha, rr[k]);
                            cpx<R> t = rr[k];
                            t.re = fma(-alpha.re, q[k].re, t.re);
                            t.re = fma(alpha.im, q[k].im, t.re);
                            t.im = fma(-alpha.re, q[k].im, t.im);
                            t.im = fma(-alpha.im, q[k].re, t.im);
                            s_rho[k][l].set(t);
                        }
                    }
                }
                // delta_o = C_o^-1 (r_o + kappa H_oe delta_e)
                __syncthreads();
                if (!odd) {
#pragma unroll
                    for (int k = 0; k < 12; ++k) s_rho[k][l].set(delta[k]);
                }
                __syncthreads();
                if (odd) {
                    cpx<R> acc[12], u[12];
                    hop_lds(acc);
#pragma unroll
                    for (int k = 0; k < 12; ++k) u[k] = {rho0[k].re + kappa * acc[k].re, rho0[k].im + kappa * acc[k].im};
                    clover_apply_by_chirality<R>(cinv, blk, l, u, delta);
                }
            }

            // ---- x_B += delta (after every lane has finished reading x and rho)
            __syncthreads();
            using RS = typename SpinorIO<P>::R;
            cpx<RS> xo[12];
            if (mode == 0) {
                SpinorIO<P>::load(xr, g.nblk, blk, l, xo);
#pragma unroll
                for (int k = 0; k < 12; ++k) xo[k] = {xo[k].re + (RS)delta[k].re, xo[k].im + (RS)delta[k].im};
            } else {
#pragma unroll
                for (int k = 0; k < 12; ++k) xo[k] = {(RS)delta[k].re, (RS)delta[k].im};
            }
            SpinorIO<P>::store(xr, g.nblk, blk, l, xo);
        }
    }
}

template <int P, int PLINK, bool GEN>
void launch_pm(const OpData& op, int colour, int n_mr, int mode, void* x, const void* b, size_t stride, int nrhs,
               int tile, int nitems, int grid, hipStream_t s, int bs) {
    const void* cl = P == P_F64 ? op.clover64 : op.clover32;
    const void* ci = P == P_F64 ? op.cinv64 : op.cinv32;
    if (bs == BLOCK_JACOBI) {
        hipLaunchKernelGGL((k_sap_halfsweep<P, PLINK, BLOCK_JACOBI, GEN>), dim3(grid), dim3(BLOCK_SITES), 0, s, op.g,
                           op.links[PLINK], ci, nullptr, op.kappa, colour, n_mr, mode, x, b, stride, nrhs, tile,
                           nitems);
    } else if (bs == BLOCK_EO) {
        hipLaunchKernelGGL((k_sap_halfsweep<P, PLINK, BLOCK_EO, GEN>), dim3(grid), dim3(BLOCK_SITES), 0, s, op.g,
                           op.links[PLINK], cl, ci, op.kappa, colour, n_mr, mode, x, b, stride, nrhs, tile, nitems);
    } else {
        hipLaunchKernelGGL((k_sap_halfsweep<P, PLINK, BLOCK_MR, GEN>), dim3(grid), dim3(BLOCK_SITES), 0, s, op.g,
                           op.links[PLINK], cl, nullptr, op.kappa, colour, n_mr, mode, x, b, stride, nrhs, tile,
                           nitems);
    }
}

template <int P, int PLINK>
hipError_t launch_p(const OpData& op, int colour, int n_mr, int mode, void* x, const void* b,
                    int nrhs, const LaunchCfg& cfg, hipStream_t s, int bs) {
    const int tile = cfg.rhs_tile < 1 ? 1 : (cfg.rhs_tile > nrhs ? nrhs : cfg.rhs_tile);
    const int nitems = (op.g.nblk / 2) * ((nrhs + tile - 1) / tile);
    const int grid = cfg.persistent_wgs > 0 && cfg.persistent_wgs < nitems ? cfg.persistent_wgs : nitems;
    const size_t stride = spinor_bytes_per_site(P) * op.g.V;
    if (mode == 0) launch_pm<P, PLINK, true>(op, colour, n_mr, mode, x, b, stride, nrhs, tile, nitems, grid, s, bs);
    else launch_pm<P, PLINK, false>(op, colour, n_mr, mode, x, b, stride, nrhs, tile, nitems, grid, s, bs);
    return hipGetLastError();
}

}  // namespace

// Lanes per site when the caller leaves the choice to the library.  The
// lane-pair kernel halves the dependent arithmetic of a block visit but fits
// one workgroup per compute unit (the one-lane kernel fits two), so it pays
// only while a colour has at most one block per compute unit (256 on
// MI355X): measured 7-10% faster at 128 and 256 blocks per colour, 35%
// slower at 1296 and 4096.
static int default_lanes_per_site(const Geom& g) { return g.nblk / 2 <= 256 ? 2 : 1; }

hipError_t launch_sap_halfsweep(const OpData& op, int prec, int colour, int n_mr, int mode, void* x,
                                const void* b, int nrhs, const LaunchCfg& cfg, hipStream_t s, int bs) {
    ProfScope ps("sap_halfsweep", s);
    // general visits (x nonzero everywhere) separately: their bytes per site
    // differ from those of the two half-sweeps that start from x = 0
    ProfScope pm(mode == 0 ? "sap_general" : "sap_from_zero", s);
    if (bs != BLOCK_MR && bs != BLOCK_JACOBI && bs != BLOCK_EO) return hipErrorInvalidValue;
    const int lanes = cfg.lanes_per_site > 0 ? cfg.lanes_per_site : default_lanes_per_site(op.g);
    // the even-odd block solver has the one-lane form only
    if (lanes == 2 && prec != P_F64 && bs != BLOCK_EO)
        return launch_sap_pair(op, prec, colour, n_mr, mode, x, b, nrhs, cfg, s, bs);
    switch (prec) {
    case P_F64: return launch_p<P_F64, P_F64>(op, colour, n_mr, mode, x, b, nrhs, cfg, s, bs);
    case P_F32: return launch_p<P_F32, P_F32>(op, colour, n_mr, mode, x, b, nrhs, cfg, s, bs);
    case P_F16: return launch_p<P_F16, P_F16>(op, colour, n_mr, mode, x, b, nrhs, cfg, s, bs);
    case P_BF16: return launch_p<P_BF16, P_BF16>(op, colour, n_mr, mode, x, b, nrhs, cfg, s, bs);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace cs
