// Clover-Wilson operator (paper Section 2, Eq. (1), with C = 1 + T):
//   (D psi)(x) = (1 + T(x)) psi(x)
//     - kappa sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)]
// One workgroup per 4^4 block, one lane per site; every load is unit-stride
// across the lanes because fields are component-major within a block.  The
// kernel is bound by HBM bandwidth: per site it reads the spinor (the eight
// neighbours come from cache), four compressed links (the backward links are
// the neighbours' forward links) and the clover term, and writes one spinor.
#include "dslash_core.hpp"

namespace cs {

namespace {

template <int PIN, int POUT, int PLINK, bool DAG, bool SUB>
__global__ CS_DSLASH_BOUNDS void k_dslash(Geom g, const void* __restrict__ links,
                                                        const void* __restrict__ clover, double kappa,
                                                        void* __restrict__ out,
                                                        const void* __restrict__ in,
                                                        const void* __restrict__ sub,
                                                        size_t in_stride, size_t out_stride) {
    using R = typename Arith<PIN>::R;
    const int blk = block_of_item(g, xcd_remap(blockIdx.x, g.nblk)), l = threadIdx.x, r = blockIdx.y;
    const char* src = (const char*)in + r * in_stride;
    const BlockPos p = block_pos(g, blk);

    cpx<R> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {(R)0, (R)0};
    GlobalSpinor<PIN, DAG> ld{src, g.nblk};
    GlobalLinks<PLINK> lk{links};
    if (CS_DSLASH_ROLLED || PIN == P_F64) hopping_sum_rolled<R>(g, p, l, ld, lk, acc);
    else hopping_sum<R>(g, p, l, ld, lk, acc);

    cpx<R> self[12], res[12];
    ld.load(blk, l, self);
    R cl[72];
    CloverIO<R>::load(clover, blk, l, cl);
    clover_apply(cl, self, res);
    const R k = (R)kappa;
#pragma unroll
    for (int i = 0; i < 12; ++i) res[i] = {res[i].re - k * acc[i].re, res[i].im - k * acc[i].im};
    if (DAG) negate_lower(res);
    using RO = typename SpinorIO<POUT>::R;
    cpx<RO> o[12];
    if (SUB) {
        SpinorIO<POUT>::load((const char*)sub + r * out_stride, g.nblk, blk, l, o);
#pragma unroll
        for (int i = 0; i < 12; ++i) o[i] = {o[i].re - (RO)res[i].re, o[i].im - (RO)res[i].im};
    } else {
#pragma unroll
        for (int i = 0; i < 12; ++i) o[i] = {(RO)res[i].re, (RO)res[i].im};
    }
    SpinorIO<POUT>::store((char*)out + r * out_stride, g.nblk, blk, l, o);
}

// Staged form of the same operator (float arithmetic): the block's input
// spinor is copied to LDS once (converted to float, with the gamma5 sign of
// D^dag applied), and every in-block hop reads its neighbour from there;
// only the hops that leave the block read HBM.  With LINKS_LDS the block's
// links (rows 0 and 1) are staged too, so the backward hops inside the block
// take the neighbour lane's link from LDS instead of re-reading it.  Each
// spinor and link word of the block is then fetched from HBM once by its own
// workgroup; the plain kernel above fetches each spinor once per hop and
// relies on the caches for the reuse.
template <int P, bool DAG>
struct StagedSpinor {
    const lds_cpx<float> (*s)[BLOCK_SITES];
    const void* base;
    int nblk;
    __device__ __forceinline__ bool want(bool) const { return true; }
    template <typename R>
    __device__ __forceinline__ void load_nb(int blk, int l, bool inside, cpx<R>* c) const {
        if (inside) {
#pragma unroll
            for (int k = 0; k < 12; ++k) c[k] = {(R)s[k][l].re, (R)s[k][l].im};
        } else {
            using RS = typename SpinorIO<P>::R;
            cpx<RS> t[12];
            SpinorIO<P>::load(base, nblk, blk, l, t);
#pragma unroll
            for (int k = 0; k < 12; ++k) c[k] = {(R)t[k].re, (R)t[k].im};
            if (DAG) negate_lower(c);
        }
    }
};

template <int PLINK>
struct StagedLinks {
    const lds_cpx<float> (*sm)[6][BLOCK_SITES];
    const void* base;
    template <typename R>
    __device__ __forceinline__ void load(int blk, int l, int mu, bool inside, cpx<R>* u) const {
        if (inside) {
#pragma unroll
            for (int k = 0; k < 6; ++k) u[k] = {(R)sm[mu][k][l].re, (R)sm[mu][k][l].im};
            su3_row2(u);
        } else {
            load_link<PLINK, R, false>(base, blk, l, mu, u);
        }
    }
};

template <bool ON>
struct StagedLinkSmem { lds_cpx<float> u[4][6][BLOCK_SITES]; };
template <>
struct StagedLinkSmem<false> { lds_cpx<float> u[1][6][1]; };

template <int PIN, int POUT, int PLINK, bool DAG, bool SUB, bool LINKS_LDS>
__global__ CS_DSLASH_BOUNDS void k_dslash_staged(Geom g, const void* __restrict__ links,
                                                 const void* __restrict__ clover, float kappa,
                                                 void* __restrict__ out, const void* __restrict__ in,
                                                 const void* __restrict__ sub, size_t in_stride,
                                                 size_t out_stride) {
    __shared__ lds_cpx<float> s_psi[12][BLOCK_SITES];
    __shared__ StagedLinkSmem<LINKS_LDS> s_lk;
    const int blk = block_of_item(g, xcd_remap(blockIdx.x, g.nblk)), l = threadIdx.x, r = blockIdx.y;
    const char* src = (const char*)in + r * in_stride;
    const BlockPos p = block_pos(g, blk);

    {
        using RS = typename SpinorIO<PIN>::R;
        cpx<RS> t[12];
        SpinorIO<PIN>::load(src, g.nblk, blk, l, t);
        cpx<float> v[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = {(float)t[k].re, (float)t[k].im};
        if (DAG) negate_lower(v);
#pragma unroll
        for (int k = 0; k < 12; ++k) s_psi[k][l].set(v[k]);
    }
    if constexpr (LINKS_LDS) {
        for (int mu = 0; mu < 4; ++mu) {
            cpx<typename LinkIO<PLINK>::R> u[6];
            LinkIO<PLINK>::load6(links, blk, l, mu, u);
#pragma unroll
            for (int k = 0; k < 6; ++k) s_lk.u[mu][k][l] = {(float)u[k].re, (float)u[k].im};
        }
    }
    __syncthreads();

    cpx<float> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {0.f, 0.f};
    StagedSpinor<PIN, DAG> ls{s_psi, src, g.nblk};
    if constexpr (LINKS_LDS) {
        StagedLinks<PLINK> lk{s_lk.u, links};
        hopping_sum_rolled<float>(g, p, l, ls, lk, acc);
    } else {
        GlobalLinks<PLINK, false> lk{links};
        hopping_sum_rolled<float>(g, p, l, ls, lk, acc);
    }

    cpx<float> self[12], res[12];
    ls.load_nb(blk, l, true, self);
    float cl[72];
    CloverIO<float>::load(clover, blk, l, cl);
    clover_apply(cl, self, res);
#pragma unroll
    for (int i = 0; i < 12; ++i) res[i] = {res[i].re - kappa * acc[i].re, res[i].im - kappa * acc[i].im};
    if (DAG) negate_lower(res);
    using RO = typename SpinorIO<POUT>::R;
    cpx<RO> o[12];
    if (SUB) {
        SpinorIO<POUT>::load((const char*)sub + r * out_stride, g.nblk, blk, l, o);
#pragma unroll
        for (int i = 0; i < 12; ++i) o[i] = {o[i].re - (RO)res[i].re, o[i].im - (RO)res[i].im};
    } else {
#pragma unroll
        for (int i = 0; i < 12; ++i) o[i] = {(RO)res[i].re, (RO)res[i].im};
    }
    SpinorIO<POUT>::store((char*)out + r * out_stride, g.nblk, blk, l, o);
}

// Multi-right-hand-side variant: work item = (block, tile of right-hand
// sides).  The block's links go to LDS once and its clover term to registers
// once per item; every right-hand side of the tile reuses them.  Backward
// links of neighbours outside the block come from HBM (cache).  With
// gridDim.x < nitems the workgroups stride over the items (persistent).
template <bool ON>
struct DLinkSmem { lds_cpx<float> u[4][6][BLOCK_SITES]; };
template <>
struct DLinkSmem<false> { lds_cpx<double> u[4][6][BLOCK_SITES]; };

template <typename RS, int PLINK>
struct MixedLinks {
    const lds_cpx<RS> (*sm)[6][BLOCK_SITES];
    const void* base;
    template <typename R>
    __device__ __forceinline__ void load(int blk, int l, int mu, bool inside, cpx<R>* u) const {
        if (inside) {
#pragma unroll
            for (int k = 0; k < 6; ++k) u[k] = {(R)sm[mu][k][l].re, (R)sm[mu][k][l].im};
            su3_row2(u);
        } else {
            load_link<PLINK, R, false>(base, blk, l, mu, u);
        }
    }
};

// The rolled hopping sum for two right-hand sides at once: each hop loads
// its link once and the two neighbour spinors together, so two loads are in
// flight where the one-right-hand-side loop waits on one.  Each sum gets the
// same terms in the same order as hopping_sum_rolled.
template <typename R, typename LS, typename LL>
__device__ __forceinline__ void hopping_sum_rolled2(const Geom& g, const BlockPos& p, int l, const LS& ls0,
                                                    const LS& ls1, const LL& lk, cpx<R>* acc0, cpx<R>* acc1) {
#pragma unroll 1
    for (int h = 0; h < 8; ++h) {
        const int mu = h >> 1, dir = (h & 1) ? -1 : +1;
        const int bc = mu == 0 ? p.bc[0] : mu == 1 ? p.bc[1] : mu == 2 ? p.bc[2] : p.bc[3];
        const int nbm = mu == 0 ? g.NB[0] : mu == 1 ? g.NB[1] : mu == 2 ? g.NB[2] : g.NB[3];
        const int st = mu == 0 ? p.stride[0] : mu == 1 ? p.stride[1] : mu == 2 ? p.stride[2] : p.stride[3];
        const int sh = 2 * mu, lc = (l >> sh) & 3;
        int nl, nb;
        bool in;
        if (dir > 0) {
            in = lc < 3;
            nl = in ? l + (1 << sh) : l - (3 << sh);
            nb = in ? p.blk : (bc == nbm - 1 ? p.blk - (nbm - 1) * st : p.blk + st);
        } else {
            in = lc > 0;
            nl = in ? l - (1 << sh) : l + (3 << sh);
            nb = in ? p.blk : (bc == 0 ? p.blk + (nbm - 1) * st : p.blk - st);
        }
        cpx<R> psi0[12], psi1[12], u[9];
        ls0.template load_nb<R>(nb, nl, in, psi0);
        ls1.template load_nb<R>(nb, nl, in, psi1);
        if (mu == 3) {
            const bool wraps = !in && (dir > 0 ? bc == nbm - 1 : bc == 0);
            time_boundary_phase(g, wraps, &psi0[0].re, 24);
            time_boundary_phase(g, wraps, &psi1[0].re, 24);
        }
        if (dir > 0) lk.template load<R>(p.blk, l, mu, true, u);
        else lk.template load<R>(nb, nl, mu, in, u);
        switch (h) {
        case 0: hop_term<0, -1>(u, psi0, acc0); hop_term<0, -1>(u, psi1, acc1); break;
        case 1: hop_term<0, +1>(u, psi0, acc0); hop_term<0, +1>(u, psi1, acc1); break;
        case 2: hop_term<1, -1>(u, psi0, acc0); hop_term<1, -1>(u, psi1, acc1); break;
        case 3: hop_term<1, +1>(u, psi0, acc0); hop_term<1, +1>(u, psi1, acc1); break;
        case 4: hop_term<2, -1>(u, psi0, acc0); hop_term<2, -1>(u, psi1, acc1); break;
        case 5: hop_term<2, +1>(u, psi0, acc0); hop_term<2, +1>(u, psi1, acc1); break;
        case 6: hop_term<3, -1>(u, psi0, acc0); hop_term<3, -1>(u, psi1, acc1); break;
        default: hop_term<3, +1>(u, psi0, acc0); hop_term<3, +1>(u, psi1, acc1); break;
        }
    }
}

template <int PIN, int POUT, int PLINK, bool DAG>
__global__ CS_DSLASH_BOUNDS void k_dslash_tiled(Geom g, const void* __restrict__ links,
                                                const void* __restrict__ clover, double kappa,
                                                void* __restrict__ out, const void* __restrict__ in,
                                                size_t in_stride, size_t out_stride, int nrhs, int tile,
                                                int nitems) {
    using R = typename Arith<PIN>::R;
    using RS = typename LinkIO<PLINK>::R;
    __shared__ lds_cpx<RS> s_lk[4][6][BLOCK_SITES];
    const int l = threadIdx.x;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int w = xcd_remap(item, nitems);
        const int blk = block_of_item(g, w % g.nblk);
        const int r0 = (w / g.nblk) * tile;
        const int r1 = r0 + tile < nrhs ? r0 + tile : nrhs;
        const BlockPos p = block_pos(g, blk);
        __syncthreads();
        for (int mu = 0; mu < 4; ++mu) {
            cpx<RS> u[6];
            LinkIO<PLINK>::load6(links, blk, l, mu, u);
#pragma unroll
            for (int k = 0; k < 6; ++k) s_lk[mu][k][l].set(u[k]);
        }
        R cl[72];
        CloverIO<R>::load(clover, blk, l, cl);
        __syncthreads();
        MixedLinks<RS, PLINK> lk{s_lk, links};
        const R k = (R)kappa;
        // the clover term and the output of one right-hand side
        auto finish = [&](int r, const GlobalSpinor<PIN, DAG>& ld, const cpx<R>* acc) {
            cpx<R> self[12], res[12];
            ld.load(blk, l, self);
            clover_apply(cl, self, res);
#pragma unroll
            for (int i = 0; i < 12; ++i) res[i] = {res[i].re - k * acc[i].re, res[i].im - k * acc[i].im};
            if (DAG) negate_lower(res);
            using RO = typename SpinorIO<POUT>::R;
            cpx<RO> o[12];
#pragma unroll
            for (int i = 0; i < 12; ++i) o[i] = {(RO)res[i].re, (RO)res[i].im};
            SpinorIO<POUT>::store((char*)out + (size_t)r * out_stride, g.nblk, blk, l, o);
        };
        int r = r0;
        if constexpr (PIN != P_F64) {
            // right-hand sides two at a time (the FP64 form keeps one: its
            // registers are full)
            for (; r + 1 < r1; r += 2) {
                GlobalSpinor<PIN, DAG> ld0{(const char*)in + (size_t)r * in_stride, g.nblk};
                GlobalSpinor<PIN, DAG> ld1{(const char*)in + (size_t)(r + 1) * in_stride, g.nblk};
                cpx<R> acc0[12], acc1[12];
#pragma unroll
                for (int i = 0; i < 12; ++i) acc0[i] = acc1[i] = {(R)0, (R)0};
                hopping_sum_rolled2<R>(g, p, l, ld0, ld1, lk, acc0, acc1);
                finish(r, ld0, acc0);
                finish(r + 1, ld1, acc1);
            }
        }
        for (; r < r1; ++r) {
            GlobalSpinor<PIN, DAG> ld{(const char*)in + (size_t)r * in_stride, g.nblk};
            cpx<R> acc[12];
#pragma unroll
            for (int i = 0; i < 12; ++i) acc[i] = {(R)0, (R)0};
            hopping_sum_rolled<R>(g, p, l, ld, lk, acc);
            finish(r, ld, acc);
        }
    }
}

template <int PIN, int POUT, int PLINK>
hipError_t launch_tiled(const OpData& op, bool dagger, void* out, const void* in, int nrhs,
                        const LaunchCfg& cfg, hipStream_t s) {
    const int tile = cfg.rhs_tile > nrhs ? nrhs : cfg.rhs_tile;
    const int nitems = op.g.nblk * ((nrhs + tile - 1) / tile);
    const int grid = cfg.persistent_wgs > 0 && cfg.persistent_wgs < nitems ? cfg.persistent_wgs : nitems;
    const size_t is = spinor_bytes_per_site(PIN) * op.g.V, os = spinor_bytes_per_site(POUT) * op.g.V;
    const void* cl = PIN == P_F64 ? op.clover64 : op.clover32;
    const void* lk = op.links[PLINK];
    if (dagger)
        hipLaunchKernelGGL((k_dslash_tiled<PIN, POUT, PLINK, true>), dim3(grid), dim3(BLOCK_SITES), 0, s, op.g, lk, cl,
                           op.kappa, out, in, is, os, nrhs, tile, nitems);
    else
        hipLaunchKernelGGL((k_dslash_tiled<PIN, POUT, PLINK, false>), dim3(grid), dim3(BLOCK_SITES), 0, s, op.g, lk, cl,
                           op.kappa, out, in, is, os, nrhs, tile, nitems);
    return hipGetLastError();
}

template <int PIN, int POUT, int PLINK>
hipError_t launch3(const OpData& op, bool dagger, void* out, const void* in, const void* sub,
                   int nrhs, hipStream_t s) {
    const dim3 grid(op.g.nblk, nrhs), block(BLOCK_SITES);
    const size_t is = spinor_bytes_per_site(PIN) * op.g.V, os = spinor_bytes_per_site(POUT) * op.g.V;
    const void* cl = PIN == P_F64 ? op.clover64 : op.clover32;
    const void* lk = op.links[PLINK];
    if constexpr (PIN != P_F64 && CS_DSLASH_STAGED) {
        constexpr bool LL = CS_DSLASH_STAGED == 2;
        const float k = (float)op.kappa;
        if (dagger) {
            if (sub) hipLaunchKernelGGL((k_dslash_staged<PIN, POUT, PLINK, true, true, LL>), grid, block, 0, s, op.g, lk, cl, k, out, in, sub, is, os);
            else hipLaunchKernelGGL((k_dslash_staged<PIN, POUT, PLINK, true, false, LL>), grid, block, 0, s, op.g, lk, cl, k, out, in, sub, is, os);
        } else {
            if (sub) hipLaunchKernelGGL((k_dslash_staged<PIN, POUT, PLINK, false, true, LL>), grid, block, 0, s, op.g, lk, cl, k, out, in, sub, is, os);
            else hipLaunchKernelGGL((k_dslash_staged<PIN, POUT, PLINK, false, false, LL>), grid, block, 0, s, op.g, lk, cl, k, out, in, sub, is, os);
        }
        return hipGetLastError();
    }
    if (dagger) {
        if (sub) hipLaunchKernelGGL((k_dslash<PIN, POUT, PLINK, true, true>), grid, block, 0, s, op.g, lk, cl, op.kappa, out, in, sub, is, os);
        else hipLaunchKernelGGL((k_dslash<PIN, POUT, PLINK, true, false>), grid, block, 0, s, op.g, lk, cl, op.kappa, out, in, sub, is, os);
    } else {
        if (sub) hipLaunchKernelGGL((k_dslash<PIN, POUT, PLINK, false, true>), grid, block, 0, s, op.g, lk, cl, op.kappa, out, in, sub, is, os);
        else hipLaunchKernelGGL((k_dslash<PIN, POUT, PLINK, false, false>), grid, block, 0, s, op.g, lk, cl, op.kappa, out, in, sub, is, os);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dslash_tiled(const OpData& op, int prec, bool dagger, void* out, const void* in, int nrhs,
                               const LaunchCfg& cfg, hipStream_t s) {
    ProfScope ps("dslash", s);
    switch (prec) {
    case P_F64: return launch_tiled<P_F64, P_F64, P_F64>(op, dagger, out, in, nrhs, cfg, s);
    case P_F32: return launch_tiled<P_F32, P_F32, P_F32>(op, dagger, out, in, nrhs, cfg, s);
    case P_F16: return launch_tiled<P_F16, P_F16, P_F16>(op, dagger, out, in, nrhs, cfg, s);
    case P_BF16: return launch_tiled<P_BF16, P_BF16, P_BF16>(op, dagger, out, in, nrhs, cfg, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dslash_tiled_to16(const OpData& op, int out_prec, void* out, const void* in, int nrhs,
                                    const LaunchCfg& cfg, hipStream_t s) {
    ProfScope ps("dslash", s);
    switch (out_prec) {
    case P_F16: return launch_tiled<P_F32, P_F16, P_F32>(op, false, out, in, nrhs, cfg, s);
    case P_BF16: return launch_tiled<P_F32, P_BF16, P_F32>(op, false, out, in, nrhs, cfg, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dslash(const OpData& op, int in_prec, int out_prec, int link_prec, bool dagger,
                         void* out, const void* in, const void* sub, int nrhs, hipStream_t s) {
    ProfScope ps("dslash", s);
    // Supported combinations: F64 -> F64 (F64 links); float arithmetic with
    // spinors in F32/F16/BF16, links F32 or the spinor's 16-bit type, output
    // F32 or the input type.
    if (in_prec == P_F64) {
        if (out_prec != P_F64) return hipErrorInvalidValue;
        return launch3<P_F64, P_F64, P_F64>(op, dagger, out, in, sub, nrhs, s);
    }
    if (in_prec == P_F32 && out_prec == P_F32 && link_prec == P_F32)
        return launch3<P_F32, P_F32, P_F32>(op, dagger, out, in, sub, nrhs, s);
    if (in_prec == P_F16 && out_prec == P_F16 && link_prec == P_F16)
        return launch3<P_F16, P_F16, P_F16>(op, dagger, out, in, sub, nrhs, s);
    if (in_prec == P_BF16 && out_prec == P_BF16 && link_prec == P_BF16)
        return launch3<P_BF16, P_BF16, P_BF16>(op, dagger, out, in, sub, nrhs, s);
    if (in_prec == P_F16 && out_prec == P_F32 && link_prec == P_F32)
        return launch3<P_F16, P_F32, P_F32>(op, dagger, out, in, sub, nrhs, s);
    if (in_prec == P_BF16 && out_prec == P_F32 && link_prec == P_F32)
        return launch3<P_BF16, P_F32, P_F32>(op, dagger, out, in, sub, nrhs, s);
    // FP32 or 16-bit input with FP32 links, written straight into a 16-bit
    // field (the 16-bit Krylov basis of the outer solver)
    if (link_prec == P_F32 && out_prec == P_F16 && in_prec == P_F32)
        return launch3<P_F32, P_F16, P_F32>(op, dagger, out, in, sub, nrhs, s);
    if (link_prec == P_F32 && out_prec == P_BF16 && in_prec == P_F32)
        return launch3<P_F32, P_BF16, P_F32>(op, dagger, out, in, sub, nrhs, s);
    if (link_prec == P_F32 && out_prec == P_F16 && in_prec == P_F16)
        return launch3<P_F16, P_F16, P_F32>(op, dagger, out, in, sub, nrhs, s);
    if (link_prec == P_F32 && out_prec == P_BF16 && in_prec == P_BF16)
        return launch3<P_BF16, P_BF16, P_F32>(op, dagger, out, in, sub, nrhs, s);
    return hipErrorInvalidValue;
}

}  // namespace cs
