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
    const int blk = xcd_remap(blockIdx.x, g.nblk), l = threadIdx.x, r = blockIdx.y;
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

template <int PIN, int POUT, int PLINK>
hipError_t launch3(const OpData& op, bool dagger, void* out, const void* in, const void* sub,
                   int nrhs, hipStream_t s) {
    const dim3 grid(op.g.nblk, nrhs), block(BLOCK_SITES);
    const size_t is = spinor_bytes_per_site(PIN) * op.g.V, os = spinor_bytes_per_site(POUT) * op.g.V;
    const void* cl = PIN == P_F64 ? op.clover64 : op.clover32;
    const void* lk = op.links[PLINK];
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
    return hipErrorInvalidValue;
}

}  // namespace cs
