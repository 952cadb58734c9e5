// The hopping sum of the clover-Wilson operator as a device function, shared
// by the standalone operator kernel and the SAP kernel.  The neighbour spinor
// and link sources are policies, so the same code runs on fields in HBM, on a
// block held in LDS, and on the Dirichlet-restricted block operator.
#pragma once

#include "fields.hpp"

namespace cs {

// Spinors from HBM; with DAG the lower two spins are negated on load (the
// gamma5 sandwich of D^dag = gamma5 D gamma5).
template <int P, bool DAG>
struct GlobalSpinor {
    const void* base;
    int nblk;
    __device__ __forceinline__ bool want(bool) const { return true; }
    template <typename R>
    __device__ __forceinline__ void load(int blk, int l, cpx<R>* c) const {
        using RS = typename SpinorIO<P>::R;
        cpx<RS> t[12];
        SpinorIO<P>::load(base, nblk, blk, l, t);
#pragma unroll
        for (int k = 0; k < 12; ++k) c[k] = {(R)t[k].re, (R)t[k].im};
        if (DAG) negate_lower(c);
    }
    template <typename R>
    __device__ __forceinline__ void load_nb(int blk, int l, bool, cpx<R>* c) const { load(blk, l, c); }
};

// Links from HBM.
template <int P>
struct GlobalLinks {
    const void* base;
    template <typename R>
    __device__ __forceinline__ void load(int blk, int l, int mu, bool, cpx<R>* u) const {
        load_link<P, R>(base, blk, l, mu, u);
    }
};

// acc += sum over the two hops in direction MU that the spinor policy wants.
template <int MU, typename R, typename LS, typename LL>
__device__ __forceinline__ void hop_dir(const Geom& g, const BlockPos& p, int l, const LS& ls,
                                        const LL& lk, cpx<R>* acc) {
    int nl;
    bool in;
    int nb = neighbour(g, p, l, MU, +1, &nl, &in);
    if (ls.want(in)) {
        cpx<R> psi[12], u[9];
        ls.template load_nb<R>(nb, nl, in, psi);
        lk.template load<R>(p.blk, l, MU, true, u);
        hop_term<MU, -1>(u, psi, acc);
    }
    nb = neighbour(g, p, l, MU, -1, &nl, &in);
    if (ls.want(in)) {
        cpx<R> psi[12], u[9];
        ls.template load_nb<R>(nb, nl, in, psi);
        lk.template load<R>(nb, nl, MU, in, u);
        hop_term<MU, +1>(u, psi, acc);
    }
}

template <typename R, typename LS, typename LL>
__device__ __forceinline__ void hopping_sum(const Geom& g, const BlockPos& p, int l, const LS& ls,
                                            const LL& lk, cpx<R>* acc) {
    hop_dir<0, R>(g, p, l, ls, lk, acc);
    hop_dir<1, R>(g, p, l, ls, lk, acc);
    hop_dir<2, R>(g, p, l, ls, lk, acc);
    hop_dir<3, R>(g, p, l, ls, lk, acc);
}

}  // namespace cs
