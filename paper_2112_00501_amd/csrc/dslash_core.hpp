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

// Links from HBM (ONCE: each link word is read once by this kernel).
template <int P, bool ONCE = true>
struct GlobalLinks {
    const void* base;
    template <typename R>
    __device__ __forceinline__ void load(int blk, int l, int mu, bool, cpx<R>* u) const {
        load_link<P, R, ONCE>(base, blk, l, mu, u);
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
        if (MU == 3) time_boundary_phase(g, wraps_time(g, p, MU, +1, in), &psi[0].re, 24);
        lk.template load<R>(p.blk, l, MU, true, u);
        hop_term<MU, -1>(u, psi, acc);
    }
    nb = neighbour(g, p, l, MU, -1, &nl, &in);
    if (ls.want(in)) {
        cpx<R> psi[12], u[9];
        ls.template load_nb<R>(nb, nl, in, psi);
        if (MU == 3) time_boundary_phase(g, wraps_time(g, p, MU, -1, in), &psi[0].re, 24);
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

// The same sum as a loop over the eight hops that is not unrolled: each
// iteration issues one neighbour's loads, so the registers held by loads in
// flight stay bounded (for kernels whose other state already fills the
// register file).
template <typename R, typename LS, typename LL>
__device__ __forceinline__ void hopping_sum_rolled(const Geom& g, const BlockPos& p, int l, const LS& ls,
                                                   const LL& lk, cpx<R>* acc) {
#pragma unroll 1
    for (int h = 0; h < 8; ++h) {
        const int mu = h >> 1, dir = (h & 1) ? -1 : +1;
        // per-direction geometry by selection (a runtime index into the small
        // arrays would put them in scratch memory)
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
        if (!ls.want(in)) continue;
        cpx<R> psi[12], u[9];
        ls.template load_nb<R>(nb, nl, in, psi);
        if (mu == 3) time_boundary_phase(g, !in && (dir > 0 ? bc == nbm - 1 : bc == 0), &psi[0].re, 24);
        if (dir > 0) lk.template load<R>(p.blk, l, mu, true, u);
        else lk.template load<R>(nb, nl, mu, in, u);
        switch (h) {
        case 0: hop_term<0, -1>(u, psi, acc); break;
        case 1: hop_term<0, +1>(u, psi, acc); break;
        case 2: hop_term<1, -1>(u, psi, acc); break;
        case 3: hop_term<1, +1>(u, psi, acc); break;
        case 4: hop_term<2, -1>(u, psi, acc); break;
        case 5: hop_term<2, +1>(u, psi, acc); break;
        case 6: hop_term<3, -1>(u, psi, acc); break;
        default: hop_term<3, +1>(u, psi, acc); break;
        }
    }
}

}  // namespace cs
