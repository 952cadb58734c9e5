// Gradient of a real function of the solution x = D^{-1} b with respect to
// the gauge links (the force), for the operator of the paper's Eq. (1)
// (Section 2).  With y = D^{-dag} eta (eta = dL/dx from the caller), every
// variation dD of the operator changes L by -Re(y^dag dD x).  Links are varied
// in left Lie-algebra coordinates, U -> exp(i w T^a) U with T^a = lambda^a / 2,
// and the kernel returns g_{mu,a}(x) = dL/dw for all eight generators, plus
// optionally the 3x3 tangent-space gradient G = 2 i (sum_a g_a T^a) U.
//
// Hopping part (U_mu(x) appears once forward at row x, once backward at row
// x+mu):  g_a = -kappa Im tr[T^a (U X1 - X2 U^dag)], with
//   X1 = sum over the two projected spins of h (x) k^dag,
//        h = P_-(x(x+mu)), k = P_-(y(x))      (P_-: spin projection of 1 - gamma_mu)
//   X2 = same with h = P_+(x(x)), k = P_+(y(x+mu)).
// Clover part: y^dag (sigma (x) F) x = tr(F Lambda) with the insertion matrix
// Lambda_{rho sigma}(z) = sum_{s s'} sigma_{s s'} x_{s'}(z) y_s(z)^dag, so that
//   dL = (kappa c_sw / 8) sum_z sum_{rho<sigma} Im tr(dQ_{rho sigma}(z) H(z)),
//   H = Lambda + Lambda^dag.
// Each link sits in 24 plaquette leaves (3 planes x 2 plaquettes x 4
// corners).  For a leaf L U R the derivative contributes U R H L, for a leaf
// L U^dag R it contributes -R H L U^dag, and g_a = (kappa c_sw / 8)
// Re tr(T^a W) for the sum W of these terms.
#include <mutex>

#include "dslash_core.hpp"
#include "su3.hpp"

namespace cs {

namespace {

using C64 = cpx<double>;
constexpr int TPB = BLOCK_SITES;

// Insertion matrices, double2 [nblk][6 planes][9][256], planes ordered
// (x,y), (x,z), (x,t), (y,z), (y,t), (z,t).
__device__ __forceinline__ int plane_of(int r, int s) {
    // r < s
    return r == 0 ? s - 1 : (r == 1 ? s + 1 : 5);
}

// outer product accumulation o += w * u (x) v^dag, w = (wr + i wi)
__device__ __forceinline__ void outer_acc(C64* o, const C64* u, const C64* v, double wr, double wi) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const C64 p = u[a] * conj(v[b]);
            o[a * 3 + b].re += wr * p.re - wi * p.im;
            o[a * 3 + b].im += wr * p.im + wi * p.re;
        }
}

// In the chiral basis sigma_{rho sigma} = diag(c0 s_m, c1 s_m) (Pauli s_m on
// the two spins of each chirality): (x,y): -s3, -s3; (x,z): s2, s2;
// (x,t): s1, -s1; (y,z): -s1, -s1; (y,t): s2, -s2; (z,t): s3, -s3.
__global__ __launch_bounds__(TPB) void k_force_insertion(Geom g, const void* __restrict__ xs,
                                                         const void* __restrict__ ys,
                                                         double2* __restrict__ H) {
    const int blk = blockIdx.x, l = threadIdx.x;
    C64 x[12], y[12];
    SpinorIO<P_F64>::load(xs, g.nblk, blk, l, x);
    SpinorIO<P_F64>::load(ys, g.nblk, blk, l, y);
    const int pm[6] = {3, 2, 1, 1, 2, 3};
    const double c0[6] = {-1, 1, 1, -1, 1, 1};
    const double c1[6] = {-1, 1, -1, -1, -1, -1};
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        C64 L[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) L[i] = {0.0, 0.0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double c = h == 0 ? c0[p] : c1[p];
            const C64* x0 = x + 6 * h;      // spin 2h
            const C64* x1 = x + 6 * h + 3;  // spin 2h+1
            const C64* y0 = y + 6 * h;
            const C64* y1 = y + 6 * h + 3;
            // sum_{s s'} (s_m)_{s s'} x_{s'} y_s^dag
            if (pm[p] == 1) {          // s1: (0,1) = (1,0) = 1
                outer_acc(L, x1, y0, c, 0);
                outer_acc(L, x0, y1, c, 0);
            } else if (pm[p] == 2) {   // s2: (0,1) = -i, (1,0) = i
                outer_acc(L, x1, y0, 0, -c);
                outer_acc(L, x0, y1, 0, c);
            } else {                   // s3: (0,0) = 1, (1,1) = -1
                outer_acc(L, x0, y0, c, 0);
                outer_acc(L, x1, y1, -c, 0);
            }
        }
        double2* dst = H + ((size_t)blk * 6 + p) * 9 * TPB + l;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const C64 v = L[a * 3 + b] + conj(L[b * 3 + a]);
                dst[(a * 3 + b) * TPB] = make_double2(v.re, v.im);
            }
    }
}

__device__ __forceinline__ void load_H(const double2* H, int blk, int l, int p, C64* h) {
    const double2* src = H + ((size_t)blk * 6 + p) * 9 * TPB + l;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double2 v = src[i * TPB];
        h[i] = {v.x, v.y};
    }
}

struct Pos {
    int c[4];
};

__device__ __forceinline__ void link_at(const Geom& g, const void* links, const int* x, int r, int da,
                                        int s, int db, int dir, C64* u) {
    int c[4] = {x[0], x[1], x[2], x[3]};
    c[r] = (c[r] + da + 2 * g.L[r]) % g.L[r];
    c[s] = (c[s] + db + 2 * g.L[s]) % g.L[s];
    int blk, l;
    site_to_internal(g, c, &blk, &l);
    load_link<P_F64, double, false>(links, blk, l, dir, u);
}

// One leaf factor in (rho, sigma) units: offset (a, b), direction (0 = rho,
// 1 = sigma), daggered.  The four leaves of Q_{rho sigma}(z), each a closed
// counter-clockwise loop from z:
//   U_r(z) U_s(z+r) U_r(z+s)^dag U_s(z)^dag
//   U_s(z) U_r(z-r+s)^dag U_s(z-r)^dag U_r(z-r)
//   U_r(z-r)^dag U_s(z-r-s)^dag U_r(z-r-s) U_s(z-s)
//   U_s(z-s)^dag U_r(z-s) U_s(z-s+r) U_r(z)^dag
struct LeafF {
    int a, b, dir, dag;
};
__device__ __forceinline__ LeafF leaf_factor(int leaf, int f) {
    switch (leaf * 4 + f) {
    case 0: return {0, 0, 0, 0};
    case 1: return {1, 0, 1, 0};
    case 2: return {0, 1, 0, 1};
    case 3: return {0, 0, 1, 1};
    case 4: return {0, 0, 1, 0};
    case 5: return {-1, 1, 0, 1};
    case 6: return {-1, 0, 1, 1};
    case 7: return {-1, 0, 0, 0};
    case 8: return {-1, 0, 0, 1};
    case 9: return {-1, -1, 1, 1};
    case 10: return {-1, -1, 0, 0};
    case 11: return {0, -1, 1, 0};
    case 12: return {0, -1, 1, 1};
    case 13: return {0, -1, 0, 0};
    case 14: return {1, -1, 1, 0};
    default: return {0, 0, 0, 1};
    }
}

// W += the derivative terms of the 8 leaves of plane (r, s) (r < s) that
// contain the link U_mu(x), mu = r (role 0) or s (role 1).
__device__ void clover_terms(const Geom& g, const void* links, const double2* H, const int* x, int r,
                             int s, int role, const C64* U, C64* W) {
    const int p = plane_of(r, s);
#pragma unroll 1
    for (int leaf = 0; leaf < 4; ++leaf) {
#pragma unroll 1
        for (int f = 0; f < 4; ++f) {
            const LeafF F = leaf_factor(leaf, f);
            if (F.dir != role) continue;
            // corner z = x - (a r + b s); the leaf's other factors relative to x
            C64 Lp[9], Rp[9], t[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                Lp[i] = {0.0, 0.0};
                Rp[i] = {0.0, 0.0};
            }
            Lp[0] = Lp[4] = Lp[8] = {1.0, 0.0};
            Rp[0] = Rp[4] = Rp[8] = {1.0, 0.0};
#pragma unroll 1
            for (int q = 0; q < 4; ++q) {
                if (q == f) continue;
                const LeafF G = leaf_factor(leaf, q);
                link_at(g, links, x, r, G.a - F.a, s, G.b - F.b, G.dir == 0 ? r : s, t);
                if (G.dag) m3_dag(t, t);
                if (q < f) m3_mul(Lp, t, Lp);
                else m3_mul(Rp, t, Rp);
            }
            int c[4] = {x[0], x[1], x[2], x[3]};
            c[r] = (c[r] - F.a + 2 * g.L[r]) % g.L[r];
            c[s] = (c[s] - F.b + 2 * g.L[s]) % g.L[s];
            int zb, zl;
            site_to_internal(g, c, &zb, &zl);
            C64 h[9];
            load_H(H, zb, zl, p, h);
            m3_mul(Rp, h, t);   // R H
            m3_mul(t, Lp, t);   // R H L
            if (!F.dag) {
                m3_mul(U, t, t);  // U R H L
#pragma unroll
                for (int i = 0; i < 9; ++i) W[i] = W[i] + t[i];
            } else {
                m3_mul_nd(t, U, t);  // R H L U^dag
#pragma unroll
                for (int i = 0; i < 9; ++i) W[i] = W[i] - t[i];
            }
        }
    }
}

// Re / Im tr(T^a M), T^a = lambda^a / 2
__device__ __forceinline__ void trace_generators(const C64* M, double* re, double* im) {
    const double is3 = 0.57735026918962576451;  // 1/sqrt(3)
    C64 t[8];
    t[0] = M[3] + M[1];
    t[1] = mul_i(M[1] - M[3]);
    t[2] = M[0] - M[4];
    t[3] = M[6] + M[2];
    t[4] = mul_i(M[2] - M[6]);
    t[5] = M[7] + M[5];
    t[6] = mul_i(M[5] - M[7]);
    t[7] = is3 * (M[0] + M[4] - 2.0 * M[8]);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        re[a] = 0.5 * t[a].re;
        im[a] = 0.5 * t[a].im;
    }
}

// X1 (S = -1) or X2 (S = +1) of one hop: sum over projected spins of h (x) k^dag
template <int MU, int S>
__device__ __forceinline__ void hop_outer(const C64* xa, const C64* yb, C64* X) {
    C64 h[6], k[6];
    spin_project<MU, S>(xa, h);
    spin_project<MU, S>(yb, k);
#pragma unroll
    for (int i = 0; i < 9; ++i) X[i] = {0.0, 0.0};
    outer_acc(X, h, k, 1.0, 0.0);
    outer_acc(X, h + 3, k + 3, 1.0, 0.0);
}

__global__ __launch_bounds__(TPB) void k_force_link(Geom g, const void* __restrict__ links, double kappa,
                                                    double csw, const void* __restrict__ xs,
                                                    const void* __restrict__ ys,
                                                    const double2* __restrict__ H, double* glie,
                                                    double2* gradU) {
    const int blk = blockIdx.x, l = threadIdx.x, mu = blockIdx.y;
    int x[4];
    internal_coords(g, blk, l, x);
    const long long site = x[0] + (long long)g.L[0] * (x[1] + (long long)g.L[1] * (x[2] + (long long)g.L[2] * x[3]));
    C64 U[9];
    load_link<P_F64, double, false>(links, blk, l, mu, U);

    // hopping part
    double gh[8];
    {
        int c[4] = {x[0], x[1], x[2], x[3]};
        c[mu] = (c[mu] + 1) % g.L[mu];
        int nb, nl;
        site_to_internal(g, c, &nb, &nl);
        C64 xo[12], yo[12], xn[12], yn[12];
        SpinorIO<P_F64>::load(xs, g.nblk, blk, l, xo);
        SpinorIO<P_F64>::load(ys, g.nblk, blk, l, yo);
        SpinorIO<P_F64>::load(xs, g.nblk, nb, nl, xn);
        SpinorIO<P_F64>::load(ys, g.nblk, nb, nl, yn);
        C64 X1[9], X2[9], M[9], t[9];
        switch (mu) {
        case 0: hop_outer<0, -1>(xn, yo, X1); hop_outer<0, +1>(xo, yn, X2); break;
        case 1: hop_outer<1, -1>(xn, yo, X1); hop_outer<1, +1>(xo, yn, X2); break;
        case 2: hop_outer<2, -1>(xn, yo, X1); hop_outer<2, +1>(xo, yn, X2); break;
        default: hop_outer<3, -1>(xn, yo, X1); hop_outer<3, +1>(xo, yn, X2); break;
        }
        m3_mul(U, X1, M);
        m3_mul_nd(X2, U, t);
#pragma unroll
        for (int i = 0; i < 9; ++i) M[i] = M[i] - t[i];
        double re[8], im[8];
        trace_generators(M, re, im);
        // both hop terms of the link U_t(x) on the last time slice cross the
        // time boundary: with antiperiodic fields they carry a factor -1
        const double hs = (mu == 3 && g.antiperiodic_t && x[3] == g.L[3] - 1) ? -1.0 : 1.0;
#pragma unroll
        for (int a = 0; a < 8; ++a) gh[a] = -hs * kappa * im[a];
    }

    // clover part
    double gc[8];
    {
        C64 W[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) W[i] = {0.0, 0.0};
        if (csw != 0.0) {
#pragma unroll 1
            for (int nu = 0; nu < 4; ++nu) {
                if (nu == mu) continue;
                if (mu < nu) clover_terms(g, links, H, x, mu, nu, 0, U, W);
                else clover_terms(g, links, H, x, nu, mu, 1, U, W);
            }
        }
        double re[8], im[8];
        trace_generators(W, re, im);
        const double pref = kappa * csw / 8.0;
#pragma unroll
        for (int a = 0; a < 8; ++a) gc[a] = pref * re[a];
    }

    double gt[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) gt[a] = gh[a] + gc[a];
    if (glie) {
        double* o = glie + (site * 4 + mu) * 8;
#pragma unroll
        for (int a = 0; a < 8; ++a) o[a] = gt[a];
    }
    if (gradU) {
        // P = sum_a g_a T^a, G = 2 i P U
        const double is3 = 0.57735026918962576451;
        C64 P[9];
        P[0] = {0.5 * (gt[2] + gt[7] * is3), 0.0};
        P[4] = {0.5 * (-gt[2] + gt[7] * is3), 0.0};
        P[8] = {-gt[7] * is3, 0.0};
        P[1] = {0.5 * gt[0], -0.5 * gt[1]};
        P[3] = {0.5 * gt[0], 0.5 * gt[1]};
        P[2] = {0.5 * gt[3], -0.5 * gt[4]};
        P[6] = {0.5 * gt[3], 0.5 * gt[4]};
        P[5] = {0.5 * gt[5], -0.5 * gt[6]};
        P[7] = {0.5 * gt[5], 0.5 * gt[6]};
        C64 G[9];
        m3_mul(P, U, G);
        double2* o = gradU + (site * 4 + mu) * 9;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const C64 v = mul_i(G[i]);
            o[i] = make_double2(2.0 * v.re, 2.0 * v.im);
        }
    }
}

// Workspace of the allocation-free entry point: the insertion matrices of
// up to FORCE_SCRATCH_BYTES / 864 sites, in a fixed device array that every
// GPU the library runs on holds until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is a stand-in, not a
// device address): the address comes from hipGetSymbolAddress, once per
// device, on that device.
__device__ __align__(256) double2 scratch[FORCE_SCRATCH_BYTES / sizeof(double2)];

std::mutex g_scratch_mu;
void* g_scratch_ptr[FORCE_SCRATCH_MAX_DEVICES] = {};

}  // namespace

hipError_t force_scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= FORCE_SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_force(const Geom& g, const void* links64, double kappa, double csw, const void* x,
                        const void* y, void* Hbuf, double* glie, void* gradU, hipStream_t s) {
    ProfScope ps("force", s);
    hipLaunchKernelGGL(k_force_insertion, dim3(g.nblk), dim3(TPB), 0, s, g, x, y, (double2*)Hbuf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_force_link, dim3(g.nblk, 4), dim3(TPB), 0, s, g, links64, kappa, csw, x, y,
                       (const double2*)Hbuf, glie, (double2*)gradU);
    return hipGetLastError();
}

}  // namespace cs
