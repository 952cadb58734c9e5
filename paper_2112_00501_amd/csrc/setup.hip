// Field setup, run once per gauge field: link compression into the internal
// layout, the clover term C = 1 + T of the paper's Eq. (1) (Section 2; the
// paper leaves building C from the gauge field to the user), and conversion
// of spinors between the canonical and the internal layouts.
#include "fields.hpp"
#include "su3.hpp"

namespace cs {

namespace {

constexpr int TPB = BLOCK_SITES;

__global__ __launch_bounds__(TPB) void k_import_links(Geom g, const double2* __restrict__ U,
                                                      void* l64, void* l32, void* l16, void* lbf) {
    const int blk = blockIdx.x, l = threadIdx.x;
    const long long s = canonical_site(g, blk, l);
    for (int mu = 0; mu < 4; ++mu) {
        cpx<double> u[6];
        const double2* src = U + (s * 4 + mu) * 9;  // rows 0 and 1 are entries 0..5
#pragma unroll
        for (int k = 0; k < 6; ++k) u[k] = {src[k].x, src[k].y};
        LinkIO<P_F64>::store6(l64, blk, l, mu, u);
        LinkIO<P_F32>::store6(l32, blk, l, mu, u);
        LinkIO<P_F16>::store6(l16, blk, l, mu, u);
        LinkIO<P_BF16>::store6(lbf, blk, l, mu, u);
    }
}

using C64 = cpx<double>;

__device__ __forceinline__ void link_at(const Geom& g, const void* links, const int* x, int da,
                                        int db, int mu, int nu, int dir, C64* u) {
    int c[4] = {x[0], x[1], x[2], x[3]};
    c[mu] = (c[mu] + da + g.L[mu]) % g.L[mu];
    c[nu] = (c[nu] + db + g.L[nu]) % g.L[nu];
    int blk, l;
    site_to_internal(g, c, &blk, &l);
    load_link<P_F64, double>(links, blk, l, dir, u);
}

// Q_{mu nu}(x): the four counter-clockwise plaquettes starting at x:
//   U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
//   U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu)
//   U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu)
//   U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^dag
__device__ void leaf_sum(const Geom& g, const void* links, const int* x, int mu, int nu, C64* Q) {
    C64 a[9], b[9], p[9];
    // leaf 1
    link_at(g, links, x, 0, 0, mu, nu, mu, a);
    link_at(g, links, x, 1, 0, mu, nu, nu, b);
    m3_mul(a, b, p);
    link_at(g, links, x, 0, 1, mu, nu, mu, a);
    m3_mul_nd(p, a, p);
    link_at(g, links, x, 0, 0, mu, nu, nu, a);
    m3_mul_nd(p, a, p);
#pragma unroll
    for (int i = 0; i < 9; ++i) Q[i] = p[i];
    // leaf 2
    link_at(g, links, x, 0, 0, mu, nu, nu, a);
    link_at(g, links, x, -1, 1, mu, nu, mu, b);
    m3_mul_nd(a, b, p);
    link_at(g, links, x, -1, 0, mu, nu, nu, a);
    m3_mul_nd(p, a, p);
    link_at(g, links, x, -1, 0, mu, nu, mu, a);
    m3_mul(p, a, p);
#pragma unroll
    for (int i = 0; i < 9; ++i) Q[i] = Q[i] + p[i];
    // leaf 3
    link_at(g, links, x, -1, 0, mu, nu, mu, a);
    link_at(g, links, x, -1, -1, mu, nu, nu, b);
    m3_mul(b, a, p);  // (U_nu U_mu)^dag = U_mu^dag U_nu^dag
    m3_dag(p, p);
    link_at(g, links, x, -1, -1, mu, nu, mu, a);
    m3_mul(p, a, p);
    link_at(g, links, x, 0, -1, mu, nu, nu, a);
    m3_mul(p, a, p);
#pragma unroll
    for (int i = 0; i < 9; ++i) Q[i] = Q[i] + p[i];
    // leaf 4
    link_at(g, links, x, 0, -1, mu, nu, nu, a);
    link_at(g, links, x, 0, -1, mu, nu, mu, b);
    m3_mul_dn(a, b, p);
    link_at(g, links, x, 1, -1, mu, nu, nu, a);
    m3_mul(p, a, p);
    link_at(g, links, x, 0, 0, mu, nu, mu, a);
    m3_mul_nd(p, a, p);
#pragma unroll
    for (int i = 0; i < 9; ++i) Q[i] = Q[i] + p[i];
}

// Upper-triangle slot of entry (i, j), i < j, of a 6x6 matrix, row-major.
__device__ __forceinline__ int up_slot(int i, int j) { return i * 6 - i * (i + 1) / 2 + (j - i - 1); }

// In the chiral basis T = diag(T+, T-), and with G1, G2, G3 the colour
// matrices multiplying sigma_1, sigma_2, sigma_3 (on the local spin pair),
//   T(h) = i kappa c_sw [[G3, G1 - i G2], [G1 + i G2, -G3]]
// where, from sigma_{kl} = -eps_{klm} diag(s_m, s_m) and
// sigma_{kt} = diag(s_k, -s_k):
//   G1 = -F_yz + sgn F_xt,  G2 = F_xz + sgn F_yt,  G3 = -F_xy + sgn F_zt,
// sgn = +1 for h = 0 and -1 for h = 1.
// Accumulates the contribution w * F to G_k of chirality h into the packed
// (1 + T) entries m[72] (host order: 6 diagonals then 15 upper entries).
__device__ void add_to_packed(double* m, int h, int k, double w, const C64* F, double kc) {
    double* d = m + 36 * h;
    double* up = d + 6;
    // H = i kc w F (Hermitian for anti-Hermitian F)
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const C64 H = kc * w * mul_i(F[a * 3 + b]);
            if (k == 3) {  // upper-left +H, lower-right -H (upper triangles only)
                if (a == b) {
                    d[a] += H.re;
                    d[3 + a] -= H.re;
                } else if (a < b) {
                    const int s1 = up_slot(a, b), s2 = up_slot(3 + a, 3 + b);
                    up[2 * s1] += H.re;
                    up[2 * s1 + 1] += H.im;
                    up[2 * s2] -= H.re;
                    up[2 * s2 + 1] -= H.im;
                }
            } else {  // upper-right block: H (k = 1) or -i H (k = 2)
                const C64 E = (k == 1) ? H : mul_mi(H);
                const int s = up_slot(a, 3 + b);
                up[2 * s] += E.re;
                up[2 * s + 1] += E.im;
            }
        }
}

__global__ __launch_bounds__(TPB) void k_clover_build(Geom g, const void* __restrict__ links,
                                                      double kappa, double csw, double2* c64,
                                                      float4* c32) {
    const int blk = blockIdx.x, l = threadIdx.x;
    int x[4];
    internal_coords(g, blk, l, x);
    double m[72];
    for (int i = 0; i < 72; ++i) m[i] = 0.0;
    for (int i = 0; i < 6; ++i) {
        m[i] = 1.0;
        m[36 + i] = 1.0;
    }
    const double kc = kappa * csw;
    // (mu, nu, G index, weight for h = 0, weight for h = 1)
    const int planes[6][2] = {{0, 1}, {0, 2}, {1, 2}, {0, 3}, {1, 3}, {2, 3}};
    const int gk[6] = {3, 2, 1, 1, 2, 3};
    const double w0[6] = {-1, 1, -1, 1, 1, 1};
    const double w1[6] = {-1, 1, -1, -1, -1, -1};
    for (int pl = 0; pl < 6; ++pl) {
        C64 Q[9], F[9];
        leaf_sum(g, links, x, planes[pl][0], planes[pl][1], Q);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const C64 q = Q[a * 3 + b], qt = conj(Q[b * 3 + a]);
                F[a * 3 + b] = 0.125 * (q - qt);
            }
        add_to_packed(m, 0, gk[pl], w0[pl], F, kc);
        add_to_packed(m, 1, gk[pl], w1[pl], F, kc);
    }
    double2* p64 = c64 + (size_t)blk * 36 * BLOCK_SITES + l;
    for (int k = 0; k < 36; ++k) p64[k * BLOCK_SITES] = make_double2(m[2 * k], m[2 * k + 1]);
    float4* p32 = c32 + (size_t)blk * 18 * BLOCK_SITES + l;
    for (int k = 0; k < 18; ++k)
        p32[k * BLOCK_SITES] = make_float4((float)m[4 * k], (float)m[4 * k + 1], (float)m[4 * k + 2],
                                           (float)m[4 * k + 3]);
}

// Canonical [V][12][12] matrix of a packed field: T = (1 + T) - 1 for the
// clover term (minus_one), or the packed matrix itself (its inverse).
__global__ __launch_bounds__(TPB) void k_clover_export(Geom g, const double2* __restrict__ c64,
                                                       double2* __restrict__ out, double minus_one) {
    const int blk = blockIdx.x, l = threadIdx.x;
    const long long s = canonical_site(g, blk, l);
    double m[72];
    CloverIO<double>::load(c64, blk, l, m);
    double2* T = out + s * 144;
    for (int i = 0; i < 144; ++i) T[i] = make_double2(0.0, 0.0);
    for (int h = 0; h < 2; ++h) {
        const double* d = m + 36 * h;
        const double* up = d + 6;
        const int o = 6 * h;
        for (int i = 0; i < 6; ++i) T[(o + i) * 12 + o + i] = make_double2(d[i] - minus_one, 0.0);
        for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j) {
                const int k = up_slot(i, j);
                T[(o + i) * 12 + o + j] = make_double2(up[2 * k], up[2 * k + 1]);
                T[(o + j) * 12 + o + i] = make_double2(up[2 * k], -up[2 * k + 1]);
            }
    }
}

// (1 + T)^-1 per site and chirality (grid.y): each 6x6 block of 1 + T is
// Hermitian positive definite (the clover term is small against the unit
// matrix: its norm is below 6 kappa c_SW times the norm of F), so in-place
// Gauss-Jordan elimination without pivoting inverts it; the result is
// symmetrised and packed like the clover term, in FP64 and FP32.
__global__ __launch_bounds__(TPB) void k_clover_invert(Geom g, const double2* __restrict__ c64,
                                                       double2* __restrict__ ci64, float4* __restrict__ ci32) {
    const int blk = blockIdx.x, h = blockIdx.y, l = threadIdx.x;
    const double2* p = c64 + ((size_t)blk * 36 + 18 * h) * BLOCK_SITES + l;
    double m[36];
    for (int k = 0; k < 18; ++k) {
        const double2 v = p[k * BLOCK_SITES];
        m[2 * k] = v.x;
        m[2 * k + 1] = v.y;
    }
    cpx<double> a[6][6];
    for (int i = 0; i < 6; ++i) {
        a[i][i] = {m[i], 0.0};
        for (int j = i + 1; j < 6; ++j) {
            const int k = up_slot(i, j);
            a[i][j] = {m[6 + 2 * k], m[7 + 2 * k]};
            a[j][i] = {m[6 + 2 * k], -m[7 + 2 * k]};
        }
    }
    for (int k = 0; k < 6; ++k) {
        const cpx<double> piv = a[k][k];
        const double n2 = piv.re * piv.re + piv.im * piv.im;
        const cpx<double> ip = {piv.re / n2, -piv.im / n2};
        a[k][k] = {1.0, 0.0};
        for (int j = 0; j < 6; ++j) a[k][j] = a[k][j] * ip;
        for (int i = 0; i < 6; ++i) {
            if (i == k) continue;
            const cpx<double> f = a[i][k];
            a[i][k] = {0.0, 0.0};
            for (int j = 0; j < 6; ++j) a[i][j] = a[i][j] - f * a[k][j];
        }
    }
    for (int i = 0; i < 6; ++i) {
        m[i] = a[i][i].re;
        for (int j = i + 1; j < 6; ++j) {
            const int k = up_slot(i, j);
            m[6 + 2 * k] = 0.5 * (a[i][j].re + a[j][i].re);
            m[7 + 2 * k] = 0.5 * (a[i][j].im - a[j][i].im);
        }
    }
    double2* q64 = ci64 + ((size_t)blk * 36 + 18 * h) * BLOCK_SITES + l;
    for (int k = 0; k < 18; ++k) q64[k * BLOCK_SITES] = make_double2(m[2 * k], m[2 * k + 1]);
    float4* q32 = ci32 + ((size_t)blk * 18 + 9 * h) * BLOCK_SITES + l;
    for (int k = 0; k < 9; ++k)
        q32[k * BLOCK_SITES] = make_float4((float)m[4 * k], (float)m[4 * k + 1], (float)m[4 * k + 2],
                                           (float)m[4 * k + 3]);
}

template <int P>
__global__ __launch_bounds__(TPB) void k_field_import(Geom g, void* dst, const double2* src,
                                                      size_t dst_stride, long long V) {
    const int blk = blockIdx.x, l = threadIdx.x, r = blockIdx.y;
    using R = typename SpinorIO<P>::R;
    const long long s = canonical_site(g, blk, l);
    const double2* p = src + ((long long)r * V + s) * 12;
    cpx<R> c[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) c[k] = {(R)p[k].x, (R)p[k].y};
    SpinorIO<P>::store((char*)dst + r * dst_stride, g.nblk, blk, l, c);
}

template <int P>
__global__ __launch_bounds__(TPB) void k_field_export(Geom g, double2* dst, const void* src,
                                                      size_t src_stride, long long V) {
    const int blk = blockIdx.x, l = threadIdx.x, r = blockIdx.y;
    using R = typename SpinorIO<P>::R;
    const long long s = canonical_site(g, blk, l);
    cpx<R> c[12];
    SpinorIO<P>::load((const char*)src + r * src_stride, g.nblk, blk, l, c);
    double2* p = dst + ((long long)r * V + s) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = make_double2((double)c[k].re, (double)c[k].im);
}

}  // namespace

hipError_t launch_import_links(const Geom& g, const void* U, void* l64, void* l32, void* l16,
                               void* lbf, hipStream_t s) {
    ProfScope ps("setup", s);
    hipLaunchKernelGGL(k_import_links, dim3(g.nblk), dim3(TPB), 0, s, g, (const double2*)U, l64, l32,
                       l16, lbf);
    return hipGetLastError();
}

hipError_t launch_clover_build(const Geom& g, const void* links64, double kappa, double csw,
                               void* c64, void* c32, hipStream_t s) {
    ProfScope ps("clover_build", s);
    hipLaunchKernelGGL(k_clover_build, dim3(g.nblk), dim3(TPB), 0, s, g, links64, kappa, csw,
                       (double2*)c64, (float4*)c32);
    return hipGetLastError();
}

hipError_t launch_clover_export(const Geom& g, const void* c64, void* dst, bool inverse, hipStream_t s) {
    hipLaunchKernelGGL(k_clover_export, dim3(g.nblk), dim3(TPB), 0, s, g, (const double2*)c64,
                       (double2*)dst, inverse ? 0.0 : 1.0);
    return hipGetLastError();
}

hipError_t launch_clover_invert(const Geom& g, const void* c64, void* ci64, void* ci32, hipStream_t s) {
    ProfScope ps("clover_build", s);
    hipLaunchKernelGGL(k_clover_invert, dim3(g.nblk, 2), dim3(TPB), 0, s, g, (const double2*)c64,
                       (double2*)ci64, (float4*)ci32);
    return hipGetLastError();
}

hipError_t launch_field_import(const Geom& g, int prec, void* dst, const void* src, int nrhs,
                               hipStream_t s) {
    const size_t stride = spinor_bytes_per_site(prec) * g.V;
    const dim3 grid(g.nblk, nrhs);
    switch (prec) {
    case P_F64: hipLaunchKernelGGL(k_field_import<P_F64>, grid, dim3(TPB), 0, s, g, dst, (const double2*)src, stride, g.V); break;
    case P_F32: hipLaunchKernelGGL(k_field_import<P_F32>, grid, dim3(TPB), 0, s, g, dst, (const double2*)src, stride, g.V); break;
    case P_F16: hipLaunchKernelGGL(k_field_import<P_F16>, grid, dim3(TPB), 0, s, g, dst, (const double2*)src, stride, g.V); break;
    case P_BF16: hipLaunchKernelGGL(k_field_import<P_BF16>, grid, dim3(TPB), 0, s, g, dst, (const double2*)src, stride, g.V); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_field_export(const Geom& g, int prec, void* dst, const void* src, int nrhs,
                               hipStream_t s) {
    const size_t stride = spinor_bytes_per_site(prec) * g.V;
    const dim3 grid(g.nblk, nrhs);
    switch (prec) {
    case P_F64: hipLaunchKernelGGL(k_field_export<P_F64>, grid, dim3(TPB), 0, s, g, (double2*)dst, src, stride, g.V); break;
    case P_F32: hipLaunchKernelGGL(k_field_export<P_F32>, grid, dim3(TPB), 0, s, g, (double2*)dst, src, stride, g.V); break;
    case P_F16: hipLaunchKernelGGL(k_field_export<P_F16>, grid, dim3(TPB), 0, s, g, (double2*)dst, src, stride, g.V); break;
    case P_BF16: hipLaunchKernelGGL(k_field_export<P_BF16>, grid, dim3(TPB), 0, s, g, (double2*)dst, src, stride, g.V); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace cs
