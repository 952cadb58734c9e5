// Device-side loads and stores of spinors, compressed links and the clover
// term in the internal block layout (see cs_internal.hpp), for every storage
// precision, plus the site-local algebra shared by the kernels: SU(3) row
// reconstruction, spin projection for the hopping term, and the clover
// matrix-vector product.
#pragma once

#include "cs_internal.hpp"

namespace cs {

template <int P>
struct Arith { using R = float; };
template <>
struct Arith<P_F64> { using R = double; };

// ---------------------------------------------------------------- 16-bit types

template <int P>
__device__ __forceinline__ unsigned short f2h(float v);
template <>
__device__ __forceinline__ unsigned short f2h<P_F16>(float v) {
    return __builtin_bit_cast(unsigned short, (_Float16)v);
}
template <>
__device__ __forceinline__ unsigned short f2h<P_BF16>(float v) {
    return __builtin_bit_cast(unsigned short, (__bf16)v);
}
template <int P>
__device__ __forceinline__ float h2f(unsigned short v);
template <>
__device__ __forceinline__ float h2f<P_F16>(unsigned short v) {
    return (float)__builtin_bit_cast(_Float16, v);
}
template <>
__device__ __forceinline__ float h2f<P_BF16>(unsigned short v) {
    return __builtin_bit_cast(float, (unsigned int)v << 16);
}
template <int P>
__device__ __forceinline__ unsigned int pack2(float a, float b) {
    return (unsigned int)f2h<P>(a) | ((unsigned int)f2h<P>(b) << 16);
}
template <int P>
__device__ __forceinline__ void unpack2(unsigned int w, float& a, float& b) {
    a = h2f<P>((unsigned short)(w & 0xffffu));
    b = h2f<P>((unsigned short)(w >> 16));
}

// -------------------------------------------------------------------- spinors

template <int P>
struct SpinorIO;

template <>
struct SpinorIO<P_F64> {
    using R = double;
    __device__ static void load(const void* base, int, int blk, int l, cpx<R>* c) {
        const double2* p = (const double2*)base + (size_t)blk * 12 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double2 v = p[k * BLOCK_SITES];
            c[k] = {v.x, v.y};
        }
    }
    __device__ static void store(void* base, int, int blk, int l, const cpx<R>* c) {
        double2* p = (double2*)base + (size_t)blk * 12 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 12; ++k) p[k * BLOCK_SITES] = make_double2(c[k].re, c[k].im);
    }
};

template <>
struct SpinorIO<P_F32> {
    using R = float;
    __device__ static void load(const void* base, int, int blk, int l, cpx<R>* c) {
        const float4* p = (const float4*)base + (size_t)blk * 6 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const float4 v = p[k * BLOCK_SITES];
            c[2 * k] = {v.x, v.y};
            c[2 * k + 1] = {v.z, v.w};
        }
    }
    __device__ static void store(void* base, int, int blk, int l, const cpx<R>* c) {
        float4* p = (float4*)base + (size_t)blk * 6 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            st_once(p + k * BLOCK_SITES, make_float4(c[2 * k].re, c[2 * k].im, c[2 * k + 1].re, c[2 * k + 1].im));
    }
};

// 16-bit spinors: 3 uint4 chunks per site and one float scale per site; the
// scales follow the chunk array of the whole field.
template <int P>
struct SpinorIO16 {
    using R = float;
    // the packed words and the scale of one site, unpacked later by unpack()
    // into the values load() gives (for kernels that keep many sites' loads
    // in flight at once)
    struct Raw {
        uint4 w[3];
        float s;
    };
    __device__ static void load_raw(const void* base, int nblk, int blk, int l, Raw& r) {
        const uint4* p = (const uint4*)base + (size_t)blk * 3 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 3; ++k) r.w[k] = p[k * BLOCK_SITES];
        r.s = scales(base, nblk)[(size_t)blk * BLOCK_SITES + l];
    }
    __device__ static void unpack(const Raw& r, cpx<R>* c) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float a, b;
            unpack2<P>(r.w[k].x, a, b); c[4 * k + 0] = {a * r.s, b * r.s};
            unpack2<P>(r.w[k].y, a, b); c[4 * k + 1] = {a * r.s, b * r.s};
            unpack2<P>(r.w[k].z, a, b); c[4 * k + 2] = {a * r.s, b * r.s};
            unpack2<P>(r.w[k].w, a, b); c[4 * k + 3] = {a * r.s, b * r.s};
        }
    }
    __device__ static const float* scales(const void* base, int nblk) {
        return (const float*)((const char*)base + (size_t)nblk * BLOCK_SITES * 48);
    }
    __device__ static void load(const void* base, int nblk, int blk, int l, cpx<R>* c) {
        const uint4* p = (const uint4*)base + (size_t)blk * 3 * BLOCK_SITES + l;
        const float s = scales(base, nblk)[(size_t)blk * BLOCK_SITES + l];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint4 v = p[k * BLOCK_SITES];
            float a, b;
            unpack2<P>(v.x, a, b); c[4 * k + 0] = {a * s, b * s};
            unpack2<P>(v.y, a, b); c[4 * k + 1] = {a * s, b * s};
            unpack2<P>(v.z, a, b); c[4 * k + 2] = {a * s, b * s};
            unpack2<P>(v.w, a, b); c[4 * k + 3] = {a * s, b * s};
        }
    }
    __device__ static void store(void* base, int nblk, int blk, int l, const cpx<R>* c) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(c[k].re), fabsf(c[k].im)));
        const float inv = m > 0.f ? 1.f / m : 0.f;
        uint4* p = (uint4*)base + (size_t)blk * 3 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint4 v;
            v.x = pack2<P>(c[4 * k + 0].re * inv, c[4 * k + 0].im * inv);
            v.y = pack2<P>(c[4 * k + 1].re * inv, c[4 * k + 1].im * inv);
            v.z = pack2<P>(c[4 * k + 2].re * inv, c[4 * k + 2].im * inv);
            v.w = pack2<P>(c[4 * k + 3].re * inv, c[4 * k + 3].im * inv);
            p[k * BLOCK_SITES] = v;
        }
        ((float*)scales(base, nblk))[(size_t)blk * BLOCK_SITES + l] = m;
    }
};
template <>
struct SpinorIO<P_F16> : SpinorIO16<P_F16> {};
template <>
struct SpinorIO<P_BF16> : SpinorIO16<P_BF16> {};

// ---------------------------------------------------------------------- links

// Row 2 of an SU(3) matrix from rows 0 and 1: conj(row0 x row1).
template <typename R>
__device__ __forceinline__ void su3_row2(cpx<R>* u) {
    u[6] = conj(u[1] * u[5] - u[2] * u[4]);
    u[7] = conj(u[2] * u[3] - u[0] * u[5]);
    u[8] = conj(u[0] * u[4] - u[1] * u[3]);
}

template <int P>
struct LinkIO;

template <>
struct LinkIO<P_F64> {
    using R = double;
    // rows 0 and 1 of U_mu at (blk, l) into u[0..5]; ONCE: the load is the
    // only use of these words in the kernel
    template <bool ONCE = true>
    __device__ static void load6(const void* base, int blk, int l, int mu, cpx<R>* u) {
        const double2* p = (const double2*)base + ((size_t)blk * 4 + mu) * 6 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double2 v = ONCE ? ld_once(p + k * BLOCK_SITES) : p[k * BLOCK_SITES];
            u[k] = {v.x, v.y};
        }
    }
    __device__ static void store6(void* base, int blk, int l, int mu, const cpx<double>* u) {
        double2* p = (double2*)base + ((size_t)blk * 4 + mu) * 6 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 6; ++k) p[k * BLOCK_SITES] = make_double2(u[k].re, u[k].im);
    }
};

template <>
struct LinkIO<P_F32> {
    using R = float;
    template <bool ONCE = true>
    __device__ static void load6(const void* base, int blk, int l, int mu, cpx<R>* u) {
        const float4* p = (const float4*)base + ((size_t)blk * 4 + mu) * 3 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float4 v = ONCE ? ld_once(p + k * BLOCK_SITES) : p[k * BLOCK_SITES];
            u[2 * k] = {v.x, v.y};
            u[2 * k + 1] = {v.z, v.w};
        }
    }
    __device__ static void store6(void* base, int blk, int l, int mu, const cpx<double>* u) {
        float4* p = (float4*)base + ((size_t)blk * 4 + mu) * 3 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            p[k * BLOCK_SITES] = make_float4((float)u[2 * k].re, (float)u[2 * k].im,
                                             (float)u[2 * k + 1].re, (float)u[2 * k + 1].im);
    }
};

template <int P>
struct LinkIO16 {
    using R = float;
    template <bool ONCE = true>
    __device__ static void load6(const void* base, int blk, int l, int mu, cpx<R>* u) {
        const uint2* p = (const uint2*)base + ((size_t)blk * 4 + mu) * 3 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint2 v = ONCE ? ld_once(p + k * BLOCK_SITES) : p[k * BLOCK_SITES];
            float a, b;
            unpack2<P>(v.x, a, b); u[2 * k] = {a, b};
            unpack2<P>(v.y, a, b); u[2 * k + 1] = {a, b};
        }
    }
    __device__ static void store6(void* base, int blk, int l, int mu, const cpx<double>* u) {
        uint2* p = (uint2*)base + ((size_t)blk * 4 + mu) * 3 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint2 v;
            v.x = pack2<P>((float)u[2 * k].re, (float)u[2 * k].im);
            v.y = pack2<P>((float)u[2 * k + 1].re, (float)u[2 * k + 1].im);
            p[k * BLOCK_SITES] = v;
        }
    }
};
template <>
struct LinkIO<P_F16> : LinkIO16<P_F16> {};
template <>
struct LinkIO<P_BF16> : LinkIO16<P_BF16> {};

// Full 3x3 link (row 2 rebuilt) in arithmetic type R.
template <int P, typename R, bool ONCE = true>
__device__ __forceinline__ void load_link(const void* base, int blk, int l, int mu, cpx<R>* u) {
    using RS = typename LinkIO<P>::R;
    cpx<RS> t[6];
    LinkIO<P>::template load6<ONCE>(base, blk, l, mu, t);
#pragma unroll
    for (int k = 0; k < 6; ++k) u[k] = {(R)t[k].re, (R)t[k].im};
    su3_row2(u);
}

// --------------------------------------------------------------------- clover

// 72 reals per site: for chirality h = 0, 1: 6 diagonal reals of 1 + T_h then
// the 15 upper entries (i < j, row-major) as (re, im).
template <typename R>
struct CloverIO;

template <>
struct CloverIO<double> {
    template <bool ONCE = true>
    __device__ static void load(const void* base, int blk, int l, double* c) {
        const double2* p = (const double2*)base + (size_t)blk * 36 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 36; ++k) {
            const double2 v = ONCE ? ld_once(p + k * BLOCK_SITES) : p[k * BLOCK_SITES];
            c[2 * k] = v.x;
            c[2 * k + 1] = v.y;
        }
    }
};
template <>
struct CloverIO<float> {
    template <bool ONCE = true>
    __device__ static void load(const void* base, int blk, int l, float* c) {
        const float4* p = (const float4*)base + (size_t)blk * 18 * BLOCK_SITES + l;
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            const float4 v = ONCE ? ld_once(p + k * BLOCK_SITES) : p[k * BLOCK_SITES];
            c[4 * k] = v.x;
            c[4 * k + 1] = v.y;
            c[4 * k + 2] = v.z;
            c[4 * k + 3] = v.w;
        }
    }
};

// out = (1 + T) in, with the packed clover c[72].
template <typename R>
__device__ __forceinline__ void clover_apply(const R* c, const cpx<R>* in, cpx<R>* out) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const R* d = c + 36 * h;
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
                cmac(o[i], a, v[j]);       // upper entry (i, j)
                cmac_conj(o[j], a, v[i]);  // its mirror (j, i) = conj
            }
#pragma unroll
        for (int i = 0; i < 6; ++i) out[6 * h + i] = o[i];
    }
}

// --------------------------------------------------------------- spin algebra

// Hopping term of one direction, chiral basis (gamma5 = diag(1, 1, -1, -1),
// gamma_mu = [[0, A_mu], [A_mu^dag, 0]] with A_x = -i s1, A_y = -i s2,
// A_z = -i s3, A_t = 1).  (1 + S gamma_mu) psi has upper half
// h = psi_up + S A psi_lo and lower half S A^dag h, so only the half spinor h
// is multiplied by the link.  S = -1: forward hop (1 - gamma_mu); S = +1:
// backward hop (1 + gamma_mu).
template <int MU, int S, typename R>
__device__ __forceinline__ void spin_project(const cpx<R>* p, cpx<R>* h) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cpx<R> s0 = p[a], s1 = p[3 + a], s2 = p[6 + a], s3 = p[9 + a];
        if (MU == 0) {  // A_x psi_lo = (-i s3, -i s2)
            h[a] = S > 0 ? s0 + mul_mi(s3) : s0 + mul_i(s3);
            h[3 + a] = S > 0 ? s1 + mul_mi(s2) : s1 + mul_i(s2);
        } else if (MU == 1) {  // A_y psi_lo = (-s3, s2)
            h[a] = S > 0 ? s0 - s3 : s0 + s3;
            h[3 + a] = S > 0 ? s1 + s2 : s1 - s2;
        } else if (MU == 2) {  // A_z psi_lo = (-i s2, i s3)
            h[a] = S > 0 ? s0 + mul_mi(s2) : s0 + mul_i(s2);
            h[3 + a] = S > 0 ? s1 + mul_i(s3) : s1 + mul_mi(s3);
        } else {  // A_t psi_lo = (s2, s3)
            h[a] = S > 0 ? s0 + s2 : s0 - s2;
            h[3 + a] = S > 0 ? s1 + s3 : s1 - s3;
        }
    }
}

// acc += (upper = v, lower = S A^dag v)
template <int MU, int S, typename R>
__device__ __forceinline__ void spin_reconstruct_add(const cpx<R>* v, cpx<R>* acc) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cpx<R> v0 = v[a], v1 = v[3 + a];
        acc[a] = acc[a] + v0;
        acc[3 + a] = acc[3 + a] + v1;
        if (MU == 0) {  // A_x^dag v = (i v1, i v0)
            acc[6 + a] = S > 0 ? acc[6 + a] + mul_i(v1) : acc[6 + a] + mul_mi(v1);
            acc[9 + a] = S > 0 ? acc[9 + a] + mul_i(v0) : acc[9 + a] + mul_mi(v0);
        } else if (MU == 1) {  // A_y^dag v = (v1, -v0)
            acc[6 + a] = S > 0 ? acc[6 + a] + v1 : acc[6 + a] - v1;
            acc[9 + a] = S > 0 ? acc[9 + a] - v0 : acc[9 + a] + v0;
        } else if (MU == 2) {  // A_z^dag v = (i v0, -i v1)
            acc[6 + a] = S > 0 ? acc[6 + a] + mul_i(v0) : acc[6 + a] + mul_mi(v0);
            acc[9 + a] = S > 0 ? acc[9 + a] + mul_mi(v1) : acc[9 + a] + mul_i(v1);
        } else {  // A_t^dag v = v
            acc[6 + a] = S > 0 ? acc[6 + a] + v0 : acc[6 + a] - v0;
            acc[9 + a] = S > 0 ? acc[9 + a] + v1 : acc[9 + a] - v1;
        }
    }
}

// v = U h (two spins), or U^dag h when DAG
template <bool DAG, typename R>
__device__ __forceinline__ void su3_mul_half(const cpx<R>* u, const cpx<R>* h, cpx<R>* v) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cpx<R> t = {(R)0, (R)0};
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (DAG) cmac_conj(t, u[b * 3 + a], h[3 * s + b]);
                else cmac(t, u[a * 3 + b], h[3 * s + b]);
            }
            v[3 * s + a] = t;
        }
}

// acc += (1 + S gamma_mu) U' psi for one neighbour, U' = U (S = -1) or U^dag (S = +1)
template <int MU, int S, typename R>
__device__ __forceinline__ void hop_term(const cpx<R>* u, const cpx<R>* psi, cpx<R>* acc) {
    cpx<R> h[6], v[6];
    spin_project<MU, S>(psi, h);
    su3_mul_half<(S > 0)>(u, h, v);
    spin_reconstruct_add<MU, S>(v, acc);
}

template <typename R>
__device__ __forceinline__ void negate_lower(cpx<R>* p) {
#pragma unroll
    for (int k = 6; k < 12; ++k) p[k] = {-p[k].re, -p[k].im};
}

}  // namespace cs
