// 3x3 complex matrix products (row-major, any arithmetic type).
#pragma once

#include "cs_internal.hpp"

namespace cs {

// c = a b (c may alias a or b)
template <typename R>
__device__ __forceinline__ void m3_mul(const cpx<R>* a, const cpx<R>* b, cpx<R>* c) {
    cpx<R> t[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cpx<R> s = {(R)0, (R)0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(s, a[i * 3 + k], b[k * 3 + j]);
            t[i * 3 + j] = s;
        }
#pragma unroll
    for (int i = 0; i < 9; ++i) c[i] = t[i];
}

// c = a b^dag
template <typename R>
__device__ __forceinline__ void m3_mul_nd(const cpx<R>* a, const cpx<R>* b, cpx<R>* c) {
    cpx<R> t[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cpx<R> s = {(R)0, (R)0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(s, a[i * 3 + k], conj(b[j * 3 + k]));
            t[i * 3 + j] = s;
        }
#pragma unroll
    for (int i = 0; i < 9; ++i) c[i] = t[i];
}

// c = a^dag b
template <typename R>
__device__ __forceinline__ void m3_mul_dn(const cpx<R>* a, const cpx<R>* b, cpx<R>* c) {
    cpx<R> t[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cpx<R> s = {(R)0, (R)0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac_conj(s, a[k * 3 + i], b[k * 3 + j]);
            t[i * 3 + j] = s;
        }
#pragma unroll
    for (int i = 0; i < 9; ++i) c[i] = t[i];
}

template <typename R>
__device__ __forceinline__ void m3_dag(const cpx<R>* a, cpx<R>* c) {
    cpx<R> t[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) t[i * 3 + j] = conj(a[j * 3 + i]);
#pragma unroll
    for (int i = 0; i < 9; ++i) c[i] = t[i];
}

}  // namespace cs
