// Measurement probe for one design decision: whether the batched product
// of a link with the half spinors of several right-hand sides (the core of
// every hop when a tile of right-hand sides shares the block's links) is
// dense enough to pay on the matrix cores.  Per site, V = U H with U a
// complex 3x3 link and H a complex 3 x 16 matrix (two spin components of a
// half spinor for 8 right-hand sides); the product is chained `reps` times
// in registers (H <- U H) so that arithmetic, not memory, sets the time.
//   VALU form: one lane per site, FP32 complex multiply-adds.
//   MFMA form: the real 6x6 form of U, [[Re U, -Im U], [Im U, Re U]], of two
//     sites as a block-diagonal 16x16 operand (rows and columns 12-15 zero),
//     times the stacked real 12x16 form of their H, one
//     v_mfma_f32_16x16x16_bf16 per site pair and chain step: bfloat16
//     inputs, FP32 accumulation; the FP32 result is rounded to bfloat16 to
//     become the next step's input (it lands in the lane and register order
//     the next B operand needs).
// Layout: U float[nsites][9][2] (row-major, re/im), H and V
// float[nsites][16][3][2] (column, colour, re/im).
#include <hip/hip_runtime.h>

#include "cs_internal.hpp"
#include "probe.hpp"

namespace cs {

namespace {

constexpr int PROBE_COLS = 16;

__global__ __launch_bounds__(256) void k_probe_valu(long long nsites, int reps, const float* __restrict__ U,
                                                    const float* __restrict__ H, float* __restrict__ V) {
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    if (s >= nsites) return;
    float u[18], h[PROBE_COLS][6];
#pragma unroll
    for (int k = 0; k < 18; ++k) u[k] = U[s * 18 + k];
#pragma unroll
    for (int c = 0; c < PROBE_COLS; ++c)
#pragma unroll
        for (int k = 0; k < 6; ++k) h[c][k] = H[(s * PROBE_COLS + c) * 6 + k];
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int c = 0; c < PROBE_COLS; ++c) {
            float v[6];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                float re = 0.f, im = 0.f;
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const float ur = u[2 * (3 * a + b)], ui = u[2 * (3 * a + b) + 1];
                    re = fmaf(ur, h[c][2 * b], re);
                    re = fmaf(-ui, h[c][2 * b + 1], re);
                    im = fmaf(ur, h[c][2 * b + 1], im);
                    im = fmaf(ui, h[c][2 * b], im);
                }
                v[2 * a] = re;
                v[2 * a + 1] = im;
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) h[c][k] = v[k];
        }
    }
#pragma unroll
    for (int c = 0; c < PROBE_COLS; ++c)
#pragma unroll
        for (int k = 0; k < 6; ++k) V[(s * PROBE_COLS + c) * 6 + k] = h[c][k];
}

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) { return __builtin_bit_cast(short, (__bf16)f); }

// Entry (i, k) of the real 6x6 form of link u (float[9][2]).
__device__ __forceinline__ float real_form(const float* __restrict__ u, int i, int k) {
    const int r = i % 3, c = k % 3;
    const float re = u[2 * (3 * r + c)], im = u[2 * (3 * r + c) + 1];
    if (i < 3) return k < 3 ? re : -im;
    return k < 3 ? im : re;
}

// One wave per PROBE_PAIRS pairs of sites (independent chains, so that the
// matrix core is not left waiting on one chain's dependency); for each pair
// lane l holds, for the 16x16x16 bf16 MFMA, A[i][k] and B[k][j] with
// i = j = l % 16 and k = 4 (l / 16) + e, and receives D[i][j] with
// j = l % 16 and i = 4 (l / 16) + e (e = 0..3).
constexpr int PROBE_PAIRS = 4;

__global__ __launch_bounds__(256) void k_probe_mfma(long long nsites, int reps, const float* __restrict__ U,
                                                    const float* __restrict__ H, float* __restrict__ V) {
    const long long wave = ((long long)blockIdx.x * 256 + threadIdx.x) / 64;
    const long long pair0 = wave * PROBE_PAIRS;
    if (2 * (pair0 + PROBE_PAIRS) > nsites) return;  // uniform over the wave; nsites is a multiple of 8
    const int l = threadIdx.x & 63, col = l % 16, kq = l / 16;
    v4s a[PROBE_PAIRS], b[PROBE_PAIRS];
    v4f d[PROBE_PAIRS];
#pragma unroll
    for (int q = 0; q < PROBE_PAIRS; ++q) {
        const long long pair = pair0 + q;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * kq + e, i = col;  // A row i = lane % 16, B column j = lane % 16
            float av = 0.f;
            if (i < 12 && k < 12 && (i < 6) == (k < 6)) {
                const long long s = 2 * pair + (i < 6 ? 0 : 1);
                av = real_form(U + s * 18, i % 6, k % 6);
            }
            a[q][e] = to_bf16(av);
            float bv = 0.f;
            if (k < 12) {
                const long long s = 2 * pair + (k < 6 ? 0 : 1);
                const int kk = k % 6;  // 0-2 real parts, 3-5 imaginary parts of the colour components
                bv = H[(s * PROBE_COLS + col) * 6 + 2 * (kk % 3) + (kk < 3 ? 0 : 1)];
            }
            b[q][e] = to_bf16(bv);
        }
        d[q] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int q = 0; q < PROBE_PAIRS; ++q) {
            const v4f z = {0.f, 0.f, 0.f, 0.f};
            d[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[q], b[q], z, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < PROBE_PAIRS; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) b[q][e] = to_bf16(d[q][e]);
    }
#pragma unroll
    for (int q = 0; q < PROBE_PAIRS; ++q) {
        const long long pair = pair0 + q;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 4 * kq + e;
            if (i < 12) {
                const long long s = 2 * pair + (i < 6 ? 0 : 1);
                const int ii = i % 6;
                V[(s * PROBE_COLS + col) * 6 + 2 * (ii % 3) + (ii < 3 ? 0 : 1)] = d[q][e];
            }
        }
    }
}

}  // namespace

hipError_t launch_probe_link_product(int kind, long long nsites, int reps, const float* U, const float* H, float* V,
                                     hipStream_t s) {
    ProfScope ps("probe", s);
    if (kind == 0) {
        const long long wgs = (nsites + 255) / 256;
        hipLaunchKernelGGL(k_probe_valu, dim3((unsigned)wgs), dim3(256), 0, s, nsites, reps, U, H, V);
    } else {
        const long long wgs = (nsites / 2 / PROBE_PAIRS + 3) / 4;  // four waves per 256-lane workgroup
        hipLaunchKernelGGL(k_probe_mfma, dim3((unsigned)wgs), dim3(256), 0, s, nsites, reps, U, H, V);
    }
    return hipGetLastError();
}

}  // namespace cs
