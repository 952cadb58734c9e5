// Internal definitions shared by the HIP sources of the cloversap library:
// geometry of the 4^4 block layout, storage formats, complex helpers and the
// host-side launch interface between translation units.
//
// Internal layout (private to the library).  Sites are grouped into 4^4
// blocks; block b = bx + NBx*(by + NBy*(bz + NBz*bt)), local site
// l = lx + 4*(ly + 4*(lz + 4*lt)).  Within a block every field is stored
// component-major ("structure of arrays"), so lane l of a 256-thread
// workgroup reads word l of each component row: all loads are unit-stride.
//
//   spinor F64  double2 [nblk][12][256]            complex component c = 3*spin + colour
//   spinor F32  float4  [nblk][6][256]             float4 k = components (2k, 2k+1)
//   spinor F16  uint4   [nblk][3][256] + float [nblk][256]
//               (8 halves = 4 complex per uint4; the float is the per-site scale,
//                the largest |re|, |im| of the site's 24 reals)
//   spinor BF16 as F16 with bfloat16 halves
//   links  F64  double2 [nblk][4][6][256]          rows 0 and 1 of U_mu(x), row-major
//   links  F32  float4  [nblk][4][3][256]
//   links  F16/BF16 uint2 [nblk][4][3][256]        2 complex per uint2
//   clover F64  double2 [nblk][36][256]            72 reals: for each chirality h,
//   clover F32  float4  [nblk][18][256]            6 diagonal reals of 1+T_h, then the
//                                                  15 upper entries (i<j, row-major)
//                                                  as (re, im)
// Multi-RHS fields are nrhs single fields one after the other.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>
#include <string>

namespace cs {

constexpr int BLOCK_SITES = 256;  // one 4^4 block = one workgroup

// Tuning knobs (compile-time; the defaults are the measured best on MI355X).
// Minimum waves per SIMD requested from the register allocator for the
// operator and smoother kernels (0 = compiler default); XCD-aware ordering of
// workgroups; non-temporal loads of the fields that are read exactly once
// (links, clover) and non-temporal stores of FP32 spinor fields, which keeps
// the caches for the face neighbours that are read twice; the operator's
// hopping sum as a rolled loop (bounded registers, 4 waves per SIMD) instead
// of fully unrolled; a raised wave priority during the loads of a SAP block
// visit.
#ifndef CS_DSLASH_WAVES
#define CS_DSLASH_WAVES 0
#endif
#ifndef CS_SAP_WAVES
#define CS_SAP_WAVES 0
#endif
#ifndef CS_XCD_REMAP
#define CS_XCD_REMAP 1
#endif
#ifndef CS_NT_LOADS
#define CS_NT_LOADS 1
#endif
#ifndef CS_NT_STORES
#define CS_NT_STORES 1
#endif
#ifndef CS_DSLASH_ROLLED
#define CS_DSLASH_ROLLED 1
#endif
// Float-arithmetic operator: 0 = every neighbour read through the caches,
// 1 = the block's spinor staged in LDS, 2 = its spinor and links staged.
#ifndef CS_DSLASH_STAGED
#define CS_DSLASH_STAGED 1
#endif
#ifndef CS_BLOCK_ORDER_TZ
#define CS_BLOCK_ORDER_TZ 2
#endif
#ifndef CS_SAP_PRIO
#define CS_SAP_PRIO 1
#endif
#ifndef CS_SAP_LDS_RESIDUAL
#define CS_SAP_LDS_RESIDUAL 1
#endif
#if CS_DSLASH_WAVES > 0
#define CS_DSLASH_BOUNDS __launch_bounds__(256, CS_DSLASH_WAVES)
#else
#define CS_DSLASH_BOUNDS __launch_bounds__(256)
#endif
#if CS_SAP_WAVES > 0
#define CS_SAP_BOUNDS __launch_bounds__(256, CS_SAP_WAVES)
#else
#define CS_SAP_BOUNDS __launch_bounds__(256)
#endif

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with its own L2.  Remapping workgroup i to item (i mod 8) * (n / 8) + i / 8
// gives every XCD one contiguous range of blocks, so blocks that share faces
// mostly run on the same XCD and meet in the same L2.
__host__ __device__ __forceinline__ int xcd_remap(int i, int n) {
#if CS_XCD_REMAP
    constexpr int NX = 8;
    if (n % NX != 0) return i;
    return (i % NX) * (n / NX) + i / NX;
#else
    (void)n;
    return i;
#endif
}

// Load of data that is used once per kernel (kept out of the caches' reuse
// set when CS_NT_LOADS is on).  FP64 data keeps ordinary loads: the FP64
// operator kernels (one and several right-hand sides per launch) must agree
// bit for bit, and the non-temporal form changed the code generated for one
// of them in the last bit of some sums.
template <typename T>
__device__ __forceinline__ T ld_once(const T* p) {
#if CS_NT_LOADS
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    typedef unsigned int v2u __attribute__((ext_vector_type(2)));
    if constexpr (std::is_same<T, double2>::value) {
        return *p;
    } else if constexpr (sizeof(T) == 16) {
        return __builtin_bit_cast(T, __builtin_nontemporal_load((const v4u*)p));
    } else if constexpr (sizeof(T) == 8) {
        return __builtin_bit_cast(T, __builtin_nontemporal_load((const v2u*)p));
    } else {
        return *p;
    }
#else
    return *p;
#endif
}

// Store of data that this kernel does not read again (streamed past the
// caches' reuse set when CS_NT_STORES is on).
template <typename T>
__device__ __forceinline__ void st_once(T* p, const T& v) {
#if CS_NT_STORES
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    if constexpr (sizeof(T) == 16) {
        __builtin_nontemporal_store(__builtin_bit_cast(v4u, v), (v4u*)p);
    } else {
        *p = v;
    }
#else
    *p = v;
#endif
}

enum Prec { P_F64 = 0, P_F32 = 1, P_F16 = 2, P_BF16 = 3 };

// ------------------------------------------------------------------ geometry

struct Geom {
    int L[4];      // lattice extents
    int NB[4];     // blocks per direction
    int nblk;      // number of blocks
    long long V;   // number of sites
    int antiperiodic_t;  // 1: fermion fields antiperiodic in time (the hops
                         // that cross the time boundary change sign)
};

// Per-thread block coordinates and block-index strides.
struct BlockPos {
    int blk;
    int bc[4];
    int stride[4];
};

__device__ __forceinline__ BlockPos block_pos(const Geom& g, int blk) {
    BlockPos p;
    p.blk = blk;
    int r = blk;
    p.bc[0] = r % g.NB[0]; r /= g.NB[0];
    p.bc[1] = r % g.NB[1]; r /= g.NB[1];
    p.bc[2] = r % g.NB[2];
    p.bc[3] = r / g.NB[2];
    p.stride[0] = 1;
    p.stride[1] = g.NB[0];
    p.stride[2] = g.NB[0] * g.NB[1];
    p.stride[3] = g.NB[0] * g.NB[1] * g.NB[2];
    return p;
}

// Neighbour of local site l in direction mu (dir = +1 or -1): returns the
// neighbour's block and writes its local index.  *inside = 1 when the
// neighbour lies in the same block.
__device__ __forceinline__ int neighbour(const Geom& g, const BlockPos& p, int l, int mu, int dir,
                                         int* nl, bool* inside) {
    const int sh = 2 * mu;
    const int lc = (l >> sh) & 3;
    if (dir > 0) {
        if (lc < 3) { *nl = l + (1 << sh); *inside = true; return p.blk; }
        *nl = l - (3 << sh);
        *inside = false;
        return p.bc[mu] == g.NB[mu] - 1 ? p.blk - (g.NB[mu] - 1) * p.stride[mu] : p.blk + p.stride[mu];
    }
    if (lc > 0) { *nl = l - (1 << sh); *inside = true; return p.blk; }
    *nl = l + (3 << sh);
    *inside = false;
    return p.bc[mu] == 0 ? p.blk + (g.NB[mu] - 1) * p.stride[mu] : p.blk - p.stride[mu];
}

// True when the hop from block p in direction mu (dir = +1 or -1) to a site
// outside the block (inside = false) crosses the lattice boundary in time.
__device__ __forceinline__ bool wraps_time(const Geom& g, const BlockPos& p, int mu, int dir, bool inside) {
    return mu == 3 && !inside && (dir > 0 ? p.bc[3] == g.NB[3] - 1 : p.bc[3] == 0);
}

// Boundary condition in time on a neighbour spinor about to enter a hop:
// with antiperiodic fields, psi(x + L_t e_t) = -psi(x), so a hop that wraps
// around in time takes the negated spinor.  The branch is uniform over a
// wave (a wave holds one time slice of a block).
template <typename R>
__device__ __forceinline__ void time_boundary_phase(const Geom& g, bool wraps, R* psi, int n) {
    if (wraps && g.antiperiodic_t) {
#pragma unroll
        for (int k = 0; k < n; ++k) psi[k] = -psi[k];
    }
}

// The c-th block of colour `colour` (colour = sum of block coordinates mod 2),
// enumerated with bx fastest; requires NB[0] even.
__host__ __device__ __forceinline__ int colour_block(const Geom& g, int colour, int c) {
    const int half = g.NB[0] / 2;
    const int hx = c % half;
    int r = c / half;
    const int by = r % g.NB[1];
    r /= g.NB[1];
#if CS_BLOCK_ORDER_TZ
    const int bt = r % g.NB[3];
    const int bz = r / g.NB[3];
#else
    const int bz = r % g.NB[2];
    const int bt = r / g.NB[2];
#endif
    const int bx = 2 * hx + ((colour + by + bz + bt) & 1);
    return bx + g.NB[0] * (by + g.NB[1] * (bz + g.NB[2] * bt));
}

// Block visited by work item w of an operator launch (w after the XCD
// remapping).  CS_BLOCK_ORDER_TZ 1: x fastest, then y, then t, then z, so
// that every XCD holds whole t columns of blocks (a block's t neighbours are
// visited next to it; only z faces cross XCDs); 2: the same with the xy
// plane walked in 4 x 4 tiles of blocks, which brings the y neighbours
// closer in visiting order as well (the L2 of an XCD keeps the spinor lines
// of roughly the last twenty blocks).  0: the block index itself.
__host__ __device__ __forceinline__ int block_of_item(const Geom& g, int w) {
#if CS_BLOCK_ORDER_TZ
    int bx, by, r;
#if CS_BLOCK_ORDER_TZ == 2
    if ((g.NB[0] & 3) == 0 && (g.NB[1] & 3) == 0) {
        // 4 x 4 tiles of blocks in the xy plane, x fastest inside a tile
        const int nxy = g.NB[0] * g.NB[1];
        const int q = w % nxy, tile = q >> 4, in = q & 15;
        const int tx = g.NB[0] >> 2;
        bx = 4 * (tile % tx) + (in & 3);
        by = 4 * (tile / tx) + (in >> 2);
        r = w / nxy;
    } else
#endif
    {
        bx = w % g.NB[0];
        r = w / g.NB[0];
        by = r % g.NB[1];
        r /= g.NB[1];
    }
    const int bt = r % g.NB[3];
    const int bz = r / g.NB[3];
    return bx + g.NB[0] * (by + g.NB[1] * (bz + g.NB[2] * bt));
#else
    (void)g;
    return w;
#endif
}

// Internal (blk, l) of the site with global coordinates c (already wrapped).
__device__ __forceinline__ void site_to_internal(const Geom& g, const int* c, int* blk, int* l) {
    *blk = (c[0] >> 2) + g.NB[0] * ((c[1] >> 2) + g.NB[1] * ((c[2] >> 2) + g.NB[2] * (c[3] >> 2)));
    *l = (c[0] & 3) + 4 * ((c[1] & 3) + 4 * ((c[2] & 3) + 4 * (c[3] & 3)));
}

// Global coordinates of (blk, l).
__device__ __forceinline__ void internal_coords(const Geom& g, int blk, int l, int* c) {
    int r = blk;
    const int bx = r % g.NB[0]; r /= g.NB[0];
    const int by = r % g.NB[1]; r /= g.NB[1];
    const int bz = r % g.NB[2];
    const int bt = r / g.NB[2];
    c[0] = bx * 4 + (l & 3);
    c[1] = by * 4 + ((l >> 2) & 3);
    c[2] = bz * 4 + ((l >> 4) & 3);
    c[3] = bt * 4 + (l >> 6);
}

// Canonical site index of (blk, l).
__device__ __forceinline__ long long canonical_site(const Geom& g, int blk, int l) {
    const BlockPos p = block_pos(g, blk);
    const int x = p.bc[0] * 4 + (l & 3);
    const int y = p.bc[1] * 4 + ((l >> 2) & 3);
    const int z = p.bc[2] * 4 + ((l >> 4) & 3);
    const int t = p.bc[3] * 4 + (l >> 6);
    return x + (long long)g.L[0] * (y + (long long)g.L[1] * (z + (long long)g.L[2] * t));
}

// ------------------------------------------------------------ storage sizes

inline size_t spinor_bytes_per_site(int prec) {
    switch (prec) {
    case P_F64: return 192;
    case P_F32: return 96;
    case P_F16:
    case P_BF16: return 52;
    default: return 0;
    }
}
inline size_t link_bytes_per_site(int prec) {  // four compressed links
    switch (prec) {
    case P_F64: return 384;
    case P_F32: return 192;
    case P_F16:
    case P_BF16: return 96;
    default: return 0;
    }
}
inline size_t clover_bytes_per_site(int prec) { return prec == P_F64 ? 576 : 288; }

// ------------------------------------------------------------ complex numbers

template <typename R>
struct cpx {
    R re, im;
};

// A complex value held in LDS, aligned to its full size: a wave's accesses
// are then single 8- or 16-byte LDS operations over consecutive addresses
// rather than two 4- or 8-byte halves at twice the stride, which map two
// lanes onto one bank.
template <typename R>
struct alignas(2 * sizeof(R)) lds_cpx {
    R re, im;
    __device__ __forceinline__ void set(const cpx<R>& v) {
        re = v.re;
        im = v.im;
    }
    __device__ __forceinline__ cpx<R> get() const { return {re, im}; }
};

template <typename R>
__device__ __forceinline__ cpx<R> cmake(R a, R b) { return cpx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> operator*(cpx<R> a, cpx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cpx<R> operator*(R s, cpx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> conj(cpx<R> a) { return {a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> mul_i(cpx<R> a) { return {-a.im, a.re}; }   // i a
template <typename R>
__device__ __forceinline__ cpx<R> mul_mi(cpx<R> a) { return {a.im, -a.re}; }  // -i a
// a += b * c
template <typename R>
__device__ __forceinline__ void cmac(cpx<R>& a, cpx<R> b, cpx<R> c) {
    a.re = fma(b.re, c.re, a.re);
    a.re = fma(-b.im, c.im, a.re);
    a.im = fma(b.re, c.im, a.im);
    a.im = fma(b.im, c.re, a.im);
}
// a += conj(b) * c
template <typename R>
__device__ __forceinline__ void cmac_conj(cpx<R>& a, cpx<R> b, cpx<R> c) {
    a.re = fma(b.re, c.re, a.re);
    a.re = fma(b.im, c.im, a.re);
    a.im = fma(b.re, c.im, a.im);
    a.im = fma(-b.im, c.re, a.im);
}

// ------------------------------------------------------------- host launch API

struct Profiler;

// Launch bookkeeping shared by all translation units: records HIP events
// around a launch when profiling is on.
void prof_begin(const char* family, hipStream_t s);
void prof_end(const char* family, hipStream_t s);

struct ProfScope {
    const char* fam;
    hipStream_t s;
    ProfScope(const char* f, hipStream_t st) : fam(f), s(st) { prof_begin(fam, s); }
    ~ProfScope() { prof_end(fam, s); }
};

// setup.hip
hipError_t launch_import_links(const Geom& g, const void* U_canonical, void* l64, void* l32,
                               void* l16, void* lbf16, hipStream_t s);
hipError_t launch_clover_build(const Geom& g, const void* links64, double kappa, double csw,
                               void* c64, void* c32, hipStream_t s);
// canonical [V][12][12]: T (inverse false) or the packed matrix itself (true)
hipError_t launch_clover_export(const Geom& g, const void* c64, void* dst, bool inverse, hipStream_t s);
// (1 + T)^-1 per site, packed like the clover term, FP64 and FP32
hipError_t launch_clover_invert(const Geom& g, const void* c64, void* ci64, void* ci32, hipStream_t s);
hipError_t launch_field_import(const Geom& g, int prec, void* dst, const void* src, int nrhs,
                               hipStream_t s);
hipError_t launch_field_export(const Geom& g, int prec, void* dst, const void* src, int nrhs,
                               hipStream_t s);

// dslash.hip: out = D in (dagger: gamma5 D gamma5).  in_prec / out_prec are
// spinor storage precisions; link and clover precision follow the arithmetic
// (F64 arithmetic when in_prec == P_F64, else F32 arithmetic with links of
// precision link_prec and F32 clover).  With sub != nullptr the kernel writes
// out = sub - D in (sub has out_prec).
struct OpData {
    Geom g;
    const void* links[4];   // indexed by Prec
    const void* clover64;
    const void* clover32;
    const void* cinv64;     // (1 + T)^-1, same packing
    const void* cinv32;
    double kappa;
};
hipError_t launch_dslash(const OpData& op, int in_prec, int out_prec, int link_prec, bool dagger,
                         void* out, const void* in, const void* sub, int nrhs, hipStream_t s);

// Launch configuration of the multi-right-hand-side kernels: right-hand
// sides per workgroup (links and clover are loaded once per tile), when
// positive the number of workgroups of a persistent launch, and the lanes per
// site of the low-precision SAP kernel (1 or 2; 0: chosen from the lattice).
struct LaunchCfg {
    int rhs_tile = 1;
    int persistent_wgs = 0;
    int lanes_per_site = 0;
};

// dslash.hip, multi-right-hand-side form (input, output and links of one
// precision; no subtraction).
hipError_t launch_dslash_tiled(const OpData& op, int prec, bool dagger, void* out, const void* in, int nrhs,
                               const LaunchCfg& cfg, hipStream_t s);

// The same batched launch from FP32 input (FP32 links) into FP16 or BF16
// output with a per-site scale (the 16-bit Krylov basis of the outer solver).
hipError_t launch_dslash_tiled_to16(const OpData& op, int out_prec, void* out, const void* in, int nrhs,
                                    const LaunchCfg& cfg, hipStream_t s);

// sap.hip: one half-sweep over the blocks of one colour.  mode 0: general;
// 1: x is zero everywhere (r = b); 2: x is zero on the blocks of this colour.
// Block solver: BLOCK_MR, n_block MR steps on D_BB; BLOCK_JACOBI, n_block
// Jacobi steps on A_BB = (C^-1 D)_BB; BLOCK_EO, n_block MR steps on the
// even-site Schur complement of D_BB (one lane per site only).
enum { BLOCK_MR = 0, BLOCK_JACOBI = 1, BLOCK_EO = 2 };
hipError_t launch_sap_halfsweep(const OpData& op, int prec, int colour, int n_block, int mode,
                                void* x, const void* b, int nrhs, const LaunchCfg& cfg, hipStream_t s,
                                int block_solver = BLOCK_MR);
// sap_pair.hip: the same half-sweep with two lanes per site (FP32, FP16, BF16).
hipError_t launch_sap_pair(const OpData& op, int prec, int colour, int n_block, int mode, void* x,
                           const void* b, int nrhs, const LaunchCfg& cfg, hipStream_t s, int block_solver);

// force.hip: g_{mu,a}(x) = dL/dw of L with dL = -Re(y^dag dD x); either output
// may be null.  Hbuf holds 864 bytes per site (insertion matrices).
hipError_t launch_force(const Geom& g, const void* links64, double kappa, double csw, const void* x,
                        const void* y, void* Hbuf, double* glie, void* gradU, hipStream_t s);
// Fixed workspace of the allocation-free force (force.hip): 128 MiB per
// device, i.e. the insertion matrices of up to 155,344 sites (a 16^3 x 32
// lattice).  force_scratch_address gives its device address on the current
// device (looked up once per device).
constexpr size_t FORCE_SCRATCH_BYTES = size_t(128) << 20;
constexpr int FORCE_SCRATCH_MAX_DEVICES = 64;
hipError_t force_scratch_address(void** out);

// blas.hip
struct BlasWork;  // defined in blas.hip

}  // namespace cs
