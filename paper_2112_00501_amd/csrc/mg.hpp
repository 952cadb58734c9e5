// Two-level multigrid preconditioner (paper Section 3): kernels in mg.hip,
// setup and application drivers in mg.cpp.
#pragma once

#include <vector>

#include "cs_internal.hpp"

namespace cs {

constexpr int MG_MAX_NV = 32;  // nc = 2 nv coarse values per aggregate fit one wave

constexpr int MG_ELEM_WG = 1024;  // workgroups of the elementwise coarse kernels (at most)
constexpr int MG_CHUNK = 8;       // coarse iterations between two host reads of the stop flag

// Scalars of the coarse BiCGStab, kept on the device.  Once a stop flag is
// set every later kernel of the solve returns at once, so a fixed number of
// iterations can be launched (or captured) without host round trips.  Slots
// [2] are indexed by iteration parity.
struct CbScalars {
    double2 rho[2], beta[2], alpha, omega;
    double rr, stop2;  // |r|^2 and the stopping threshold tol^2 |r_0|^2
    int stopped[2], brk[2];
};

struct CbVecs {
    float2 *x, *r, *rh, *p[2], *v[2], *s, *t;
    float2* tau;  // the +mu terms of a product, [aggregate][mu][nc]
};

// Workgroup partial sums of the elementwise kernels (at most MG_ELEM_WG
// workgroups each): A of <rh, r>, |r|^2, B of <rh, v>, C of <t, s>, |t|^2.
struct CbPartials {
    double2 *A, *B, *C;
};

struct MgParams {
    int nv, n_cy_setup, n_mr, n_adapt, n_coarse, n_cy_post;
    double tol_coarse;
    int coarse_half;    // the coarse solve reads an FP16 copy of D_c
    int transfer_half;  // restriction and prolongation read an FP16 copy of P
};

// The prolongator as restriction and prolongation read it.
struct Transfer {
    const void* P;
    int prec;  // P_F32 or P_F16
};

// The coarse matrices as the coarse solver reads them.
struct CoarseMat {
    const void* m;
    bool half;
};

// Device state of one hierarchy.  P: nv FP32 fields (field i holds
// p_{a,chi,i}); V: the nv null vectors before orthonormalisation; Dc:
// float2[nblk][9][nc][nc]; coarse vectors float2[nblk][nc].
struct MgData {
    Geom g{};
    MgParams p{};
    void* P = nullptr;
    void* P16 = nullptr;  // FP16 copy (transfer_half)
    void* V = nullptr;
    void* tmp = nullptr;  // one FP32 field
    float2* Dc = nullptr;
    void* Dc16 = nullptr;  // FP16 copy (coarse_half)
    float2* rc = nullptr;
    CbVecs cv{};
    CbScalars* sc = nullptr;
    CbPartials pa{};
    LaunchCfg sap_cfg{};
    int* host_flag = nullptr;  // pinned copy of a stop flag
    unsigned long long id = 0; // distinct for every allocation (keys of captured graphs)
    // captured graphs of the coarse phase, one set per input field `r`:
    // restriction of r, start and the first chunk; then chunk j covers
    // iterations [(j + 1) MG_CHUNK, ...)
    struct Graphs {
        const void* r = nullptr;
        hipGraphExec_t first = nullptr;
        std::vector<hipGraphExec_t> chunk;
    };
    mutable std::vector<Graphs> gr;
    void drop_graphs() const;

    int nc() const { return 2 * p.nv; }
    size_t field_bytes() const;
    size_t coarse_bytes() const { return (size_t)g.nblk * nc() * sizeof(float2); }
    size_t dc_bytes() const { return (size_t)g.nblk * 9 * nc() * nc() * sizeof(float2); }
    CoarseMat coarse() const { return p.coarse_half ? CoarseMat{Dc16, true} : CoarseMat{Dc, false}; }
    Transfer transfer() const { return p.transfer_half ? Transfer{P16, P_F16} : Transfer{P, P_F32}; }
    hipError_t alloc(const Geom& g, const MgParams& p);
    void release();
    ~MgData() { release(); }
};

// mg.hip
hipError_t mg_orthonormalize(const Geom& g, void* P, int nv, hipStream_t s);
hipError_t mg_assemble(const OpData& op, const void* P, int nv, float2* Dc, hipStream_t s);
hipError_t mg_restrict(const Geom& g, Transfer T, int nv, const void* r, float2* rc, hipStream_t s);
hipError_t mg_prolong(const Geom& g, Transfer T, int nv, const float2* ec, void* z, hipStream_t s);
// the same for nr consecutive FP32 fields and nr consecutive coarse vectors
// (the null vectors of an adaptive setup pass), every field with the sums of
// the one-field launches
hipError_t mg_restrict_many(const Geom& g, Transfer T, int nv, const void* r, int nr, float2* rc,
                            hipStream_t s);
hipError_t mg_prolong_many(const Geom& g, Transfer T, int nv, const float2* ec, int nr, void* z, hipStream_t s);
// Dc16 = FP16 copy of the n complex entries of Dc
hipError_t mg_coarse_half(const float2* Dc, void* Dc16, size_t n, hipStream_t s);
// y = D_c x
hipError_t mg_coarse_apply(const Geom& g, CoarseMat M, int nc, const float2* x, float2* y, float2* tau,
                           hipStream_t s);
// cv.x = BiCGStab(D_c, rc) from zero: at most max_iter iterations, fewer once
// |r| <= tol |rc| or on a breakdown (all decided on the device)
hipError_t mg_coarse_bicgstab(const Geom& g, CoarseMat M, int nc, const float2* rc, const CbVecs& cv,
                              CbScalars* sc, const CbPartials& pa, int max_iter, double tol, hipStream_t s);
// The same solve in pieces: the start with the stop test of iteration 0, then
// iterations [it0, it1), each ending with the stop test of the next one.
hipError_t mg_coarse_begin(const Geom& g, int nc, const float2* rc, const CbVecs& cv, CbScalars* sc,
                           const CbPartials& pa, double tol, hipStream_t s);
hipError_t mg_coarse_iters(const Geom& g, CoarseMat M, int nc, const CbVecs& cv, CbScalars* sc,
                           const CbPartials& pa, int it0, int it1, hipStream_t s);

// mg.cpp
// Null vectors from the nv FP32 fields etas, P and D_c, n_adapt adaptive passes.
hipError_t mg_setup(const OpData& op, MgData& m, const void* etas, hipStream_t s);
// z = M_MG r (FP32 fields, z != r): coarse correction, then n_cy_post SAP cycles.
hipError_t mg_apply(const OpData& op, const MgData& m, void* z, const void* r, hipStream_t s);
// The first part of M_MG r: r_c = P^dag r and the coarse solve into m.cv.x,
// run in chunks of MG_CHUNK iterations with a host read of the stop flag
// after each (synchronises s); with use_graph the pieces are captured once
// (s must then be a non-null stream) and replayed.
hipError_t mg_coarse_phase(const MgData& m, const void* r, hipStream_t s, bool use_graph);
// The second part: z = P m.cv.x, then n_cy_post SAP cycles on D z = r.
hipError_t mg_finish(const OpData& op, const MgData& m, void* z, const void* r, hipStream_t s);

}  // namespace cs
