// C ABI of the cloversap library (include/cloversap.h): handle management,
// argument validation, error reporting and launch profiling.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "../../include/cloversap.h"
#include "blas.hpp"
#include "bicgstab.hpp"
#include "gcr.hpp"
#include "mg.hpp"
#include "probe.hpp"

struct cs_lattice_s {
    cs::Geom g;
};

struct cs_gauge_s {
    cs::Geom g;
    void* links[4] = {nullptr, nullptr, nullptr, nullptr};
};

struct cs_mg_s {
    cs_gauge_s* gauge = nullptr;
    struct cs_clover_s* clover = nullptr;
    cs::MgData data;
};

struct cs_clover_s {
    cs_gauge_s* gauge = nullptr;
    double kappa = 0, csw = 0;
    void* c64 = nullptr;
    void* c32 = nullptr;
    void* ci64 = nullptr;   // (1 + T)^-1
    void* ci32 = nullptr;
    std::unique_ptr<cs::GcrWork> work;
    std::vector<std::unique_ptr<cs::GcrWork>> group_work;  // one per concurrent group of right-hand sides
    std::unique_ptr<cs::BicgWork> bicg;
    void* force_H = nullptr;   // insertion matrices of the force, 864 B/site
    void* dag_tmp = nullptr;   // FP64 fields for the adjoint solve
    int dag_tmp_nrhs = 0;
    // autotuned multi-right-hand-side launch shapes, keyed by (precision, nrhs)
    std::map<std::pair<int, int>, std::pair<cs::LaunchCfg, cs::LaunchCfg>> tuned;
};

namespace {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int ok() {
    g_last_error.clear();
    return CS_OK;
}

#define CS_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) return fail(CS_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

bool valid_prec(int p) { return p >= CS_F64 && p <= CS_BF16; }

cs::OpData make_op(const cs_gauge_s* g, const cs_clover_s* c) {
    cs::OpData op;
    op.g = g->g;
    for (int i = 0; i < 4; ++i) op.links[i] = g->links[i];
    op.clover64 = c->c64;
    op.clover32 = c->c32;
    op.cinv64 = c->ci64;
    op.cinv32 = c->ci32;
    op.kappa = c->kappa;
    return op;
}

int check_op(cs_gauge g, cs_clover c) {
    if (!g || !c) return fail(CS_ERR_NULL, "gauge or clover handle is NULL");
    if (c->gauge != g) return fail(CS_ERR_INVALID, "clover handle was built from a different gauge handle");
    return CS_OK;
}

bool sap_geometry_ok(const cs::Geom& g) {
    for (int m = 0; m < 4; ++m)
        if (g.NB[m] % 2 != 0) return false;
    return true;
}

// ---------------------------------------------------------------- profiler

struct ProfRec {
    std::string fam;
    hipStream_t s;  // records of concurrent solves on other streams stay apart
    hipEvent_t a, b;
    bool closed;
};
std::mutex g_pm;
bool g_prof_on = false;
std::vector<ProfRec> g_pending;
std::vector<hipEvent_t> g_event_pool;
std::map<std::string, std::pair<long long, double>> g_prof;

hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void drain_pending() {
    for (auto& r : g_pending) {
        if (r.closed && hipEventSynchronize(r.b) == hipSuccess) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                auto& slot = g_prof[r.fam];
                slot.first += 1;
                slot.second += ms;
            }
        }
        g_event_pool.push_back(r.a);
        g_event_pool.push_back(r.b);
    }
    g_pending.clear();
}

}  // namespace

namespace cs {

void prof_begin(const char* family, hipStream_t s) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_pm);
    ProfRec r{family, s, take_event(), take_event(), false};
    if (!r.a || !r.b) return;
    hipEventRecord(r.a, s);
    g_pending.push_back(r);
}

void prof_end(const char* family, hipStream_t s) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_pm);
    for (auto it = g_pending.rbegin(); it != g_pending.rend(); ++it) {
        if (!it->closed && it->s == s && it->fam == family) {
            hipEventRecord(it->b, s);
            it->closed = true;
            break;
        }
    }
}

}  // namespace cs

extern "C" {

const char* cs_last_error(void) { return g_last_error.c_str(); }

const char* cs_strerror(int status) {
    switch (status) {
    case CS_OK: return "ok";
    case CS_ERR_INVALID: return "invalid argument";
    case CS_ERR_GEOMETRY: return "unsupported lattice geometry";
    case CS_ERR_NULL: return "null pointer or handle";
    case CS_ERR_PRECISION: return "unsupported precision";
    case CS_ERR_HIP: return "HIP runtime error";
    case CS_ERR_ALLOC: return "device allocation failed";
    case CS_NOT_CONVERGED: return "not converged within max_iter";
    case CS_BREAKDOWN: return "solver breakdown";
    case CS_NONFINITE: return "non-finite residual";
    default: return "unknown status";
    }
}

int cs_lattice_create(const int dims[4], const int block[4], int flags, cs_lattice* out) {
    if (!dims || !block || !out) return fail(CS_ERR_NULL, "dims, block and out must be non-NULL");
    if (flags & ~CS_ANTIPERIODIC_T) return fail(CS_ERR_INVALID, "unknown lattice flags 0x%x", (unsigned)flags);
    cs::Geom g{};
    g.antiperiodic_t = (flags & CS_ANTIPERIODIC_T) ? 1 : 0;
    long long V = 1;
    for (int m = 0; m < 4; ++m) {
        if (block[m] != 4)
            return fail(CS_ERR_GEOMETRY, "block must be 4x4x4x4 (got %d in direction %d)", block[m], m);
        if (dims[m] <= 0 || dims[m] % 4 != 0)
            return fail(CS_ERR_GEOMETRY, "extent %d in direction %d is not a positive multiple of 4", dims[m], m);
        g.L[m] = dims[m];
        g.NB[m] = dims[m] / 4;
        V *= dims[m];
    }
    if (V / cs::BLOCK_SITES > (1LL << 30)) return fail(CS_ERR_GEOMETRY, "lattice too large");
    g.V = V;
    g.nblk = (int)(V / cs::BLOCK_SITES);
    *out = new cs_lattice_s{g};
    return ok();
}

int cs_lattice_destroy(cs_lattice lat) {
    delete lat;
    return ok();
}

long long cs_lattice_volume(cs_lattice lat) { return lat ? lat->g.V : 0; }

size_t cs_field_bytes(cs_lattice lat, cs_prec prec, int nrhs) {
    if (!lat || !valid_prec(prec) || nrhs < 0) return 0;
    return cs::spinor_bytes_per_site(prec) * (size_t)lat->g.V * (size_t)nrhs;
}

int cs_field_import(cs_lattice lat, cs_prec prec, void* dst, const void* src, int nrhs, void* stream) {
    if (!lat || !dst || !src) return fail(CS_ERR_NULL, "lattice, dst and src must be non-NULL");
    if (!valid_prec(prec)) return fail(CS_ERR_PRECISION, "unknown precision %d", (int)prec);
    if (nrhs < 1 || nrhs > 65535) return fail(CS_ERR_INVALID, "nrhs must be in 1..65535");
    CS_HIP(cs::launch_field_import(lat->g, prec, dst, src, nrhs, (hipStream_t)stream));
    return ok();
}

int cs_field_export(cs_lattice lat, cs_prec prec, void* dst, const void* src, int nrhs, void* stream) {
    if (!lat || !dst || !src) return fail(CS_ERR_NULL, "lattice, dst and src must be non-NULL");
    if (!valid_prec(prec)) return fail(CS_ERR_PRECISION, "unknown precision %d", (int)prec);
    if (nrhs < 1 || nrhs > 65535) return fail(CS_ERR_INVALID, "nrhs must be in 1..65535");
    CS_HIP(cs::launch_field_export(lat->g, prec, dst, src, nrhs, (hipStream_t)stream));
    return ok();
}

int cs_gauge_create(cs_lattice lat, const void* U, void* stream, cs_gauge* out) {
    if (!lat || !U || !out) return fail(CS_ERR_NULL, "lattice, U and out must be non-NULL");
    auto* g = new cs_gauge_s;
    g->g = lat->g;
    for (int p = 0; p < 4; ++p) {
        if (hipMalloc(&g->links[p], cs::link_bytes_per_site(p) * g->g.V) != hipSuccess) {
            cs_gauge_destroy(g);
            return fail(CS_ERR_ALLOC, "could not allocate %zu bytes of links",
                        cs::link_bytes_per_site(p) * (size_t)g->g.V);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = cs::launch_import_links(g->g, U, g->links[0], g->links[1], g->links[2], g->links[3], s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        cs_gauge_destroy(g);
        return fail(CS_ERR_HIP, "link import: %s", hipGetErrorString(e));
    }
    *out = g;
    return ok();
}

int cs_gauge_destroy(cs_gauge g) {
    if (!g) return ok();
    for (int p = 0; p < 4; ++p)
        if (g->links[p]) hipFree(g->links[p]);
    delete g;
    return ok();
}

int cs_clover_create(cs_gauge g, double kappa, double csw, void* stream, cs_clover* out) {
    if (!g || !out) return fail(CS_ERR_NULL, "gauge and out must be non-NULL");
    if (!std::isfinite(kappa) || !std::isfinite(csw)) return fail(CS_ERR_INVALID, "kappa and c_sw must be finite");
    auto* c = new cs_clover_s;
    c->gauge = g;
    c->kappa = kappa;
    c->csw = csw;
    if (hipMalloc(&c->c64, cs::clover_bytes_per_site(cs::P_F64) * g->g.V) != hipSuccess ||
        hipMalloc(&c->c32, cs::clover_bytes_per_site(cs::P_F32) * g->g.V) != hipSuccess ||
        hipMalloc(&c->ci64, cs::clover_bytes_per_site(cs::P_F64) * g->g.V) != hipSuccess ||
        hipMalloc(&c->ci32, cs::clover_bytes_per_site(cs::P_F32) * g->g.V) != hipSuccess) {
        cs_clover_destroy(c);
        return fail(CS_ERR_ALLOC, "could not allocate the clover term");
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = cs::launch_clover_build(g->g, g->links[cs::P_F64], kappa, csw, c->c64, c->c32, s);
    if (e == hipSuccess) e = cs::launch_clover_invert(g->g, c->c64, c->ci64, c->ci32, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        cs_clover_destroy(c);
        return fail(CS_ERR_HIP, "clover build: %s", hipGetErrorString(e));
    }
    *out = c;
    return ok();
}

int cs_clover_destroy(cs_clover c) {
    if (!c) return ok();
    c->work.reset();
    c->group_work.clear();
    if (c->force_H) hipFree(c->force_H);
    if (c->dag_tmp) hipFree(c->dag_tmp);
    if (c->c64) hipFree(c->c64);
    if (c->c32) hipFree(c->c32);
    if (c->ci64) hipFree(c->ci64);
    if (c->ci32) hipFree(c->ci32);
    delete c;
    return ok();
}

int cs_clover_export(cs_clover c, void* dst, void* stream) {
    if (!c || !dst) return fail(CS_ERR_NULL, "clover and dst must be non-NULL");
    CS_HIP(cs::launch_clover_export(c->gauge->g, c->c64, dst, false, (hipStream_t)stream));
    return ok();
}

int cs_clover_inverse_export(cs_clover c, void* dst, void* stream) {
    if (!c || !dst) return fail(CS_ERR_NULL, "clover and dst must be non-NULL");
    CS_HIP(cs::launch_clover_export(c->gauge->g, c->ci64, dst, true, (hipStream_t)stream));
    return ok();
}

static bool overlap(const void* a, const void* b, size_t bytes) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + bytes && y < x + bytes;
}

static cs::LaunchCfg to_cfg(const cs_launch_config* c) {
    cs::LaunchCfg r;
    if (c) {
        r.rhs_tile = c->rhs_tile < 1 ? 1 : c->rhs_tile;
        r.persistent_wgs = c->persistent_wgs < 0 ? 0 : c->persistent_wgs;
        r.lanes_per_site = c->lanes_per_site == 1 || c->lanes_per_site == 2 ? c->lanes_per_site : 0;
    }
    return r;
}

static int apply(cs_gauge g, cs_clover c, cs_prec prec, void* out, const void* in, int nrhs,
                 const cs_launch_config* cfg, void* stream, bool dagger) {
    int st = check_op(g, c);
    if (st) return st;
    if (!out || !in) return fail(CS_ERR_NULL, "out and in must be non-NULL");
    if (!valid_prec(prec)) return fail(CS_ERR_PRECISION, "unknown precision %d", (int)prec);
    if (nrhs < 1 || nrhs > 65535) return fail(CS_ERR_INVALID, "nrhs must be in 1..65535");
    const size_t bytes = cs::spinor_bytes_per_site(prec) * (size_t)g->g.V * nrhs;
    if (overlap(in, out, bytes)) return fail(CS_ERR_INVALID, "out and in overlap");
    const cs::LaunchCfg lc = to_cfg(cfg);
    if (lc.rhs_tile > 1 || lc.persistent_wgs > 0)
        CS_HIP(cs::launch_dslash_tiled(make_op(g, c), prec, dagger, out, in, nrhs, lc, (hipStream_t)stream));
    else
        CS_HIP(cs::launch_dslash(make_op(g, c), prec, prec, prec, dagger, out, in, nullptr, nrhs, (hipStream_t)stream));
    return ok();
}

int cs_apply_D(cs_gauge g, cs_clover c, cs_prec prec, void* out, const void* in, int nrhs, void* stream) {
    return apply(g, c, prec, out, in, nrhs, nullptr, stream, false);
}

int cs_apply_Ddag(cs_gauge g, cs_clover c, cs_prec prec, void* out, const void* in, int nrhs, void* stream) {
    return apply(g, c, prec, out, in, nrhs, nullptr, stream, true);
}

int cs_apply_D_cfg(cs_gauge g, cs_clover c, cs_prec prec, void* out, const void* in, int nrhs,
                   const cs_launch_config* cfg, void* stream) {
    return apply(g, c, prec, out, in, nrhs, cfg, stream, false);
}

static int sap_common(cs_gauge g, cs_clover c, cs_prec prec, void* x, const void* b, int n_cy, int n_mr,
                      int x0_is_zero, int nrhs, const cs_launch_config* cfg, void* stream, int solver) {
    int st = check_op(g, c);
    if (st) return st;
    if (!x || !b) return fail(CS_ERR_NULL, "x and b must be non-NULL");
    if (!valid_prec(prec)) return fail(CS_ERR_PRECISION, "unknown precision %d", (int)prec);
    if (n_cy < 0 || n_mr < 0) return fail(CS_ERR_INVALID, "n_cy and n_mr must be >= 0");
    if (nrhs < 1 || nrhs > 65535) return fail(CS_ERR_INVALID, "nrhs must be in 1..65535");
    if (!sap_geometry_ok(g->g))
        return fail(CS_ERR_GEOMETRY, "the red/black block colouring needs an even number of blocks per direction");
    const size_t bytes = cs::spinor_bytes_per_site(prec) * (size_t)g->g.V * nrhs;
    if (overlap(b, x, bytes)) return fail(CS_ERR_INVALID, "x and b overlap");
    const cs::OpData op = make_op(g, c);
    const cs::LaunchCfg lc = to_cfg(cfg);
    hipStream_t s = (hipStream_t)stream;
    if (n_cy == 0 && x0_is_zero) {
        CS_HIP(hipMemsetAsync(x, 0, bytes, s));
        return ok();
    }
    for (int cy = 0; cy < n_cy; ++cy)
        for (int col = 0; col < 2; ++col) {
            const int mode = (x0_is_zero && cy == 0) ? (col == 0 ? 1 : 2) : 0;
            CS_HIP(cs::launch_sap_halfsweep(op, prec, col, n_mr, mode, x, b, nrhs, lc, s, solver));
        }
    return ok();
}

int cs_sap_smooth_cfg(cs_gauge g, cs_clover c, cs_prec prec, void* x, const void* b, int n_cy, int n_mr,
                      int x0_is_zero, int nrhs, const cs_launch_config* cfg, void* stream) {
    return sap_common(g, c, prec, x, b, n_cy, n_mr, x0_is_zero, nrhs, cfg, stream, cs::BLOCK_MR);
}

int cs_sap_smooth_eo(cs_gauge g, cs_clover c, cs_prec prec, void* x, const void* b, int n_cy, int n_mr,
                     int x0_is_zero, int nrhs, const cs_launch_config* cfg, void* stream) {
    return sap_common(g, c, prec, x, b, n_cy, n_mr, x0_is_zero, nrhs, cfg, stream, cs::BLOCK_EO);
}

int cs_sap_smooth_jacobi(cs_gauge g, cs_clover c, cs_prec prec, void* x, const void* b, int n_cy, int n_jac,
                         int x0_is_zero, int nrhs, const cs_launch_config* cfg, void* stream) {
    return sap_common(g, c, prec, x, b, n_cy, n_jac, x0_is_zero, nrhs, cfg, stream, cs::BLOCK_JACOBI);
}

int cs_sap_smooth(cs_gauge g, cs_clover c, cs_prec prec, void* x, const void* b, int n_cy, int n_mr,
                  int x0_is_zero, int nrhs, void* stream) {
    return cs_sap_smooth_cfg(g, c, prec, x, b, n_cy, n_mr, x0_is_zero, nrhs, nullptr, stream);
}

// Autotuner: time one SAP application (the four half-sweeps of n_cy = 2 from
// x = 0, n_mr = 4) and one operator application per candidate launch shape.
static int autotune(cs_gauge g, cs_clover c, int prec, int nrhs, hipStream_t s, cs::LaunchCfg* best_sap,
                    cs::LaunchCfg* best_d) {
    const auto key = std::make_pair(prec, nrhs);
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) {
        *best_sap = it->second.first;
        *best_d = it->second.second;
        return ok();
    }
    const cs::OpData op = make_op(g, c);
    const size_t bytes = cs::spinor_bytes_per_site(prec) * (size_t)g->g.V * nrhs;
    void *xb = nullptr, *bb = nullptr;
    if (hipMalloc(&xb, bytes) != hipSuccess || hipMalloc(&bb, bytes) != hipSuccess) {
        if (xb) hipFree(xb);
        return fail(CS_ERR_ALLOC, "autotune scratch (%zu bytes)", 2 * bytes);
    }
    int cus = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    cs::BlasCtx bc{g->g, nrhs, nullptr, nullptr, nullptr, nullptr};
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    hipError_t err = cs::blas_fill_pattern(bc, prec, bb, s);
    std::vector<cs::LaunchCfg> cands;
    for (int t : {1, 4, 8, 12}) {
        if (t > nrhs) continue;
        for (int pw : {0, 2 * cus})
            for (int lanes : {1, 2}) {
                if (lanes == 2 && prec == CS_F64) continue;
                cs::LaunchCfg lc;
                lc.rhs_tile = t;
                lc.persistent_wgs = pw;
                lc.lanes_per_site = lanes;
                cands.push_back(lc);
            }
    }
    float best_s = 1e30f, best_dd = 1e30f;
    cs::LaunchCfg bs, bd;
    for (const cs::LaunchCfg& lc : cands) {
        if (err != hipSuccess) break;
        for (int kind = 0; kind < 2 && err == hipSuccess; ++kind) {
            auto run = [&]() -> hipError_t {
                if (kind == 0) {
                    for (int h = 0; h < 4; ++h) {
                        hipError_t e2 = cs::launch_sap_halfsweep(op, prec, h & 1, 4, h == 0 ? 1 : (h == 1 ? 2 : 0),
                                                                 xb, bb, nrhs, lc, s);
                        if (e2 != hipSuccess) return e2;
                    }
                    return hipSuccess;
                }
                if (lc.rhs_tile > 1 || lc.persistent_wgs > 0) return cs::launch_dslash_tiled(op, prec, false, xb, bb, nrhs, lc, s);
                return cs::launch_dslash(op, prec, prec, prec, false, xb, bb, nullptr, nrhs, s);
            };
            err = run();  // warm-up
            if (err != hipSuccess) break;
            hipEventRecord(e0, s);
            for (int rep = 0; rep < 3 && err == hipSuccess; ++rep) err = run();
            hipEventRecord(e1, s);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess) hipEventElapsedTime(&ms, e0, e1);
            if (kind == 0 && ms < best_s) { best_s = ms; bs = lc; }
            if (kind == 1 && ms < best_dd) { best_dd = ms; bd = lc; bd.lanes_per_site = 0; }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(xb);
    hipFree(bb);
    if (err != hipSuccess) return fail(CS_ERR_HIP, "autotune: %s", hipGetErrorString(err));
    c->tuned[key] = std::make_pair(bs, bd);
    *best_sap = bs;
    *best_d = bd;
    return ok();
}

int cs_autotune(cs_gauge g, cs_clover c, cs_prec prec, int nrhs, cs_launch_config* sap, cs_launch_config* dslash,
                void* stream) {
    int st = check_op(g, c);
    if (st) return st;
    if (!valid_prec(prec)) return fail(CS_ERR_PRECISION, "unknown precision %d", (int)prec);
    if (nrhs < 1 || nrhs > 65535) return fail(CS_ERR_INVALID, "nrhs must be in 1..65535");
    if (!sap_geometry_ok(g->g))
        return fail(CS_ERR_GEOMETRY, "the red/black block colouring needs an even number of blocks per direction");
    cs::LaunchCfg a, b;
    st = autotune(g, c, prec, nrhs, (hipStream_t)stream, &a, &b);
    if (st) return st;
    if (sap) *sap = cs_launch_config{a.rhs_tile, a.persistent_wgs, a.lanes_per_site};
    if (dslash) *dslash = cs_launch_config{b.rhs_tile, b.persistent_wgs, 0};
    return ok();
}

void cs_solver_params_default(cs_solver_params* p) {
    if (!p) return;
    p->restart = 16;
    p->max_iter = 2000;
    p->n_cy = 2;
    p->n_mr = 4;
    p->tol = 1e-10;
    p->inner_prec = CS_F32;
    p->basis_prec = CS_F32;
    p->reliable_delta = 1e-5;
    p->rhs_tile = 0;
    p->use_graph = 1;
    p->block_solver = 0;
    p->rhs_groups = 1;
}

static int gcr_common(cs_gauge g, cs_clover c, const cs_solver_params* p, void* x, const void* b, int nrhs,
                      cs_solver_stats* stats, void* stream, bool dagger, const cs::MgData* mg = nullptr) {
    int st = check_op(g, c);
    if (st) return st;
    if (!p || !x || !b) return fail(CS_ERR_NULL, "params, x and b must be non-NULL");
    if (p->restart < 1 || p->restart > cs::GCR_MAX_RESTART)
        return fail(CS_ERR_INVALID, "restart must be in 1..%d", cs::GCR_MAX_RESTART);
    if (p->max_iter < 0 || p->n_cy < 0 || (p->n_cy > 0 && p->n_mr < 1))
        return fail(CS_ERR_INVALID, "max_iter and n_cy must be >= 0 and n_mr >= 1 when n_cy > 0");
    if (!(p->tol >= 0.0)) return fail(CS_ERR_INVALID, "tol must be >= 0");
    if (p->block_solver < 0 || p->block_solver > 2) return fail(CS_ERR_INVALID, "block_solver must be 0, 1 or 2");
    if (!valid_prec(p->inner_prec)) return fail(CS_ERR_PRECISION, "unknown inner precision");
    if (!valid_prec(p->basis_prec)) return fail(CS_ERR_PRECISION, "unknown basis precision");
    if (p->inner_prec == CS_F64 && p->basis_prec != CS_F64)
        return fail(CS_ERR_PRECISION, "an FP64 inner solve needs an FP64 basis");
    if ((p->basis_prec == CS_F16 || p->basis_prec == CS_BF16) && p->inner_prec != CS_F32 &&
        p->inner_prec != p->basis_prec)
        return fail(CS_ERR_PRECISION, "a 16-bit basis needs inner_prec CS_F32 or the basis' own type");
    if (mg && p->basis_prec != CS_F32 && p->basis_prec != CS_F64)
        return fail(CS_ERR_PRECISION, "the multigrid preconditioner takes basis_prec CS_F32 or CS_F64");
    if (nrhs < 1 || nrhs > 65535) return fail(CS_ERR_INVALID, "nrhs must be in 1..65535");
    if (p->rhs_tile < 0) return fail(CS_ERR_INVALID, "rhs_tile must be >= 0");
    if (p->rhs_groups < 0) return fail(CS_ERR_INVALID, "rhs_groups must be >= 0");
    if ((p->n_cy > 0 || mg) && !sap_geometry_ok(g->g))
        return fail(CS_ERR_GEOMETRY, "the red/black block colouring needs an even number of blocks per direction");
    if (mg && (nrhs != 1 || p->inner_prec != CS_F32))
        return fail(CS_ERR_INVALID, "the multigrid preconditioner takes one right-hand side and inner_prec CS_F32");
    const size_t f64 = cs::spinor_bytes_per_site(cs::P_F64) * (size_t)g->g.V;
    if (overlap(b, x, f64 * nrhs)) return fail(CS_ERR_INVALID, "x and b overlap");
    hipStream_t s = (hipStream_t)stream;
    if (dagger && c->dag_tmp_nrhs < nrhs) {
        if (c->dag_tmp) hipFree(c->dag_tmp);
        c->dag_tmp = nullptr;
        c->dag_tmp_nrhs = 0;
        if (hipMalloc(&c->dag_tmp, f64 * nrhs) != hipSuccess) {
            c->dag_tmp = nullptr;
            return fail(CS_ERR_ALLOC, "adjoint-solve workspace");
        }
        c->dag_tmp_nrhs = nrhs;
    }
    bool prof;
    {
        std::lock_guard<std::mutex> lk(g_pm);
        prof = g_prof_on;
    }
    // groups of right-hand sides: [first[q], first[q] + count[q]), each its
    // own batch (one group: the whole batch on the handle's main workspace)
    int G = p->rhs_groups > 1 && !mg ? (p->rhs_groups < nrhs ? p->rhs_groups : nrhs) : 1;
    std::vector<int> first(G), count(G);
    for (int q = 0, at = 0; q < G; ++q) {
        count[q] = nrhs / G + (q < nrhs % G ? 1 : 0);
        first[q] = at;
        at += count[q];
    }
    std::vector<cs::GcrParams> gps(G);
    std::vector<cs::GcrWork*> works(G);
    if (G > 1 && (int)c->group_work.size() < G) c->group_work.resize(G);
    for (int q = 0; q < G; ++q) {
        cs::LaunchCfg sap_cfg, d_cfg;
        if (count[q] > 1) {
            if (p->rhs_tile == 0) {
                st = autotune(g, c, p->inner_prec, count[q], s, &sap_cfg, &d_cfg);
                if (st) return st;
            } else {
                sap_cfg.rhs_tile = d_cfg.rhs_tile = p->rhs_tile;
            }
        }
        std::unique_ptr<cs::GcrWork>& wp = G > 1 ? c->group_work[q] : c->work;
        if (!wp) wp.reset(new cs::GcrWork);
        hipError_t e = wp->ensure(g->g, p->restart, p->inner_prec, p->basis_prec, count[q]);
        if (e != hipSuccess) {
            wp->release();
            return fail(CS_ERR_ALLOC, "solver workspace: %s", hipGetErrorString(e));
        }
        works[q] = wp.get();
        gps[q] = cs::GcrParams{p->restart, p->max_iter, p->n_cy, p->n_mr, p->tol, p->inner_prec, p->basis_prec,
                               p->reliable_delta, sap_cfg, d_cfg, p->use_graph != 0 && !prof, p->block_solver};
        gps[q].mg = mg;
    }
    std::vector<cs::GcrResult> res(nrhs);
    std::vector<hipError_t> errs(G, hipSuccess);
    const cs::OpData op = make_op(g, c);
    auto run = [&](int q) {
        const size_t off = f64 * (size_t)first[q];
        errs[q] = cs::gcr_solve(op, gps[q], *works[q], (char*)x + off, (const char*)b + off, count[q], dagger,
                                dagger ? (char*)c->dag_tmp + off : nullptr, res.data() + first[q], s);
    };
    const auto t0 = std::chrono::steady_clock::now();
    if (G == 1) {
        run(0);
    } else {
        std::vector<std::thread> th;
        int q = 0;
        try {
            for (; q < G; ++q) th.emplace_back(run, q);
        } catch (const std::system_error&) {
            for (; q < G; ++q) run(q);  // no thread to be had: the rest on this one, one after another
        }
        for (std::thread& t : th) t.join();
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (cs::GcrResult& r : res) r.seconds = secs;
    }
    for (int q = 0; q < G; ++q)
        if (errs[q] != hipSuccess) {
            for (cs::GcrWork* w : works) w->drop_graphs();
            return fail(CS_ERR_HIP, "solve: %s", hipGetErrorString(errs[q]));
        }
    int first_bad = CS_OK;
    for (int r = 0; r < nrhs; ++r) {
        if (stats) {
            stats[r].iters = res[r].iters;
            stats[r].restarts = res[r].restarts;
            stats[r].true_relres = res[r].true_relres;
            stats[r].seconds = res[r].seconds;
        }
        if (res[r].status != cs::GCR_OK && first_bad == CS_OK) first_bad = res[r].status;
    }
    if (first_bad != CS_OK) return fail(first_bad, "%s", cs_strerror(first_bad));
    return ok();
}

static int bicgstab_common(cs_gauge g, cs_clover c, const cs_solver_params* p, void* x, const void* b,
                           cs_solver_stats* stats, void* stream, const cs::MgData* mg) {
    int st = check_op(g, c);
    if (st) return st;
    if (!p || !x || !b) return fail(CS_ERR_NULL, "params, x and b must be non-NULL");
    if (p->max_iter < 0 || p->n_cy < 0 || (p->n_cy > 0 && p->n_mr < 1))
        return fail(CS_ERR_INVALID, "max_iter and n_cy must be >= 0 and n_mr >= 1 when n_cy > 0");
    if (!(p->tol >= 0.0)) return fail(CS_ERR_INVALID, "tol must be >= 0");
    if (p->block_solver < 0 || p->block_solver > 2) return fail(CS_ERR_INVALID, "block_solver must be 0, 1 or 2");
    if (!valid_prec(p->inner_prec)) return fail(CS_ERR_PRECISION, "unknown inner precision");
    if (p->n_cy > 0 && !sap_geometry_ok(g->g))
        return fail(CS_ERR_GEOMETRY, "the red/black block colouring needs an even number of blocks per direction");
    const size_t f64 = cs::spinor_bytes_per_site(cs::P_F64) * (size_t)g->g.V;
    if (overlap(b, x, f64)) return fail(CS_ERR_INVALID, "x and b overlap");
    if (p->basis_prec != CS_F64 && p->basis_prec != CS_F32)
        return fail(CS_ERR_PRECISION, "vector precision (basis_prec) must be CS_F64 or CS_F32");
    if (p->inner_prec == CS_F64 && p->basis_prec != CS_F64)
        return fail(CS_ERR_PRECISION, "an FP64 inner solve needs FP64 vectors");
    if (p->basis_prec == CS_F32 && !(p->reliable_delta > 0.0 && p->reliable_delta < 1.0))
        return fail(CS_ERR_INVALID, "the single-precision form needs 0 < reliable_delta < 1");
    if (mg && p->inner_prec != CS_F32)
        return fail(CS_ERR_INVALID, "the multigrid preconditioner needs inner_prec CS_F32");
    if (mg && !sap_geometry_ok(g->g))
        return fail(CS_ERR_GEOMETRY, "the red/black block colouring needs an even number of blocks per direction");
    if (!c->bicg) c->bicg.reset(new cs::BicgWork);
    hipError_t e = c->bicg->ensure(g->g, p->inner_prec, p->basis_prec);
    if (e != hipSuccess) {
        c->bicg->release();
        return fail(CS_ERR_ALLOC, "solver workspace: %s", hipGetErrorString(e));
    }
    bool prof;
    {
        std::lock_guard<std::mutex> lk(g_pm);
        prof = g_prof_on;
    }
    cs::GcrParams gp{p->restart, p->max_iter, p->n_cy, p->n_mr, p->tol, p->inner_prec, p->basis_prec,
                     p->reliable_delta, cs::LaunchCfg{}, cs::LaunchCfg{}, p->use_graph != 0 && !prof,
                     p->block_solver};
    gp.mg = mg;
    cs::GcrResult res{};
    e = cs::bicgstab_solve(make_op(g, c), gp, *c->bicg, x, b, &res, (hipStream_t)stream);
    if (e != hipSuccess) {
        c->bicg->drop_graph();
        return fail(CS_ERR_HIP, "solve: %s", hipGetErrorString(e));
    }
    if (stats) {
        stats->iters = res.iters;
        stats->restarts = res.restarts;
        stats->true_relres = res.true_relres;
        stats->seconds = res.seconds;
    }
    if (res.status != cs::GCR_OK) return fail(res.status, "%s", cs_strerror(res.status));
    return ok();
}

int cs_bicgstab_solve(cs_gauge g, cs_clover c, const cs_solver_params* p, void* x, const void* b,
                      cs_solver_stats* stats, void* stream) {
    return bicgstab_common(g, c, p, x, b, stats, stream, nullptr);
}

int cs_gcr_solve(cs_gauge g, cs_clover c, const cs_solver_params* p, void* x, const void* b, int nrhs,
                 cs_solver_stats* stats, void* stream) {
    return gcr_common(g, c, p, x, b, nrhs, stats, stream, false);
}

int cs_gcr_solve_dag(cs_gauge g, cs_clover c, const cs_solver_params* p, void* x, const void* b, int nrhs,
                     cs_solver_stats* stats, void* stream) {
    return gcr_common(g, c, p, x, b, nrhs, stats, stream, true);
}

void cs_mg_params_default(cs_mg_params* p) {
    if (!p) return;
    p->nv = 8;
    p->n_cy_setup = 4;
    p->n_mr = 4;
    p->n_adapt = 1;
    p->n_coarse = 50;
    p->n_cy_post = 2;
    p->tol_coarse = 0.05;
    p->coarse_prec = CS_F32;
    p->transfer_prec = CS_F32;
}

int cs_mg_create(cs_gauge g, cs_clover c, const cs_mg_params* p, const void* etas, void* stream, cs_mg* out) {
    int st = check_op(g, c);
    if (st) return st;
    if (!p || !etas || !out) return fail(CS_ERR_NULL, "params, etas and out must be non-NULL");
    *out = nullptr;
    if (p->nv < 1 || p->nv > cs::MG_MAX_NV) return fail(CS_ERR_INVALID, "nv must be in 1..%d", cs::MG_MAX_NV);
    if (p->n_cy_setup < 1 || p->n_mr < 1 || p->n_adapt < 0 || p->n_coarse < 1 || p->n_cy_post < 0)
        return fail(CS_ERR_INVALID, "need n_cy_setup, n_mr, n_coarse >= 1 and n_adapt, n_cy_post >= 0");
    if (!(p->tol_coarse >= 0.0)) return fail(CS_ERR_INVALID, "tol_coarse must be >= 0");
    if (!sap_geometry_ok(g->g))
        return fail(CS_ERR_GEOMETRY, "the red/black block colouring needs an even number of blocks per direction");
    std::unique_ptr<cs_mg_s> m(new cs_mg_s);
    m->gauge = g;
    m->clover = c;
    if (p->coarse_prec != CS_F32 && p->coarse_prec != CS_F16)
        return fail(CS_ERR_PRECISION, "coarse_prec must be CS_F32 or CS_F16");
    if (p->transfer_prec != CS_F32 && p->transfer_prec != CS_F16)
        return fail(CS_ERR_PRECISION, "transfer_prec must be CS_F32 or CS_F16");
    const cs::MgParams mp{p->nv,       p->n_cy_setup, p->n_mr,       p->n_adapt,
                          p->n_coarse, p->n_cy_post,  p->tol_coarse, p->coarse_prec == CS_F16 ? 1 : 0,
                          p->transfer_prec == CS_F16 ? 1 : 0};
    hipError_t e = m->data.alloc(g->g, mp);
    if (e != hipSuccess) return fail(CS_ERR_ALLOC, "multigrid workspace: %s", hipGetErrorString(e));
    if (overlap(etas, m->data.V, m->data.field_bytes() * p->nv))
        return fail(CS_ERR_INVALID, "etas overlap the hierarchy");
    CS_HIP(cs::mg_setup(make_op(g, c), m->data, etas, (hipStream_t)stream));
    *out = m.release();
    return ok();
}

int cs_mg_destroy(cs_mg m) {
    if (!m) return fail(CS_ERR_NULL, "multigrid handle is NULL");
    hipDeviceSynchronize();
    delete m;
    return ok();
}

int cs_mg_export(cs_mg m, void* P, void* Dc, void* stream) {
    if (!m) return fail(CS_ERR_NULL, "multigrid handle is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (P) CS_HIP(hipMemcpyAsync(P, m->data.P, m->data.field_bytes() * m->data.p.nv, hipMemcpyDeviceToDevice, s));
    if (Dc) CS_HIP(hipMemcpyAsync(Dc, m->data.Dc, m->data.dc_bytes(), hipMemcpyDeviceToDevice, s));
    return ok();
}

int cs_mg_restrict(cs_mg m, const void* r, void* rc, void* stream) {
    if (!m || !r || !rc) return fail(CS_ERR_NULL, "handle, r and rc must be non-NULL");
    CS_HIP(cs::mg_restrict(m->data.g, m->data.transfer(), m->data.p.nv, r, (float2*)rc, (hipStream_t)stream));
    return ok();
}

int cs_mg_prolong(cs_mg m, const void* ec, void* z, void* stream) {
    if (!m || !ec || !z) return fail(CS_ERR_NULL, "handle, ec and z must be non-NULL");
    CS_HIP(cs::mg_prolong(m->data.g, m->data.transfer(), m->data.p.nv, (const float2*)ec, z, (hipStream_t)stream));
    return ok();
}

int cs_mg_coarse_apply(cs_mg m, const void* x, void* y, void* stream) {
    if (!m || !x || !y) return fail(CS_ERR_NULL, "handle, x and y must be non-NULL");
    if (overlap(x, y, m->data.coarse_bytes())) return fail(CS_ERR_INVALID, "x and y overlap");
    CS_HIP(cs::mg_coarse_apply(m->data.g, m->data.coarse(), m->data.nc(), (const float2*)x, (float2*)y,
                               m->data.cv.tau, (hipStream_t)stream));
    return ok();
}

int cs_mg_coarse_solve(cs_mg m, const void* rc, void* ec, int n_iter, double tol, void* stream) {
    if (!m || !rc || !ec) return fail(CS_ERR_NULL, "handle, rc and ec must be non-NULL");
    if (n_iter < 0 || !(tol >= 0.0)) return fail(CS_ERR_INVALID, "need n_iter >= 0 and tol >= 0");
    hipStream_t s = (hipStream_t)stream;
    const cs::MgData& d = m->data;
    CS_HIP(cs::mg_coarse_bicgstab(d.g, d.coarse(), d.nc(), (const float2*)rc, d.cv, d.sc, d.pa, n_iter, tol, s));
    CS_HIP(hipMemcpyAsync(ec, d.cv.x, d.coarse_bytes(), hipMemcpyDeviceToDevice, s));
    return ok();
}

int cs_mg_apply(cs_mg m, void* z, const void* r, void* stream) {
    if (!m || !z || !r) return fail(CS_ERR_NULL, "handle, z and r must be non-NULL");
    if (overlap(z, r, m->data.field_bytes())) return fail(CS_ERR_INVALID, "z and r overlap");
    CS_HIP(cs::mg_apply(make_op(m->gauge, m->clover), m->data, z, r, (hipStream_t)stream));
    return ok();
}

int cs_gcr_solve_mg(cs_gauge g, cs_clover c, cs_mg m, const cs_solver_params* p, void* x, const void* b,
                    cs_solver_stats* stats, void* stream) {
    if (!m) return fail(CS_ERR_NULL, "multigrid handle is NULL");
    if (m->gauge != g || m->clover != c)
        return fail(CS_ERR_INVALID, "the multigrid handle was built for a different operator");
    return gcr_common(g, c, p, x, b, 1, stats, stream, false, &m->data);
}

int cs_bicgstab_solve_mg(cs_gauge g, cs_clover c, cs_mg m, const cs_solver_params* p, void* x, const void* b,
                         cs_solver_stats* stats, void* stream) {
    if (!m) return fail(CS_ERR_NULL, "multigrid handle is NULL");
    if (m->gauge != g || m->clover != c)
        return fail(CS_ERR_INVALID, "the multigrid handle was built for a different operator");
    return bicgstab_common(g, c, p, x, b, stats, stream, &m->data);
}

int cs_force(cs_gauge g, cs_clover c, const void* x, const void* y, double* g_lie, void* grad_U, void* stream) {
    int st = check_op(g, c);
    if (st) return st;
    if (!x || !y) return fail(CS_ERR_NULL, "x and y must be non-NULL");
    if (!g_lie && !grad_U) return fail(CS_ERR_NULL, "at least one of g_lie and grad_U must be non-NULL");
    if (!c->force_H && hipMalloc(&c->force_H, (size_t)864 * g->g.V) != hipSuccess) {
        c->force_H = nullptr;
        return fail(CS_ERR_ALLOC, "force workspace (%zu bytes)", (size_t)864 * g->g.V);
    }
    CS_HIP(cs::launch_force(g->g, g->links[cs::P_F64], c->kappa, c->csw, x, y, c->force_H, g_lie, grad_U,
                            (hipStream_t)stream));
    return ok();
}

int cs_force_noalloc(cs_gauge g, cs_clover c, const void* x, const void* y, double* g_lie, void* grad_U,
                     void* stream) {
    int st = check_op(g, c);
    if (st) return st;
    if (!x || !y) return fail(CS_ERR_NULL, "x and y must be non-NULL");
    if (!g_lie && !grad_U) return fail(CS_ERR_NULL, "at least one of g_lie and grad_U must be non-NULL");
    const size_t need = (size_t)864 * g->g.V;
    if (need > cs::FORCE_SCRATCH_BYTES)
        return fail(CS_ERR_INVALID, "lattice of %lld sites needs %zu bytes of force workspace; the fixed "
                    "workspace holds %zu bytes (%zu sites)", g->g.V, need, cs::FORCE_SCRATCH_BYTES,
                    cs::FORCE_SCRATCH_BYTES / 864);
    void* H = nullptr;
    CS_HIP(cs::force_scratch_address(&H));
    CS_HIP(cs::launch_force(g->g, g->links[cs::P_F64], c->kappa, c->csw, x, y, H, g_lie, grad_U,
                            (hipStream_t)stream));
    return ok();
}

int cs_probe_link_product(int kind, long long nsites, int reps, const float* U, const float* H, float* V,
                          void* stream) {
    if (!U || !H || !V) return fail(CS_ERR_NULL, "U, H and V must be non-NULL");
    if (kind != 0 && kind != 1) return fail(CS_ERR_INVALID, "kind must be 0 (VALU) or 1 (MFMA)");
    if (nsites <= 0 || reps < 0 || (kind == 1 && nsites % 8 != 0) || nsites > (1LL << 31))
        return fail(CS_ERR_INVALID, "nsites must be positive (a multiple of 8 for the MFMA form) and reps >= 0");
    CS_HIP(cs::launch_probe_link_product(kind, nsites, reps, U, H, V, (hipStream_t)stream));
    return ok();
}

int cs_device_copy(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src) return fail(CS_ERR_NULL, "dst and src must be non-NULL");
    if (bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0)
        return fail(CS_ERR_INVALID, "bytes and both pointers must be multiples of 16");
    const char* d = (const char*)dst;
    const char* sp = (const char*)src;
    if (d < sp + bytes && sp < d + bytes) return fail(CS_ERR_INVALID, "dst and src overlap");
    CS_HIP(cs::stream_copy(dst, src, bytes, (hipStream_t)stream));
    return ok();
}

int cs_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_pm);
    g_prof_on = on != 0;
    return ok();
}

int cs_profile_query(const char* name, long long* count, double* total_ms) {
    if (!name || !count || !total_ms) return fail(CS_ERR_NULL, "name, count and total_ms must be non-NULL");
    std::lock_guard<std::mutex> lk(g_pm);
    drain_pending();
    auto it = g_prof.find(name);
    *count = it == g_prof.end() ? 0 : it->second.first;
    *total_ms = it == g_prof.end() ? 0.0 : it->second.second;
    return ok();
}

int cs_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_pm);
    drain_pending();
    g_prof.clear();
    return ok();
}

}  // extern "C"
