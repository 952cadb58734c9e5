"""Benchmark: mixed-precision SAP-preconditioned flexible GCR on one MI355X.

One step = one solve of D x = b to a true relative residual of 1e-10 on the
HBM-resident 32^3 x 64 synthetic gauge field (eps 0.25, kappa 0.1370, c_sw
1.1): FP32 SAP smoother (2 red/black cycles of 4 MR steps on 4^4 blocks) and
FP32 w = D z inside an FP64 flexible GCR(16) with FP64 residual
recomputation.  b is resident in HBM and x starts at zero; iterations are
replayed as captured HIP graphs.

Prints one JSON line: the timed solves (value = solves per second), the
FP64-only GPU solve of the same system and the mixed/FP64 ratio, the
roofline of the dominant kernel (the SAP half-sweep with x nonzero, HIP
events around every launch in an eager pass of the same solves, against
1008 algorithmic bytes per visited site), the operator's bandwidth, the
library's plain copy kernel in the same run, the FP16 / BF16 smoothers, and
the FP64 CPU oracle timed on the host.  Side measurements (cache-resident
16^3 x 32, the 16^4 low-precision sub-run against the oracle, 24 right-hand
sides on 24^3 x 48, the gradient, multigrid and the solver variants) follow
unless --no-extras.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Dslash/SAP HBM GB/s (% peak); time-to-1e-10 residual, mixed vs FP64, 1 GPU"
SAP_KERNEL_SOURCES = ["sap.hip", "dslash_core.hpp", "fields.hpp", "cs_internal.hpp", "wave.hpp"]
DSLASH_KERNEL_SOURCES = ["dslash.hip", "dslash_core.hpp", "fields.hpp", "cs_internal.hpp"]

# Algorithmic bytes per visited site of one SAP half-sweep, FP32 storage:
# every field the visit needs, counted once per site: b (96), x (96), the two
# face-neighbour spinors a site has on average (192), the written x (96), four
# own links (192) plus the one boundary-crossing backward link per site on
# average (48), the clover term (288).  The first half-sweep from x = 0 needs
# neither x nor the halo nor the backward links; the second needs no own x.
SAP_BYTES_F32 = {1: 96 + 192 + 288 + 96, 2: 96 + 192 + 192 + 48 + 288 + 96, 0: 1008}
DSLASH_BYTES_F32 = 96 + 96 + 192 + 288  # in, out, four links, clover

# Floating-point operations per visited site of a SAP half-sweep (complex add
# 2, multiply 6, multiply-add 8).  One hop: spin projection 12, SU(3) times a
# half spinor 132, reconstruction into the sum 24, so 168; the clover term of
# both chiralities 2 x (36 mul + 30 add) = 552; out = cx - kappa acc 48.  Full
# operator 1944; the Dirichlet block operator keeps 6 of the 8 hops on
# average (1608).  MR step: D_BB + <q,q> 48 + <q,rho> 96 + two axpys 192 =
# 1944.  Visit: mode 0 = residual (1944 + 24) + 4 MR steps + x update 24;
# mode 1 (x = 0) = 4 MR steps; mode 2 (own block zero) = 2 face hops on
# average + combine (384) + 4 MR steps.
SAP_FLOPS = {0: 1968 + 4 * 1944 + 24, 1: 4 * 1944, 2: 384 + 4 * 1944}
# Published FP32 vector peak of MI355X (256 CUs at 2.4 GHz).  The library
# emits no packed FP32 instructions; FMA-dense code without them reached
# 105 TFLOP/s on this part (bench.py --mfma-probe), above the 78.6 TFLOP/s
# that 16 FMA lanes per SIMD would allow, so the published figure is the
# ceiling used.
FP32_VALU_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2112_00501_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(record: str, sources):
    """HBM bytes per launch from a committed rocprofv3 counter record, if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"{record}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash(sources):
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def timed_events(torch, fn, n):
    """Average duration (us) of fn() over n calls, HIP events on the current
    stream (the one the library launches on), after one untimed call."""
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(n):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n * 1e3


def copy_bandwidth(cs, torch, nbytes=1 << 30, reps=10):
    """Read + write bandwidth of the library's plain copy kernel (GB/s)."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    c = torch.empty_like(a)
    us = timed_events(torch, lambda: cs.device_copy(c, a), reps)
    del a, c
    torch.cuda.empty_cache()
    return dict(bytes_copied=nbytes, reps=reps, avg_us=round(us, 2), GBps=round(2 * nbytes / (us * 1e-6) / 1e9, 1),
                kernel="k_stream_copy (cs_device_copy): one 16-byte word per lane, read + write counted")


def cpu_baseline(U, b, c, gpu_fp64_iters, small):
    """The FP64 oracle (plain C, -O3 -march=native, OpenMP over sites and
    blocks) on this host.  The metric's unit is solves/s on the 32^3x64
    system; a full oracle solve there takes hours, so the sample is two
    FGCR(16) iterations of that solve on all host threads, scaled by the
    iteration count of the GPU's FP64-only solve.  Beside it: the operator
    and one SAP application at 16^3x32 and 32^3x64 on all threads and at
    16^3x32 on one thread, at 16^4 and 24^3x48 on all threads, and complete
    FP64 solves to 1e-10 at 8^4 and 16^3x32."""
    import numpy as np

    import oracle
    dims, kappa, csw = c["dims"], c["kappa"], c["csw"]
    threads = min(16, len(os.sched_getaffinity(0)))
    res = dict(kind="oracle", cpu_model=cpu_model(), affinity_cpus=len(os.sched_getaffinity(0)),
               build=oracle.build_flags())
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    T = oracle.clover_field(dims, U, kappa, csw)
    t_cl = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.apply_D(dims, U, T, kappa, b)
    t_d = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, st, it, rel, _ = oracle.fgcr(dims, (4, 4, 4, 4), U, T, kappa, b, n_cy=2, n_mr=4, restart=16, tol=1e-10,
                                    max_iter=2)
    t_2 = time.perf_counter() - t0
    per_iter = t_2 / 2
    solve_s = per_iter * gpu_fp64_iters
    res.update(value=round(1.0 / solve_s, 6), unit="solves/s", cores=threads,
               sample=(f"2 FGCR(16) iterations of the FP64 oracle on the {'x'.join(map(str, dims))} system "
                       f"({t_2:.2f} s on {threads} threads, clover build {t_cl:.2f} s excluded), per-iteration "
                       f"time x {gpu_fp64_iters} iterations (the FP64-only GPU solve's count) = "
                       f"{solve_s:.1f} s per solve"),
               seconds_per_iteration=round(per_iter, 3), estimated_solve_s=round(solve_s, 1))
    per = {}
    t0 = time.perf_counter()
    oracle.sap(dims, (4, 4, 4, 4), U, T, kappa, 2, 4, b)
    per["x".join(map(str, dims))] = dict(threads=threads, apply_D_s=round(t_d, 3),
                                         sap_application_s=round(time.perf_counter() - t0, 3))
    del T
    Us, bs, cs_ = small
    ds = cs_["dims"]
    Ts = oracle.clover_field(ds, Us, cs_["kappa"], cs_["csw"])
    for th in sorted({1, threads}):
        oracle.set_threads(th)
        t0 = time.perf_counter()
        oracle.apply_D(ds, Us, Ts, cs_["kappa"], bs)
        td = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.sap(ds, (4, 4, 4, 4), Us, Ts, cs_["kappa"], 2, 4, bs)
        per[f"16x16x16x32_{th}_threads"] = dict(threads=th, apply_D_s=round(td, 4),
                                                sap_application_s=round(time.perf_counter() - t0, 4))
    oracle.set_threads(threads)
    # complete FP64 SAP-FGCR(16) solves to 1e-10 where they take seconds, and
    # the operator and one SAP application on the other lattices
    for name, cfgname in (("8x8x8x8", "plain_fp64_8x8x8x8"), ("16x16x16x32", "mixed_16x16x16x32")):
        cc = synth_configs()[cfgname]
        if cfgname == "mixed_16x16x16x32":
            Uc, bc, Tc = Us, bs, Ts
        else:
            Uc = synth_gauge(cc)
            bc = synth_source(cc)
            Tc = oracle.clover_field(cc["dims"], Uc, cc["kappa"], cc["csw"])
        t0 = time.perf_counter()
        _, st_, it_, rel_, _ = oracle.fgcr(cc["dims"], (4, 4, 4, 4), Uc, Tc, cc["kappa"], bc, n_cy=2, n_mr=4,
                                           restart=16, tol=1e-10)
        per[f"{name}_fgcr_solve"] = dict(threads=threads, seconds=round(time.perf_counter() - t0, 3),
                                         iterations=it_, status=st_, true_relres=float(f"{rel_:.2e}"))
    for name, cfgname in (("16x16x16x16", "lowprec_sub_16x16x16x16"), ("24x24x24x48", "multirhs_24x24x24x48")):
        cc = synth_configs()[cfgname]
        Uc, bc = synth_gauge(cc), synth_source(cc)
        Tc = oracle.clover_field(cc["dims"], Uc, cc["kappa"], cc["csw"])
        t0 = time.perf_counter()
        oracle.apply_D(cc["dims"], Uc, Tc, cc["kappa"], bc)
        td = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.sap(cc["dims"], (4, 4, 4, 4), Uc, Tc, cc["kappa"], 2, 4, bc)
        per[name] = dict(threads=threads, apply_D_s=round(td, 4), sap_application_s=round(time.perf_counter() - t0, 4))
        del Uc, bc, Tc
    res["per_lattice"] = per
    res["next_rows"] = next_rows_oracle(Us, bs, cs_, Ts)
    return res


def next_rows_oracle(U, b, c, T):
    """The oracle on the work that next_rows() times on the GPU: one Jacobi
    and one even-odd SAP application and complete flexible-BiCGStab
    (reliable updates at 1e-5, as the library's default) and Richardson
    solves on the 16^3x32 system, and the two-level multigrid (setup, then
    MG-FGCR to 1e-10) on 8^4 with 8 null vectors, all FP64 on the threads
    set by the caller."""
    import oracle
    from oracle import mg
    dims, kappa, bdim = c["dims"], c["kappa"], (4, 4, 4, 4)
    out = {}
    t0 = time.perf_counter()
    oracle.sap_jacobi(dims, bdim, U, T, kappa, 2, 4, b)
    out["sap_jacobi_application_s"] = round(time.perf_counter() - t0, 4)
    t0 = time.perf_counter()
    oracle.sap_eo(dims, bdim, U, T, kappa, 2, 4, b)
    out["sap_eo_application_s"] = round(time.perf_counter() - t0, 4)
    t0 = time.perf_counter()
    _, st, it, rs, rel, _ = oracle.fbicgstab(dims, bdim, U, T, kappa, b, n_cy=2, n_mr=4, tol=1e-10, delta=1e-5)
    out["fbicgstab_solve"] = dict(seconds=round(time.perf_counter() - t0, 3), iterations=it, restarts=rs,
                                  status=st, true_relres=float(f"{rel:.2e}"))
    t0 = time.perf_counter()
    _, st, it, outer, rel = oracle.richardson_bicgstab(dims, bdim, U, T, kappa, b, n_cy=2, n_mr=4, tol=1e-10)
    out["richardson_bicgstab_solve"] = dict(seconds=round(time.perf_counter() - t0, 3), inner_iterations=it,
                                            outer_steps=outer, status=st, true_relres=float(f"{rel:.2e}"))
    res = {"16x16x16x32": out}
    c8 = synth_configs()["mg_8x8x8x8"]
    d8, k8 = c8["dims"], c8["kappa"]
    U8, b8 = synth_gauge(c8), synth_source(c8)
    T8 = oracle.clover_field(d8, U8, k8, c8["csw"])
    from paper_2112_00501_amd import synth
    q = MG8_PARAMS
    etas = [synth.source(d8, c8["mg_eta_seed"] + i) for i in range(q["nv"])]
    t0 = time.perf_counter()
    P, Dc, aggs, _ = mg.setup(d8, bdim, U8, T8, k8, etas, n_cy_setup=q["n_cy_setup"], n_mr=q["n_mr"],
                              n_adapt=q["n_adapt"], n_coarse=q["n_coarse"], n_cy_post=q["n_cy_post"],
                              tol_coarse=q["tol_coarse"])
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, it, rel = mg.fgcr(lambda v: oracle.apply_D(d8, U8, T8, k8, v),
                         lambda r: mg.mg_apply(d8, bdim, U8, T8, k8, P, aggs, Dc, r, q["n_coarse"], q["n_cy_post"],
                                               q["n_mr"], q["tol_coarse"]), b8, restart=16, tol=1e-10)
    res["8x8x8x8"] = dict(mg_setup_s=round(t_setup, 3),
                          mg_fgcr_solve=dict(seconds=round(time.perf_counter() - t0, 3), iterations=it,
                                             true_relres=float(f"{rel:.2e}")),
                          params=dict(q))
    return res


def next_rows(cs, synth, torch, reps=3):
    """The rows beyond the SAP-FGCR path, timed where the oracle's timing of
    the same work (cpu_baseline's next_rows) is quick: one application of
    the Jacobi and even-odd SAP smoothers (FP64 and FP32) and complete
    flexible-BiCGStab (FP64 and FP32 smoother) and Richardson solves on the
    16^3x32 system, and the two-level multigrid on 8^4 (setup, then MG-FGCR
    to 1e-10).  Wall times of whole calls, medians after a warm-up."""
    c = synth.CONFIGS["mixed_16x16x16x32"]
    dims = c["dims"]
    U = synth.gauge_field(dims, c["eps"], c["gauge_seed"])
    b = synth.source(dims, c["src_seed"])
    lat = cs.Lattice(dims)
    op = cs.Operator(lat, torch.from_numpy(U).cuda(), c["kappa"], c["csw"])
    out = {}
    for prec, name in ((cs.F64, "f64"), (cs.F32, "f32")):
        bp = lat.import_field(torch.from_numpy(b).cuda(), prec)
        xp = lat.new_field(prec)
        out[f"sap_jacobi_application_us_{name}"] = round(timed_events(
            torch, lambda: op.sap_smooth_jacobi(xp, bp, prec, n_cy=2, n_jac=4, x0_is_zero=True), 10), 1)
        out[f"sap_eo_application_us_{name}"] = round(timed_events(
            torch, lambda: op.sap_smooth_eo(xp, bp, prec, n_cy=2, n_mr=4, x0_is_zero=True), 10), 1)
        del bp, xp
    bd = lat.import_field(torch.from_numpy(b).cuda(), cs.F64)
    xd = lat.new_field(cs.F64)
    for name, p in (("fbicgstab_fp64_smoother", cs.SolverParams(inner_prec=cs.F64, basis_prec=cs.F64)),
                    ("fbicgstab_fp32_smoother", cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F64)),
                    ("sp_bicgstab_in_fp64_richardson", cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32))):
        t, it, st = time_bicgstab(cs, torch, op, xd, bd, p, reps)
        out[name] = dict(ms=round(t * 1e3, 3), iterations=it, status=st)
    del op, bd, xd
    res = {"16x16x16x32": out}
    c8 = synth.CONFIGS["mg_8x8x8x8"]
    d8 = c8["dims"]
    U8, b8 = synth.gauge_field(d8, c8["eps"], c8["gauge_seed"]), synth.source(d8, c8["src_seed"])
    lat8 = cs.Lattice(d8)
    op8 = cs.Operator(lat8, torch.from_numpy(U8).cuda(), c8["kappa"], c8["csw"])
    prm = cs.MgParams(**MG8_PARAMS)
    fb = lat8.field_bytes(cs.F32)
    etas = lat8.new_field(cs.F32, prm.nv)
    for i in range(prm.nv):
        lat8.import_field(torch.from_numpy(synth.source(d8, c8["mg_eta_seed"] + i)).cuda(), cs.F32,
                          out=etas[i * fb:(i + 1) * fb])
    bd8 = lat8.import_field(torch.from_numpy(b8).cuda(), cs.F64)
    xd8 = lat8.new_field(cs.F64)
    setups = []
    for i in range(reps + 1):
        torch.cuda.synchronize()
        t = time.perf_counter()
        m = cs.Multigrid(op8, etas, prm)
        torch.cuda.synchronize()
        if i:
            setups.append(time.perf_counter() - t)
        if i < reps:
            del m
    p = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32, tol=1e-10)
    times = []
    for i in range(reps + 1):
        xd8.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, stats = m.gcr_solve(xd8, bd8, p, allow_fail=True)
        torch.cuda.synchronize()
        if i:
            times.append(time.perf_counter() - t)
    res["8x8x8x8"] = dict(mg_setup_ms=round(sorted(setups)[len(setups) // 2] * 1e3, 3),
                          mg_fgcr_solve=dict(ms=round(sorted(times)[len(times) // 2] * 1e3, 3),
                                             iterations=stats["iters"], status=st),
                          params=dict(MG8_PARAMS),
                          note="FP32 hierarchy inside FP64 FGCR; 16 aggregates, latency-bound at this size")
    del m, op8
    torch.cuda.empty_cache()
    return res


def synth_configs():
    from paper_2112_00501_amd import synth
    return synth.CONFIGS


def synth_gauge(c):
    from paper_2112_00501_amd import synth
    return synth.gauge_field(c["dims"], c["eps"], c["gauge_seed"])


def synth_source(c):
    from paper_2112_00501_amd import synth
    return synth.source(c["dims"], c["src_seed"])


# Two-level multigrid of the paper's Section 3: N_vec = 16 null vectors from
# SAP-smoothed random vectors and 4 adaptive passes, coarse BiCGStab to 5%
# (at most 50 iterations), 2 SAP post-smoothing cycles of 4 MR steps.
MG_PARAMS = dict(nv=16, n_cy_setup=4, n_mr=4, n_adapt=4, n_coarse=50, n_cy_post=2, tol_coarse=0.05)
# The same hierarchy with 8 null vectors, for the 8^4 comparison with the
# oracle (whose dense coarse operator is assembled column by column).
MG8_PARAMS = dict(MG_PARAMS, nv=8)


def multigrid_measurement(cs, synth, torch, op, lat, c, U, b, bd, xd, sap_s, sap_it, reps=3, half=False):
    """MG-preconditioned FGCR to 1e-10 on the same system as SAP-FGCR:
    setup time, solve time (median of reps), iterations, per-family kernel
    time of one solve, and the paper's outer solver (flexible BiCGStab)
    around the same hierarchy."""
    import numpy as np

    import oracle
    dims = c["dims"]
    prm = cs.MgParams(**MG_PARAMS)
    if half:  # FP16 copies of D_c and P for the bandwidth-bound coarse products and transfers
        prm.coarse_prec = prm.transfer_prec = cs.F16
    fb = lat.field_bytes(cs.F32)
    etas = lat.new_field(cs.F32, prm.nv)
    for i in range(prm.nv):
        eta = torch.from_numpy(synth.source(dims, c["mg_eta_seed"] + i)).cuda()
        lat.import_field(eta, cs.F32, out=etas[i * fb:(i + 1) * fb])
        del eta
    torch.cuda.synchronize()
    t = time.perf_counter()
    m = cs.Multigrid(op, etas, prm)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    p = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32, tol=1e-10)
    times = []
    for i in range(reps + 1):
        xd.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, stats = m.gcr_solve(xd, bd, p, allow_fail=True)
        torch.cuda.synchronize()
        if i:
            times.append(time.perf_counter() - t)
    solve_s = float(sorted(times)[len(times) // 2])
    x = lat.export_field(xd, cs.F64).cpu().numpy()
    rel = oracle.residual_norm(dims, U, c["kappa"], c["csw"], b, x) / np.linalg.norm(b)
    # the paper's outer solver around the same hierarchy: flexible BiCGStab
    pb = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F64, tol=1e-10, reliable_delta=1e-5)
    btimes = []
    for i in range(reps + 1):
        xd.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        bst, bstats = m.bicgstab_solve(xd, bd, pb, allow_fail=True)
        torch.cuda.synchronize()
        if i:
            btimes.append(time.perf_counter() - t)
    bsolve_s = float(sorted(btimes)[len(btimes) // 2])
    xb = lat.export_field(xd, cs.F64).cpu().numpy()
    brel = oracle.residual_norm(dims, U, c["kappa"], c["csw"], b, xb) / np.linalg.norm(b)
    cs.profile_reset()
    cs.profile_enable(True)
    xd.zero_()
    m.gcr_solve(xd, bd, p, allow_fail=True)
    torch.cuda.synchronize()
    cs.profile_enable(False)
    fam = {k: cs.profile_query(k) for k in ("mg", "sap_halfsweep", "dslash", "blas")}
    del m, etas
    torch.cuda.empty_cache()
    return dict(params=dict(MG_PARAMS, coarse_prec="f16" if half else "f32", transfer_prec="f16" if half else "f32"),
                setup_s=round(setup_s, 4), solve_s=round(solve_s, 4),
                iterations=stats["iters"], status=st, oracle_checked_relres=float(f"{rel:.3e}"),
                sap_fgcr_solve_s=round(sap_s, 4), sap_fgcr_iterations=sap_it,
                solve_speedup_vs_sap_fgcr=round(sap_s / solve_s, 3),
                kernels_ms_one_solve={k: round(v[1], 3) for k, v in fam.items()},
                fbicgstab=dict(solve_s=round(bsolve_s, 4), iterations=bstats["iters"], status=bst,
                               oracle_checked_relres=float(f"{brel:.3e}"),
                               note="flexible BiCGStab (FP64 vectors) with M_MG on the right, two applications "
                                    "per iteration: the paper's outer solver"),
                note=("FP32 multigrid preconditioner (P, D_c and coarse vectors FP32, coarse reductions "
                      "FP64) inside FP64 flexible GCR(16); aggregates are the 4^4 SAP blocks; the "
                      "kernel times come from an eager pass with HIP events around every launch"))


def kappa_scan(cs, synth, torch, lat, c, U, b, kappas=(0.1375, 0.1380, 0.1385)):
    """SAP-FGCR against MG-FGCR (FP16 copies of D_c and P) on the same gauge
    field and source at lighter quark masses (kappa closer to critical):
    the regime where the paper finds the multigrid solver ahead.  Each
    solve timed after one warm-up solve; a fresh hierarchy per kappa."""
    dims = c["dims"]
    prm = cs.MgParams(**MG_PARAMS)
    prm.coarse_prec = prm.transfer_prec = cs.F16
    fb = lat.field_bytes(cs.F32)
    etas = lat.new_field(cs.F32, prm.nv)
    for i in range(prm.nv):
        lat.import_field(torch.from_numpy(synth.source(dims, c["mg_eta_seed"] + i)).cuda(), cs.F32,
                         out=etas[i * fb:(i + 1) * fb])
    Ud = torch.from_numpy(U).cuda()
    bd = lat.import_field(torch.from_numpy(b).cuda(), cs.F64)
    xd = lat.new_field(cs.F64)
    p = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32, max_iter=3000)
    rows = []
    for kappa in kappas:
        op = cs.Operator(lat, Ud, kappa, c["csw"])

        def timed(solve):
            xd.zero_()
            solve()  # warm-up: workspace and graph capture
            xd.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            st, stats = solve()
            torch.cuda.synchronize()
            st_ = stats[0] if isinstance(stats, list) else stats
            return time.perf_counter() - t, st_["iters"], st
        ts, its, sts = timed(lambda: op.gcr_solve(xd, bd, p, allow_fail=True))
        torch.cuda.synchronize()
        t = time.perf_counter()
        m = cs.Multigrid(op, etas, prm)
        torch.cuda.synchronize()
        tset = time.perf_counter() - t
        tm, itm, stm = timed(lambda: m.gcr_solve(xd, bd, p, allow_fail=True))
        rows.append(dict(kappa=kappa, sap_fgcr_s=round(ts, 4), sap_fgcr_iterations=its, sap_fgcr_status=sts,
                         mg_setup_s=round(tset, 4), mg_fgcr_s=round(tm, 4), mg_fgcr_iterations=itm,
                         mg_fgcr_status=stm, solve_speedup=round(ts / tm, 3),
                         twelve_equations_speedup=round(12 * ts / (tset + 12 * tm), 3)))
        del m, op
        torch.cuda.empty_cache()
    return rows


def time_gcr(cs, torch, op, xd, bd, p, reps):
    """Median wall time (s) of FGCR solves from x = 0 after one warm-up."""
    times = []
    for i in range(reps + 1):
        xd.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, stats = op.gcr_solve(xd, bd, p, allow_fail=True)
        torch.cuda.synchronize()
        if i:
            times.append(time.perf_counter() - t)
    return float(sorted(times)[len(times) // 2]), stats[0]["iters"], st


def time_bicgstab(cs, torch, op, xd, bd, p, reps):
    """Median wall time (s) of flexible BiCGStab solves from x = 0 after one
    warm-up solve, with the iteration count and status of the last."""
    times = []
    for i in range(reps + 1):
        xd.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, stats = op.bicgstab_solve(xd, bd, p, allow_fail=True)
        torch.cuda.synchronize()
        if i:
            times.append(time.perf_counter() - t)
    return float(sorted(times)[len(times) // 2]), stats["iters"], st


def lowprec_subrun(cs, synth, torch):
    """16^4 sub-run of the low-precision configuration: FP16 / BF16 smoother
    solutions against the FP64 oracle's solution, and the iteration penalty."""
    import numpy as np

    import oracle
    c = synth.CONFIGS["lowprec_sub_16x16x16x16"]
    dims = c["dims"]
    U = synth.gauge_field(dims, c["eps"], c["gauge_seed"])
    b = synth.source(dims, c["src_seed"])
    oracle.set_threads(min(16, len(os.sched_getaffinity(0))))
    T = oracle.clover_field(dims, U, c["kappa"], c["csw"])
    xo, st, ito, relo, _ = oracle.fgcr(dims, (4, 4, 4, 4), U, T, c["kappa"], b, tol=1e-12)
    lat = cs.Lattice(dims)
    op = cs.Operator(lat, torch.from_numpy(U).cuda(), c["kappa"], c["csw"])
    bd = lat.import_field(torch.from_numpy(b).cuda(), cs.F64)
    xd = lat.new_field(cs.F64)
    res = dict(lattice="16x16x16x16", oracle_iterations=ito, oracle_relres=float(f"{relo:.2e}"))
    for name, inner in (("f32", cs.F32), ("f16", cs.F16), ("bf16", cs.BF16), ("f64", cs.F64)):
        xd.zero_()
        st, stats = op.gcr_solve(xd, bd, cs.SolverParams(inner_prec=inner,
                                                         basis_prec=cs.F64 if inner == cs.F64 else cs.F32),
                                 allow_fail=True)
        x = lat.export_field(xd, cs.F64).cpu().numpy()
        res[f"{name}_iterations"] = stats[0]["iters"]
        res[f"{name}_rel_error_vs_oracle"] = float(f"{np.linalg.norm(x - xo) / np.linalg.norm(xo):.3e}")
        res[f"{name}_oracle_checked_relres"] = float(
            f"{oracle.residual_norm(dims, U, c['kappa'], c['csw'], b, x) / np.linalg.norm(b):.3e}")
    return res


def multirhs_measurement(cs, synth, torch, nrhs=24):
    """24 right-hand sides on 24^3 x 48: autotuned tile and launch shape,
    bandwidth per right-hand side of the batched operator and smoother, and
    time to 1e-10 for all 24 (one batch, and two concurrent groups of 12,
    graph-replayed) against 24 one-by-one solves."""
    import numpy as np
    c = synth.CONFIGS["multirhs_24x24x24x48"]
    dims = c["dims"]
    U = synth.gauge_field(dims, c["eps"], c["gauge_seed"])
    lat = cs.Lattice(dims)
    op = cs.Operator(lat, torch.from_numpy(U).cuda(), c["kappa"], c["csw"])
    del U
    V = lat.volume
    B = torch.empty((nrhs, V, 4, 3), dtype=torch.complex128)
    for j in range(nrhs):
        B[j] = torch.from_numpy(synth.source(dims, c["src_seed"] + 100 * j))
    Bd = B.cuda()
    del B
    sap_cfg, d_cfg = op.autotune(cs.F32, nrhs)
    b32 = lat.import_field(Bd, cs.F32)
    x32 = lat.new_field(cs.F32, nrhs)
    op.apply_D_cfg(x32, b32, cs.F32, nrhs, d_cfg)
    op.sap_smooth_cfg(x32, b32, cs.F32, nrhs, sap_cfg)
    torch.cuda.synchronize()
    cs.profile_reset()
    cs.profile_enable(True)
    for _ in range(5):
        op.apply_D_cfg(x32, b32, cs.F32, nrhs, d_cfg)
    for _ in range(3):
        op.sap_smooth_cfg(x32, b32, cs.F32, nrhs, sap_cfg)
    torch.cuda.synchronize()
    cs.profile_enable(False)
    nd, msd = cs.profile_query("dslash")
    ns, mss = cs.profile_query("sap_halfsweep")
    d_us = msd / nd * 1e3
    s_us = mss / 3 * 1e3
    t = sap_cfg.rhs_tile
    td = d_cfg.rhs_tile
    # algorithmic bytes with link and clover reuse over a tile of t right-hand sides
    d_bytes = (192 + 480 / td) * V * nrhs
    # own links (192) and clover (288) are read once per tile of t right-hand sides
    s_bytes = sum((SAP_BYTES_F32[m] - 480 + 480 / t) for m in (1, 2, 0, 0)) * V / 2 * nrhs
    res = dict(lattice="24x24x24x48", nrhs=nrhs, sap_rhs_tile=t, sap_persistent_wgs=sap_cfg.persistent_wgs,
               dslash_rhs_tile=td, dslash_persistent_wgs=d_cfg.persistent_wgs,
               dslash_us_all_rhs=round(d_us, 1), dslash_GBps=round(d_bytes / (d_us * 1e-6) / 1e9, 1),
               dslash_us_per_rhs=round(d_us / nrhs, 2),
               sap_application_us_all_rhs=round(s_us, 1), sap_GBps=round(s_bytes / (s_us * 1e-6) / 1e9, 1),
               sap_application_us_per_rhs=round(s_us / nrhs, 2))
    del b32, x32
    bd = lat.import_field(Bd, cs.F64)
    del Bd
    xd = lat.new_field(cs.F64, nrhs)
    p = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32, rhs_tile=0, use_graph=True)
    xd.zero_()
    op.gcr_solve(xd, bd, p, nrhs=nrhs, allow_fail=True)  # warm-up: workspace, graphs
    xd.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, stats = op.gcr_solve(xd, bd, p, nrhs=nrhs, allow_fail=True)
    torch.cuda.synchronize()
    res["batched_time_to_1e-10_all_rhs_s"] = round(time.perf_counter() - t0, 4)
    res["batched_status"] = st
    res["iterations_min_max"] = [min(s["iters"] for s in stats), max(s["iters"] for s in stats)]
    res["worst_true_relres"] = float(f"{max(s['true_relres'] for s in stats):.3e}")
    # the same batch as two groups of 12 solved concurrently (own workspaces,
    # streams and host threads inside the one call)
    pg = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32, rhs_tile=0, use_graph=True, rhs_groups=2)
    xd.zero_()
    op.gcr_solve(xd, bd, pg, nrhs=nrhs, allow_fail=True)  # warm-up: workspaces, graphs
    xd.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st2, stats2 = op.gcr_solve(xd, bd, pg, nrhs=nrhs, allow_fail=True)
    torch.cuda.synchronize()
    res["groups2_time_to_1e-10_all_rhs_s"] = round(time.perf_counter() - t0, 4)
    res["groups2_status"] = st2
    res["groups2_worst_true_relres"] = float(f"{max(s['true_relres'] for s in stats2):.3e}")
    # the same 24 right-hand sides one by one (single-RHS path, graphs on)
    fbytes = lat.field_bytes(cs.F64)
    x1 = lat.new_field(cs.F64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(nrhs):
        x1.zero_()
        op.gcr_solve(x1, bd[j * fbytes:(j + 1) * fbytes], cs.SolverParams(), allow_fail=True)
    torch.cuda.synchronize()
    res["sequential_time_to_1e-10_all_rhs_s"] = round(time.perf_counter() - t0, 4)
    res["batched_speedup"] = round(res["sequential_time_to_1e-10_all_rhs_s"] / res["batched_time_to_1e-10_all_rhs_s"], 3)
    res["groups2_speedup"] = round(res["sequential_time_to_1e-10_all_rhs_s"] / res["groups2_time_to_1e-10_all_rhs_s"], 3)
    return res


def gradient_measurement(cs, synth, torch):
    """Forward solve and backward pass (adjoint solve + force) of
    L = Re(eta^dag D^-1 b) on 32^3 x 64 through torch.autograd, with the
    forward solution and operator kept for the backward pass, and with both
    recomputed in the backward pass instead (nothing held in between)."""
    c = synth.CONFIGS["grad_32x32x32x64"]
    dims = c["dims"]
    U0 = torch.from_numpy(synth.gauge_field(dims, c["eps"], c["gauge_seed"])).cuda()
    b0 = torch.from_numpy(synth.source(dims, c["src_seed"])).cuda()
    eta = torch.from_numpy(synth.source(dims, c["eta_seed"])).cuda()
    lat = cs.Lattice(dims)
    params = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32)
    res = dict(lattice="32x32x32x64")
    for recompute in (False, True):
        U = U0.clone().requires_grad_(True)
        b = b0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = cs.CloverSolve.apply(U, b, lat, c["kappa"], c["csw"], params, recompute)
        L = (torch.conj(eta) * x).sum().real
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        key = "recompute" if recompute else "stored"
        res[key] = dict(forward_s=round(t1 - t0, 4), backward_s=round(t2 - t1, 4),
                        grad_U_maxabs=float(f"{float(U.grad.abs().max()):.4e}"),
                        loss=float(f"{float(L.detach()):.6e}"))
        del U, b, x, L
        torch.cuda.empty_cache()
    res["note"] = ("forward includes gauge import and clover build; backward = adjoint solve + force (and, "
                   "with recompute, the operator rebuild and the forward solve again)")
    return res


def cached_field(synth, cfg, cache_dir):
    """Gauge field and source of a configuration, generated once and kept as
    .npy files in cache_dir (if given) for later processes of the same job."""
    import numpy as np
    dims = cfg["dims"]
    if cache_dir:
        os.makedirs(cache_dir, exist_ok=True)
        tag = f"{'x'.join(map(str, dims))}_{cfg['gauge_seed']}_{cfg['src_seed']}_{cfg['eps']}"
        pu, pb = os.path.join(cache_dir, f"U_{tag}.npy"), os.path.join(cache_dir, f"b_{tag}.npy")
        if os.path.exists(pu) and os.path.exists(pb):
            return np.load(pu), np.load(pb)
    U = synth.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    b = synth.source(dims, cfg["src_seed"])
    if cache_dir:
        np.save(pu + ".tmp.npy", U)
        np.save(pb + ".tmp.npy", b)
        os.replace(pu + ".tmp.npy", pu)
        os.replace(pb + ".tmp.npy", pb)
    return U, b


def probe32(cs, synth, torch, prec, cache_dir, n_sap=10, n_d=10, n_copy=5):
    """A short fixed workload on the 32^3x64 field for profiler passes:
    n_sap SAP applications (2 cycles of 4 MR steps) from a nonzero start
    vector, so that every half-sweep is a general (mode 0) visit, n_d
    operator launches, and n_copy 1 GiB device copies by the library's
    copy kernel (the bandwidth reference and counter calibration)."""
    c = synth.CONFIGS["lowprec_32x32x32x64"]
    U, b = cached_field(synth, c, cache_dir)
    lat = cs.Lattice(c["dims"])
    op = cs.Operator(lat, torch.from_numpy(U).cuda(), c["kappa"], c["csw"])
    del U
    bd = lat.import_field(torch.from_numpy(b).cuda(), prec)
    xd = lat.import_field(torch.from_numpy(b).cuda(), prec)
    out = lat.new_field(prec)
    torch.cuda.synchronize()
    log(f"[probe32] {n_sap} SAP applications, prec {prec}")
    for _ in range(n_sap):
        op.sap_smooth(xd, bd, prec, n_cy=2, n_mr=4, x0_is_zero=False)
    log(f"[probe32] {n_d} operator launches")
    for _ in range(n_d):
        op.apply_D(out, bd, prec)
    torch.cuda.synchronize()
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    d = torch.empty_like(a)
    log(f"[probe32] {n_copy} device copies of 1 GiB")
    for _ in range(n_copy):
        cs.device_copy(d, a)
    torch.cuda.synchronize()
    print(json.dumps(dict(probe="32x32x32x64", prec=prec, sap_applications=n_sap, sap_mode=0,
                          dslash_launches=n_d, copies=n_copy, copy_bytes=n)), flush=True)


def headline(cs, synth, torch, steps, warmup, cache_dir):
    """The metric's configuration: time-to-1e-10 on 32^3 x 64, mixed FP32 vs
    FP64-only, the SAP and operator rooflines, the copy reference, and the
    FP16 / BF16 smoothers."""
    import numpy as np

    import oracle
    c = synth.CONFIGS["lowprec_32x32x32x64"]
    dims = c["dims"]
    log(f"[bench] generating the {dims} gauge field and source")
    U, b = cached_field(synth, c, cache_dir)
    lat = cs.Lattice(dims)
    V = lat.volume
    op = cs.Operator(lat, torch.from_numpy(U).cuda(), c["kappa"], c["csw"])
    bd = lat.import_field(torch.from_numpy(b).cuda(), cs.F64)
    xd = lat.new_field(cs.F64)
    mixed = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32, restart=16, n_cy=2, n_mr=4, tol=1e-10)
    fp64 = cs.SolverParams(inner_prec=cs.F64, basis_prec=cs.F64, restart=16, n_cy=2, n_mr=4, tol=1e-10)

    log(f"[bench] warmup {warmup}")
    for _ in range(max(1, warmup)):
        xd.zero_()
        op.gcr_solve(xd, bd, mixed)
    torch.cuda.synchronize()
    log(f"[bench] timing {steps} mixed-precision solves")
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        xd.zero_()
        _, stats = op.gcr_solve(xd, bd, mixed)
        iters.append(stats[0]["iters"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) / steps * 1e3
    x_gpu = lat.export_field(xd, cs.F64).cpu().numpy()
    oracle.set_threads(min(16, len(os.sched_getaffinity(0))))
    rel_or = oracle.residual_norm(dims, U, c["kappa"], c["csw"], b, x_gpu) / np.linalg.norm(b)
    del x_gpu

    # The same solve again with HIP events around every kernel launch on the
    # stream it runs on (events cannot sit inside the replayed graphs, so
    # this pass runs the kernels eagerly).
    log("[bench] profiled pass")
    cs.profile_reset()
    cs.profile_enable(True)
    tp0 = time.perf_counter()
    xd.zero_()
    op.gcr_solve(xd, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32, use_graph=False))
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    cs.profile_enable(False)
    fam = {k: cs.profile_query(k) for k in ("sap_halfsweep", "sap_general", "sap_from_zero", "dslash", "blas")}
    n_gen, ms_gen = fam["sap_general"]
    sap_us = ms_gen / n_gen * 1e3
    sap_bytes = SAP_BYTES_F32[0] * V / 2
    achieved = sap_bytes / (sap_us * 1e-6) / 1e9
    sap_flops = SAP_FLOPS[0] * V / 2
    n_d, ms_d = fam["dslash"]
    d_us_solve = ms_d / n_d * 1e3

    log("[bench] copy reference and operator launches")
    copy = copy_bandwidth(cs, torch)
    b32 = lat.import_field(torch.from_numpy(b).cuda(), cs.F32)
    o32 = lat.new_field(cs.F32)
    d_us = timed_events(torch, lambda: op.apply_D(o32, b32, cs.F32), 20)
    d_gbs = DSLASH_BYTES_F32 * V / (d_us * 1e-6) / 1e9
    x32 = lat.import_field(torch.from_numpy(b).cuda(), cs.F32)
    app_us = timed_events(torch, lambda: op.sap_smooth(x32, b32, cs.F32, n_cy=2, n_mr=4, x0_is_zero=False), 5)
    del b32, o32, x32

    roofline = dict(
        bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
        frac=round(achieved / HBM_PEAK_GBS, 4),
        traffic=load_traffic("sap_halfsweep_32x32x32x64", SAP_KERNEL_SOURCES),
        kernel="k_sap_halfsweep<1, 1, 0, true> (FP32, one lane per site, general visits: x nonzero)",
        lattice="32x32x32x64", avg_launch_us=round(sap_us, 2), launches=n_gen,
        alg_bytes_per_launch=int(sap_bytes), alg_bytes_per_visited_site=SAP_BYTES_F32[0],
        visited_sites_per_launch=V // 2,
        frac_of_copy=round(achieved / copy["GBps"], 4),
        alu=dict(achieved=round(sap_flops / (sap_us * 1e-6) / 1e12, 2), peak=round(FP32_VALU_PEAK_TFLOPS, 1),
                 unit="TFLOP/s", frac=round(sap_flops / (sap_us * 1e-6) / 1e12 / FP32_VALU_PEAK_TFLOPS, 4),
                 flops_per_visited_site=SAP_FLOPS[0]),
        note=("average duration of the general (mode 0) half-sweeps, HIP events around every launch in an "
              "eager pass of the timed solve; traffic = FETCH_SIZE x 2 + WRITE_SIZE per launch from the "
              "committed counter record (null when the kernel sources changed since)"))

    log("[bench] FP64-only GPU solves")
    fp64_s, fp64_it, fp64_st = time_gcr(cs, torch, op, xd, bd, fp64, 2)
    lowp = {}
    for name, inner in (("f16", cs.F16), ("bf16", cs.BF16)):
        log(f"[bench] {name} smoother solves")
        t, it, st = time_gcr(cs, torch, op, xd, bd, cs.SolverParams(inner_prec=inner, basis_prec=cs.F32), 2)
        lowp[name] = dict(time_to_1e10_ms=round(t * 1e3, 2), iterations=it, status=st,
                          speedup_vs_fp64=round(fp64_s / t, 3))
    del op, bd, xd
    torch.cuda.empty_cache()
    out = dict(metric=METRIC, value=round(steps / (t1 - t0), 4), unit="solves/s",
               n_gpus=1, steps=steps, warmup=warmup, ms_per_step=round(ms_per_step, 3),
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32/f64",
               data="synthetic",
               config=dict(workload=("mixed_32x32x32x64: SAP(2 cycles x 4 MR, 4^4 blocks, FP32)-preconditioned "
                                     "FP64 flexible GCR(16) to a true relative residual of 1e-10, HIP-graph replay"),
                           lattice="32x32x32x64", eps=c["eps"], kappa=c["kappa"], csw=c["csw"],
                           gauge_seed=c["gauge_seed"], source_seed=c["src_seed"]),
               time_to_1e10_ms=round(ms_per_step, 2), iterations=int(np.median(iters)),
               fp64_time_to_1e10_ms=round(fp64_s * 1e3, 2), fp64_iterations=fp64_it, fp64_status=fp64_st,
               speedup_mixed_vs_fp64=round(fp64_s * 1e3 / ms_per_step, 3),
               oracle_checked_relres=float(f"{rel_or:.3e}"),
               low_precision_smoothers=lowp,
               dslash=dict(kernel="FP32 operator, one launch", avg_us=round(d_us, 2), GBps=round(d_gbs, 1),
                           frac_hbm_peak=round(d_gbs / HBM_PEAK_GBS, 4), frac_of_copy=round(d_gbs / copy["GBps"], 4),
                           alg_bytes_per_site=DSLASH_BYTES_F32, avg_us_in_solve=round(d_us_solve, 2),
                           traffic=load_traffic("dslash_32x32x32x64", DSLASH_KERNEL_SOURCES)),
               sap_application=dict(avg_us=round(app_us, 1),
                                    GBps=round(4 * sap_bytes / (app_us * 1e-6) / 1e9, 1),
                                    note="2 cycles of 4 MR steps from a nonzero x (four general half-sweeps)"),
               copy_reference=copy,
               kernels_in_profiled_solve={k: dict(launches=v[0], total_ms=round(v[1], 3),
                                                  avg_us=round(v[1] / max(v[0], 1) * 1e3, 2))
                                          for k, v in fam.items()},
               profiled_solve_ms=round((tp1 - tp0) * 1e3, 2),
               roofline=roofline)
    return out, (U, b, c)


def cache_resident_16(cs, synth, torch, reps=10):
    """The 16^3 x 32 system (working set inside the 256 MB last-level cache):
    mixed and FP64-only time to 1e-10."""
    c = synth.CONFIGS["mixed_16x16x16x32"]
    dims = c["dims"]
    U = synth.gauge_field(dims, c["eps"], c["gauge_seed"])
    b = synth.source(dims, c["src_seed"])
    lat = cs.Lattice(dims)
    op = cs.Operator(lat, torch.from_numpy(U).cuda(), c["kappa"], c["csw"])
    bd = lat.import_field(torch.from_numpy(b).cuda(), cs.F64)
    xd = lat.new_field(cs.F64)
    tm, itm, stm = time_gcr(cs, torch, op, xd, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32), reps)
    t64, it64, st64 = time_gcr(cs, torch, op, xd, bd, cs.SolverParams(inner_prec=cs.F64, basis_prec=cs.F64), reps)
    return dict(lattice="16x16x16x32", eps=c["eps"], kappa=c["kappa"], csw=c["csw"],
                mixed_time_to_1e10_ms=round(tm * 1e3, 3), mixed_iterations=itm, mixed_status=stm,
                fp64_time_to_1e10_ms=round(t64 * 1e3, 3), fp64_iterations=it64, fp64_status=st64,
                speedup_mixed_vs_fp64=round(t64 / tm, 3),
                note="cache-resident: the working set fits the 256 MB last-level cache; no HBM fraction quoted")


def solver_variants(cs, synth, torch, U, b, c):
    """The smoother and outer-solver variants and the two-level multigrid
    preconditioner on the 32^3 x 64 system."""
    import numpy as np

    import oracle
    dims = c["dims"]
    lat = cs.Lattice(dims)
    op = cs.Operator(lat, torch.from_numpy(U).cuda(), c["kappa"], c["csw"])
    bd = lat.import_field(torch.from_numpy(b).cuda(), cs.F64)
    xd = lat.new_field(cs.F64)
    res = {}
    t, it, st = time_bicgstab(cs, torch, op, xd, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F64), 1)
    res["fbicgstab_f32_smoother"] = dict(time_to_1e10_ms=round(t * 1e3, 2), iterations=it, status=st)
    t, it, st = time_bicgstab(cs, torch, op, xd, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32), 1)
    res["sp_bicgstab_in_fp64_richardson"] = dict(time_to_1e10_ms=round(t * 1e3, 2), iterations=it, status=st)
    t, it, st = time_gcr(cs, torch, op, xd, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32,
                                                                block_solver=1), 1)
    res["fgcr_jacobi_smoother"] = dict(time_to_1e10_ms=round(t * 1e3, 2), iterations=it, status=st)
    t, it, st = time_gcr(cs, torch, op, xd, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32,
                                                                block_solver=2), 1)
    res["fgcr_even_odd_block_mr"] = dict(time_to_1e10_ms=round(t * 1e3, 2), iterations=it, status=st)
    # the Krylov basis w_k stored in 16 bits with one scale per site (FP64
    # orthogonalisation arithmetic); an early restart at a 1e-3 drop of the
    # recursive residual keeps it within the storage accuracy
    for name, bp in (("fgcr_f16_krylov_basis", cs.F16), ("fgcr_bf16_krylov_basis", cs.BF16)):
        p16 = cs.SolverParams(inner_prec=cs.F32, basis_prec=bp, reliable_delta=1e-3)
        t, it, st = time_gcr(cs, torch, op, xd, bd, p16, 3)
        x = lat.export_field(xd, cs.F64).cpu().numpy()
        rr = oracle.residual_norm(dims, U, c["kappa"], c["csw"], b, x) / float(np.linalg.norm(b))
        res[name] = dict(time_to_1e10_ms=round(t * 1e3, 2), iterations=it, status=st,
                         oracle_checked_relres=float(f"{rr:.3e}"))
    t, it, st = time_gcr(cs, torch, op, xd, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32), 1)
    log("[bench] 32^3x64 two-level multigrid")
    res["multigrid"] = multigrid_measurement(cs, synth, torch, op, lat, c, U, b, bd, xd, t, it)
    del op, bd, xd
    torch.cuda.empty_cache()
    return res


def mfma_probe(cs, torch, nsites=1 << 21, reps=1024):
    """The batched link x half-spinor product (8 right-hand sides, 16 complex
    columns per link) chained in registers: FP32 vector arithmetic against
    the bfloat16 matrix cores (cs_probe_link_product).  Unitary links keep
    the chain bounded.  Per-step time = (t(1 + reps) - t(1)) / reps, so the
    loads and stores drop out."""
    g = torch.Generator(device="cuda").manual_seed(77)
    z = torch.randn(nsites, 2, 3, dtype=torch.complex64, device="cuda", generator=g)
    r0 = z[:, 0] / z[:, 0].norm(dim=1, keepdim=True)
    r1 = z[:, 1] - (r0.conj() * z[:, 1]).sum(dim=1, keepdim=True) * r0
    r1 = r1 / r1.norm(dim=1, keepdim=True)
    r2 = torch.linalg.cross(r0, r1).conj()
    U = torch.view_as_real(torch.stack([r0, r1, r2], dim=1).contiguous()).reshape(nsites, 9, 2).contiguous()
    del z, r0, r1, r2
    h = torch.randn(nsites, 16, 3, dtype=torch.complex64, device="cuda", generator=g)
    H = torch.view_as_real(h).reshape(nsites, 16, 3, 2).contiguous()
    V0 = torch.empty_like(H)
    V1 = torch.empty_like(H)
    res = dict(nsites=nsites, columns=16, reps=reps,
               useful_flops_per_step=nsites * 16 * 72)
    cs.probe_link_product(0, U, H, V0, 1)
    cs.probe_link_product(1, U, H, V1, 1)
    torch.cuda.synchronize()
    res["mfma_vs_valu_rel_diff_one_step"] = float(f"{float((V1 - V0).norm() / V0.norm()):.3e}")
    cs.probe_link_product(0, U, H, V0, 8)
    cs.probe_link_product(1, U, H, V1, 8)
    torch.cuda.synchronize()
    res["mfma_vs_valu_rel_diff_eight_steps"] = float(f"{float((V1 - V0).norm() / V0.norm()):.3e}")
    for kind, name in ((0, "valu_f32"), (1, "mfma_bf16")):
        log(f"[mfma-probe] {name}")
        t1 = timed_events(torch, lambda: cs.probe_link_product(kind, U, H, V0, 1), 3)
        tr = timed_events(torch, lambda: cs.probe_link_product(kind, U, H, V0, 1 + reps), 3)
        step = (tr - t1) / reps
        res[name] = dict(one_step_us=round(t1, 1), per_step_us=round(step, 2),
                         useful_TFLOPs=round(nsites * 16 * 72 / (step * 1e-6) / 1e12, 2))
    res["mfma_speedup_per_step"] = round(res["valu_f32"]["per_step_us"] / res["mfma_bf16"]["per_step_us"], 2)
    return res


# Side measurements that --only runs alone (the 32^3x64 variants take the
# headline's field, generated or read from --field-cache).
LEGS = {
    "cache_resident_16x16x16x32": cache_resident_16,
    "variants_32x32x32x64": None,
    "lowprec_sub_16x16x16x16": lowprec_subrun,
    "multirhs_24x24x24x48": multirhs_measurement,
    "grad_32x32x32x64": gradient_measurement,
    "next_rows": next_rows,
}


# The contract's fields first, then the mixed-vs-FP64 comparison, the
# roofline and CPU baseline objects, and after them the headline details and
# the side measurements (readers that keep only the start of the line still
# see all of these).
FRONT_KEYS = ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "time_to_1e10_ms", "iterations",
              "fp64_time_to_1e10_ms", "fp64_iterations", "fp64_status", "speedup_mixed_vs_fp64",
              "oracle_checked_relres", "roofline", "cpu_baseline"]


def ordered_line(out: dict) -> dict:
    return {**{k: out[k] for k in FRONT_KEYS if k in out}, **{k: v for k, v in out.items() if k not in FRONT_KEYS}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the side measurements (cache-resident lattice, low-precision sub-run, multi-RHS, "
                         "gradient, solver variants and multigrid)")
    ap.add_argument("--paper-comparisons", action="store_true",
                    help="also run the kappa scan towards the critical mass and the one/twelve-equation costs "
                         "with the multigrid setup (the shape of the paper's comparisons; off by default)")
    ap.add_argument("--field-cache", default="",
                    help="directory in which generated gauge fields are kept between runs")
    ap.add_argument("--probe32", action="store_true",
                    help="only mode-0 SAP applications, operator launches and device copies on the "
                         "32^3x64 field (a short run for kernel-trace and hardware-counter passes)")
    ap.add_argument("--probe-prec", default="f32", choices=["f64", "f32", "f16", "bf16"])
    ap.add_argument("--only", choices=sorted(LEGS),
                    help="only one side measurement (no headline, no CPU baseline): a short run for "
                         "kernel-trace and hardware-counter passes")
    ap.add_argument("--mfma-probe", action="store_true",
                    help="only the link x half-spinor product probe: FP32 vector arithmetic against the "
                         "bfloat16 matrix cores")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not an implementation", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2112_00501_amd import cloversap as cs
    from paper_2112_00501_amd import synth

    import oracle
    # the oracle built for this host's CPU (same arithmetic as the generic
    # build: no contraction, no reordering), for the residual checks and the
    # CPU baseline
    oracle.use_native_build()

    if args.probe32:
        probe32(cs, synth, torch, cs.PREC[args.probe_prec], args.field_cache)
        return
    if args.mfma_probe:
        print(json.dumps(dict(link_product_probe=mfma_probe(cs, torch))), flush=True)
        return
    if args.only:
        log(f"[bench] only {args.only}")
        if args.only == "variants_32x32x32x64":
            c = synth.CONFIGS["lowprec_32x32x32x64"]
            U, b = cached_field(synth, c, args.field_cache)
            res = solver_variants(cs, synth, torch, U, b, c)
        else:
            res = LEGS[args.only](cs, synth, torch)
        print(json.dumps({args.only: res}), flush=True)
        return

    out, (U, b, c) = headline(cs, synth, torch, args.steps, args.warmup, args.field_cache)
    torch.cuda.empty_cache()
    if not args.no_extras:
        log("[bench] 16^3x32 cache-resident solves")
        out["cache_resident_16x16x16x32"] = cache_resident_16(cs, synth, torch)
        log("[bench] 32^3x64 solver variants and multigrid")
        out["variants_32x32x32x64"] = solver_variants(cs, synth, torch, U, b, c)
        log("[bench] 16^4 low-precision sub-run against the oracle")
        out["lowprec_sub_16x16x16x16"] = lowprec_subrun(cs, synth, torch)
        log("[bench] 24 right-hand sides on 24^3x48")
        out["multirhs_24x24x24x48"] = multirhs_measurement(cs, synth, torch)
        torch.cuda.empty_cache()
        log("[bench] gradient on 32^3x64")
        out["grad_32x32x32x64"] = gradient_measurement(cs, synth, torch)
        torch.cuda.empty_cache()
        log("[bench] next rows on 16^3x32 and 8^4 (the oracle's timings of the same work: cpu_baseline)")
        out["next_rows"] = next_rows(cs, synth, torch)
    if args.paper_comparisons:
        log("[bench] kappa scan towards the critical mass, SAP-FGCR vs MG-FGCR")
        out["kappa_scan_32x32x32x64"] = kappa_scan(cs, synth, torch, cs.Lattice(c["dims"]), c, U, b)
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cs16 = synth.CONFIGS["mixed_16x16x16x32"]
        small = (synth.gauge_field(cs16["dims"], cs16["eps"], cs16["gauge_seed"]),
                 synth.source(cs16["dims"], cs16["src_seed"]), cs16)
        out["cpu_baseline"] = cpu_baseline(U, b, c, out["fp64_iterations"], small)
    print(json.dumps(ordered_line(out)), flush=True)


if __name__ == "__main__":
    main()
