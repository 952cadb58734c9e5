"""Benchmark: mixed-precision SAP-preconditioned flexible GCR on one MI355X.

One step = one solve of D x = b to a true relative residual of 1e-10 on the
16^3 x 32 synthetic gauge field (eps 0.3, kappa 0.1355, c_sw 1.0): FP32 SAP
smoother (2 red/black cycles of 4 MR steps on 4^4 blocks) and FP32 w = D z
inside an FP64 flexible GCR(16) with FP64 residual recomputation.  b is
resident in HBM and x starts at zero.

Prints one JSON line.  Besides the timed steps it reports the FP64-only GPU
solve of the same system (mixed vs FP64), the roofline of the dominant kernel
from HIP events recorded around every launch in the timed region, HBM
bandwidth of the operator and the smoother on the HBM-resident 32^3 x 64
lattice, and the FP64 CPU oracle timed on the host as a reference.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Dslash/SAP HBM GB/s (% peak); time-to-1e-10 residual, mixed vs FP64, 1 GPU"
SAP_KERNEL_SOURCES = ["sap.hip", "sap_pair.hip", "dslash_core.hpp", "fields.hpp", "cs_internal.hpp", "wave.hpp"]

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
# FP32 vector peak without packed FP32 instructions (this library disables
# them): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.
FP32_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2112_00501_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, per_launch_alg_bytes: float):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash(SAP_KERNEL_SOURCES):
        return None
    return rec.get("hbm_bytes_per_launch")


def sap_kernel_name(nblk: int) -> str:
    """The FP32 SAP kernel the library launches by default: the lane-pair
    kernel while a colour has at most 256 blocks (one per compute unit)."""
    return "k_sap_pair<f32>" if nblk // 2 <= 256 else "k_sap_halfsweep<f32>"


def sap_flops_per_application(V: int, n_cy: int) -> float:
    """Flops of one SAP application from x = 0 (the four half-sweep modes of
    n_cy = 2: 1, 2, then 0, 0), V / 2 sites per half-sweep."""
    return V / 2 * (SAP_FLOPS[1] + SAP_FLOPS[2] + (2 * n_cy - 2) * SAP_FLOPS[0])


def sap_bytes_per_application(V: int, n_cy: int) -> float:
    modes = [1, 2] + [0, 0] * (n_cy - 1)
    return sum(SAP_BYTES_F32[m] for m in modes) * V / 2


def cpu_baseline(dims, U, b, kappa, csw):
    import numpy as np

    import oracle
    threads = min(16, len(os.sched_getaffinity(0)))
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    T = oracle.clover_field(dims, U, kappa, csw)
    t1 = time.perf_counter()
    x, st, it, rel, _ = oracle.fgcr(dims, (4, 4, 4, 4), U, T, kappa, b, n_cy=2, n_mr=4,
                                    restart=16, tol=1e-10)
    t2 = time.perf_counter()
    return dict(value=1.0 / (t2 - t1), unit="solves/s", cores=threads, kind="oracle",
                sample=(f"one complete FP64 SAP-FGCR(16) solve of the same "
                        f"{'x'.join(map(str, dims))} field and source to 1e-10 by the plain-C "
                        f"oracle ({it} iterations, status {st}, true relres {rel:.2e}); "
                        f"clover build ({t1 - t0:.2f} s) excluded like on the GPU"),
                seconds=t2 - t1, iterations=it), x


def hbm_resident_measurement(cs, synth, torch, reps_d=20, reps_sap=10):
    """Dslash and SAP bandwidth on 32^3 x 64 (working set far above the
    256 MB last-level cache), FP32 storage, HIP events per launch; then
    time-to-1e-10 for the FP32, FP16 and BF16 smoothers and the FP64-only
    solve on the same field (low-precision storage: iteration penalty)."""
    import numpy as np
    c = synth.CONFIGS["lowprec_32x32x32x64"]
    dims = c["dims"]
    U = synth.gauge_field(dims, c["eps"], c["gauge_seed"])
    b = synth.source(dims, c["src_seed"])
    lat = cs.Lattice(dims)
    op = cs.Operator(lat, torch.from_numpy(U).cuda(), c["kappa"], c["csw"])
    V = lat.volume
    bin32 = lat.import_field(torch.from_numpy(b).cuda(), cs.F32)
    out32 = lat.new_field(cs.F32)
    for _ in range(3):
        op.apply_D(out32, bin32, cs.F32)
        op.sap_smooth(out32, bin32, cs.F32)
    torch.cuda.synchronize()
    cs.profile_reset()
    cs.profile_enable(True)
    for _ in range(reps_d):
        op.apply_D(out32, bin32, cs.F32)
    for _ in range(reps_sap):
        op.sap_smooth(out32, bin32, cs.F32, n_cy=2, n_mr=4)
    torch.cuda.synchronize()
    cs.profile_enable(False)
    nd, msd = cs.profile_query("dslash")
    ns, mss = cs.profile_query("sap_halfsweep")
    d_us = msd / nd * 1e3
    sap_app_us = mss / reps_sap * 1e3
    d_gbs = DSLASH_BYTES_F32 * V / (d_us * 1e-6) / 1e9
    s_gbs = sap_bytes_per_application(V, 2) / (sap_app_us * 1e-6) / 1e9
    res = dict(lattice="32x32x32x64", eps=c["eps"], kappa=c["kappa"], csw=c["csw"], storage="f32",
               dslash_us=round(d_us, 2), dslash_GBps=round(d_gbs, 1),
               dslash_frac_hbm_peak=round(d_gbs / HBM_PEAK_GBS, 4),
               sap_application_us=round(sap_app_us, 2), sap_GBps=round(s_gbs, 1),
               sap_frac_hbm_peak=round(s_gbs / HBM_PEAK_GBS, 4))
    del bin32, out32
    bd = lat.import_field(torch.from_numpy(b).cuda(), cs.F64)
    xd = lat.new_field(cs.F64)
    import oracle
    for name, inner, basis in (("mixed_f32", cs.F32, cs.F32), ("mixed_f16", cs.F16, cs.F32),
                               ("mixed_bf16", cs.BF16, cs.F32), ("fp64", cs.F64, cs.F64)):
        p = cs.SolverParams(inner_prec=inner, basis_prec=basis)
        xd.zero_()
        op.gcr_solve(xd, bd, p, allow_fail=True)  # warm-up (workspace, graphs)
        xd.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, stats = op.gcr_solve(xd, bd, p, allow_fail=True)
        torch.cuda.synchronize()
        res[f"{name}_time_to_1e-10_s"] = round(time.perf_counter() - t, 4)
        res[f"{name}_iterations"] = stats[0]["iters"]
        res[f"{name}_status"] = st
        if name == "mixed_f32":
            x = lat.export_field(xd, cs.F64).cpu().numpy()
            res["mixed_f32_oracle_checked_relres"] = float(
                f"{oracle.residual_norm(dims, U, c['kappa'], c['csw'], b, x) / np.linalg.norm(b):.3e}")
    res["speedup_mixed_f32_vs_fp64"] = round(res["fp64_time_to_1e-10_s"] / res["mixed_f32_time_to_1e-10_s"], 3)
    # the paper's outer solver, flexible BiCGStab, with the same FP32 smoother
    t, it, st = time_bicgstab(cs, torch, op, xd, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F64), 1)
    res["fbicgstab_mixed_f32_time_to_1e-10_s"] = round(t, 4)
    res["fbicgstab_mixed_f32_iterations"] = it
    res["fbicgstab_mixed_f32_status"] = st
    t, it, st = time_bicgstab(cs, torch, op, xd, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32), 1)
    res["sp_bicgstab_richardson_f32_time_to_1e-10_s"] = round(t, 4)
    res["sp_bicgstab_richardson_f32_iterations"] = it
    res["sp_bicgstab_richardson_f32_status"] = st
    # FGCR with the even-odd block solver in the smoother
    t, it, st = time_gcr(cs, torch, op, xd, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32,
                                                                 block_solver=2), 1)
    res["eo_smoother_f32_time_to_1e-10_s"] = round(t, 4)
    res["eo_smoother_f32_iterations"] = it
    res["eo_smoother_f32_status"] = st
    # SAP-FGCR again right before the multigrid runs (median of 3), then MG
    t, it, st = time_gcr(cs, torch, op, xd, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32), 3)
    log("[bench] 32^3x64 two-level multigrid")
    res["multigrid"] = multigrid_measurement(cs, synth, torch, op, lat, c, U, b, bd, xd, t, it)
    log("[bench] 32^3x64 two-level multigrid, FP16 coarse matrices and prolongator")
    res["multigrid_f16_storage"] = multigrid_measurement(cs, synth, torch, op, lat, c, U, b, bd, xd, t, it,
                                                         half=True)
    del op, bd, xd
    torch.cuda.empty_cache()
    log("[bench] 32^3x64 kappa scan towards the critical mass, SAP-FGCR vs MG-FGCR")
    res["kappa_scan"] = kappa_scan(cs, synth, torch, lat, c, U, b)
    return res


# Two-level multigrid of the paper's Section 3: N_vec = 16 null vectors from
# SAP-smoothed random vectors and 4 adaptive passes, coarse BiCGStab to 5%
# (at most 50 iterations), 2 SAP post-smoothing cycles of 4 MR steps.
MG_PARAMS = dict(nv=16, n_cy_setup=4, n_mr=4, n_adapt=4, n_coarse=50, n_cy_post=2, tol_coarse=0.05)


def multigrid_measurement(cs, synth, torch, op, lat, c, U, b, bd, xd, sap_s, sap_it, reps=3, half=False):
    """MG-preconditioned FGCR to 1e-10 on the same system as SAP-FGCR:
    setup time, solve time (median of reps), iterations, per-family kernel
    time of one solve, and the paper's comparison of one and of twelve
    equations with the setup included."""
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
                one_equation_incl_setup_s=round(setup_s + solve_s, 4),
                twelve_equations_incl_setup_s=round(setup_s + 12 * solve_s, 4),
                twelve_equations_sap_fgcr_s=round(12 * sap_s, 4),
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
    time to 1e-10 for all 24 (batched, graph-replayed) against 24 one-by-one
    solves."""
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
    return res


def gradient_measurement(cs, synth, torch):
    """Forward solve and backward pass (adjoint solve + force) of
    L = Re(eta^dag D^-1 b) on 32^3 x 64 through torch.autograd."""
    import numpy as np
    c = synth.CONFIGS["grad_32x32x32x64"]
    dims = c["dims"]
    U = torch.from_numpy(synth.gauge_field(dims, c["eps"], c["gauge_seed"])).cuda().requires_grad_(True)
    b = torch.from_numpy(synth.source(dims, c["src_seed"])).cuda().requires_grad_(True)
    eta = torch.from_numpy(synth.source(dims, c["eta_seed"])).cuda()
    lat = cs.Lattice(dims)
    params = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x = cs.CloverSolve.apply(U, b, lat, c["kappa"], c["csw"], params)
    L = (torch.conj(eta) * x).sum().real
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    gn = float(U.grad.abs().max())
    return dict(lattice="32x32x32x64", forward_s=round(t1 - t0, 4), backward_s=round(t2 - t1, 4),
                note="forward includes gauge import and clover build; backward = adjoint solve + force",
                grad_U_maxabs=float(f"{gn:.4e}"), loss=float(f"{float(L):.6e}"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hbm", action="store_true", help="skip the 32^3x64 side measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the low-precision, multi-RHS and gradient side measurements")
    ap.add_argument("--hbm-only", action="store_true",
                    help="only the 32^3x64 HBM-resident operator, smoother and solve measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of 1 GiB five times (counter calibration)")
    ap.add_argument("--sap-probe", action="store_true",
                    help="only 10 FP32 SAP applications and 10 FP32 operator launches on the 16^3x32 "
                         "benchmark field (a short run for hardware-counter passes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not an implementation", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        c = torch.empty_like(a)
        for _ in range(5):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes=n, copies=5)), flush=True)
        return

    from paper_2112_00501_amd import cloversap as cs
    from paper_2112_00501_amd import synth

    if args.sap_probe:
        cfg = synth.CONFIGS["mixed_16x16x16x32"]
        dims = cfg["dims"]
        lat = cs.Lattice(dims)
        op = cs.Operator(lat, torch.from_numpy(synth.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])).cuda(),
                         cfg["kappa"], cfg["csw"])
        b32 = lat.import_field(torch.from_numpy(synth.source(dims, cfg["src_seed"])).cuda(), cs.F32)
        x32 = lat.new_field(cs.F32)
        for _ in range(10):
            op.sap_smooth(x32, b32, cs.F32, n_cy=2, n_mr=4)
            op.apply_D(x32, b32, cs.F32)
        torch.cuda.synchronize()
        print(json.dumps(dict(sap_applications=10, dslash_launches=10, lattice="16x16x16x32")), flush=True)
        return

    if args.hbm_only:
        log("[bench] 32^3x64 HBM-resident measurement")
        print(json.dumps(dict(hbm_resident_32x32x32x64=hbm_resident_measurement(cs, synth, torch))), flush=True)
        return

    cfg = synth.CONFIGS["mixed_16x16x16x32"]
    dims, kappa, csw = cfg["dims"], cfg["kappa"], cfg["csw"]
    log(f"[bench] generating {dims} gauge field and source")
    U = synth.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    b = synth.source(dims, cfg["src_seed"])
    lat = cs.Lattice(dims)
    V = lat.volume
    op = cs.Operator(lat, torch.from_numpy(U).cuda(), kappa, csw)
    bd = lat.import_field(torch.from_numpy(b).cuda(), cs.F64)
    xd = lat.new_field(cs.F64)
    mixed = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32, restart=16, n_cy=2, n_mr=4,
                            tol=1e-10)
    fp64 = cs.SolverParams(inner_prec=cs.F64, basis_prec=cs.F64, restart=16, n_cy=2, n_mr=4,
                           tol=1e-10)

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        xd.zero_()
        op.gcr_solve(xd, bd, mixed)
    torch.cuda.synchronize()

    log(f"[bench] timing {args.steps} mixed-precision solves")
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        xd.zero_()
        _, stats = op.gcr_solve(xd, bd, mixed)
        iters.append(stats[0]["iters"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) / args.steps * 1e3
    x_gpu = lat.export_field(xd, cs.F64).cpu().numpy()

    # The same steps again with HIP events recorded around every kernel launch
    # on the stream it runs on (per-launch events cannot be placed inside the
    # captured graphs of the timed pass, so this pass runs the kernels eagerly).
    log(f"[bench] profiled pass of {args.steps} solves")
    cs.profile_reset()
    cs.profile_enable(True)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        xd.zero_()
        op.gcr_solve(xd, bd, mixed)
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    cs.profile_enable(False)
    fam = {k: cs.profile_query(k) for k in ("sap_halfsweep", "dslash", "blas")}

    # dominant kernel: the SAP half-sweep (largest summed time)
    n_sap, ms_sap = fam["sap_halfsweep"]
    n_apps = n_sap // 4
    alg_bytes = sap_bytes_per_application(V, 2) * n_apps
    per_launch_bytes = alg_bytes / n_sap
    avg_us = ms_sap / n_sap * 1e3
    achieved = per_launch_bytes / (avg_us * 1e-6) / 1e9
    per_launch_flops = sap_flops_per_application(V, 2) * n_apps / n_sap
    alu_tflops = per_launch_flops / (avg_us * 1e-6) / 1e12
    dominant = max(fam, key=lambda k: fam[k][1])
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=load_traffic("sap_halfsweep_16x16x16x32", per_launch_bytes),
                    kernel=sap_kernel_name(V // 256), avg_launch_us=round(avg_us, 2),
                    alg_bytes_per_launch=int(per_launch_bytes), launches=n_sap,
                    dominant_by_time=dominant,
                    profiled_pass_ms_per_step=round((tp1 - tp0) / args.steps * 1e3, 3),
                    alu=dict(achieved=round(alu_tflops, 2), peak=round(FP32_VALU_PEAK_TFLOPS, 1),
                             unit="TFLOP/s", frac=round(alu_tflops / FP32_VALU_PEAK_TFLOPS, 4),
                             flops_per_launch=int(per_launch_flops),
                             note="FP32 vector arithmetic without packed FP32; at this lattice the "
                                  "half-sweep is bound by instruction issue, not by HBM"),
                    note=("kernel durations from HIP events around every launch in a profiled pass of "
                          "the same steps (eager); working set ~90 MB fits the 256 MB last-level cache "
                          "at this lattice; the HBM-resident figure is hbm_resident_32x32x32x64.sap_GBps"))

    log("[bench] FP64-only GPU solves")
    fp64_times, fp64_iters = [], []
    for _ in range(4):
        xd.zero_()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        _, st64 = op.gcr_solve(xd, bd, fp64)
        torch.cuda.synchronize()
        fp64_times.append(time.perf_counter() - ta)
        fp64_iters.append(st64[0]["iters"])
    fp64_ms = float(np.median(fp64_times[1:])) * 1e3

    log("[bench] flexible BiCGStab solves")
    bi64 = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F64, n_cy=2, n_mr=4, tol=1e-10)
    bi_s, bi_it, bi_st = time_bicgstab(cs, torch, op, xd, bd, bi64, 5)
    x_bi = lat.export_field(xd, cs.F64).cpu().numpy()
    bi32 = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32, n_cy=2, n_mr=4, tol=1e-10)
    sp_s, sp_it, sp_st = time_bicgstab(cs, torch, op, xd, bd, bi32, 5)
    x_sp = lat.export_field(xd, cs.F64).cpu().numpy()
    log("[bench] solves with the Jacobi smoother on C^-1 D")
    jac_gcr = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32, n_cy=2, n_mr=4, tol=1e-10, block_solver=1)
    jg_s, jg_it, jg_st = time_gcr(cs, torch, op, xd, bd, jac_gcr, 5)
    jq_s, jq_it, jq_st = time_bicgstab(cs, torch, op, xd, bd, cs.SolverParams(
        inner_prec=cs.F32, basis_prec=cs.F32, n_cy=2, n_mr=4, tol=1e-10, block_solver=1), 5)
    log("[bench] solves with even-odd preconditioned block MR")
    eo_gcr = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32, n_cy=2, n_mr=4, tol=1e-10, block_solver=2)
    eg_s, eg_it, eg_st = time_gcr(cs, torch, op, xd, bd, eo_gcr, 5)

    log("[bench] two-level multigrid on the same system")
    mg16 = multigrid_measurement(cs, synth, torch, op, lat, cfg, U, b, bd, xd, ms_per_step / 1e3,
                                 int(np.median(iters)), reps=5)

    import oracle
    rel_or = oracle.residual_norm(dims, U, kappa, csw, b, x_gpu) / np.linalg.norm(b)
    rel_bi = oracle.residual_norm(dims, U, kappa, csw, b, x_bi) / np.linalg.norm(b)
    rel_sp = oracle.residual_norm(dims, U, kappa, csw, b, x_sp) / np.linalg.norm(b)

    out = dict(metric=METRIC, value=round(args.steps / (t1 - t0), 3), unit="solves/s",
               n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_per_step, 3),
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32/f64",
               data="synthetic",
               config=dict(workload=("mixed_16x16x16x32: SAP(2 cycles x 4 MR, 4^4 blocks, FP32)-"
                                     "preconditioned FP64 flexible GCR(16) to 1e-10, HIP-graph replay"),
                           lattice="16x16x16x32", eps=cfg["eps"], kappa=kappa, csw=csw,
                           gauge_seed=cfg["gauge_seed"], source_seed=cfg["src_seed"]),
               time_to_1e10_ms=round(ms_per_step, 3), iterations=int(np.median(iters)),
               fp64_time_to_1e10_ms=round(fp64_ms, 3), fp64_iterations=int(np.median(fp64_iters)),
               speedup_mixed_vs_fp64=round(fp64_ms / ms_per_step, 3),
               oracle_checked_relres=float(f"{rel_or:.3e}"),
               fbicgstab=dict(time_to_1e10_ms=round(bi_s * 1e3, 3), iterations=bi_it, status=bi_st,
                              oracle_checked_relres=float(f"{rel_bi:.3e}"),
                              note="flexible BiCGStab (two SAP and two operator applications per "
                                   "iteration), same FP32 smoother, median of 5"),
               jacobi_smoother=dict(fgcr_time_to_1e10_ms=round(jg_s * 1e3, 3), fgcr_iterations=jg_it,
                                    fgcr_status=jg_st,
                                    sp_bicgstab_richardson_time_to_1e10_ms=round(jq_s * 1e3, 3),
                                    sp_bicgstab_richardson_iterations=jq_it, sp_bicgstab_richardson_status=jq_st,
                                    note="SAP on C^-1 D with 4 Jacobi steps per block (the QWS smoother form), "
                                         "FP32, median of 5"),
               eo_smoother=dict(fgcr_time_to_1e10_ms=round(eg_s * 1e3, 3), fgcr_iterations=eg_it, fgcr_status=eg_st,
                                note="SAP with 4 even-odd preconditioned MR steps per block (Schur complement on "
                                     "the even sites), FP32, one lane per site, median of 5"),
               sp_bicgstab_richardson=dict(time_to_1e10_ms=round(sp_s * 1e3, 3), iterations=sp_it, status=sp_st,
                                           oracle_checked_relres=float(f"{rel_sp:.3e}"),
                                           note="FP32-vector BiCGStab inner solves to 1e-5 inside an FP64 "
                                                "Richardson iteration, same FP32 smoother, median of 5"),
               multigrid=mg16,
               kernels={k: dict(launches=v[0], total_ms=round(v[1], 3),
                                avg_us=round(v[1] / max(v[0], 1) * 1e3, 2))
                        for k, v in fam.items()},
               roofline=roofline)
    del op, lat, bd, xd
    torch.cuda.empty_cache()
    if not args.no_hbm:
        log("[bench] 32^3x64 HBM-resident measurement")
        out["hbm_resident_32x32x32x64"] = hbm_resident_measurement(cs, synth, torch)
        torch.cuda.empty_cache()
    if not args.no_extras:
        log("[bench] 16^4 low-precision sub-run against the oracle")
        out["lowprec_sub_16x16x16x16"] = lowprec_subrun(cs, synth, torch)
        log("[bench] 24 right-hand sides on 24^3x48")
        out["multirhs_24x24x24x48"] = multirhs_measurement(cs, synth, torch)
        torch.cuda.empty_cache()
        log("[bench] gradient on 32^3x64")
        out["grad_32x32x32x64"] = gradient_measurement(cs, synth, torch)
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cb, _ = cpu_baseline(dims, U, b, kappa, csw)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
