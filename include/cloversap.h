/*
 * cloversap -- clover-Wilson Dirac operator, red/black SAP smoother and
 * flexible GCR for one AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Every function returns an int status (cs_status); no exception
 * crosses the boundary.  cs_last_error() gives a message for the last
 * failure on the calling thread.
 *
 * Objects
 *   cs_lattice  geometry and the 4^4 block decomposition (host object)
 *   cs_gauge    the links, stored on the device in compressed form (rows 0
 *               and 1 of each SU(3) matrix) in every storage precision
 *   cs_clover   C = 1 + T for one (kappa, c_sw), stored on the device as two
 *               6x6 Hermitian blocks per site
 * Handles are owned by the library and released with the matching destroy
 * call.  Spinor fields are caller-owned device buffers (for example torch
 * tensors) in the library's internal layout; cs_field_bytes() gives their
 * size and cs_field_import / cs_field_export convert from / to the
 * canonical layout below.
 *
 * Canonical layouts (complex double, interleaved re/im, site index x fastest:
 * s = x + Lx*(y + Ly*(z + Lz*t)), directions mu = 0..3 for x, y, z, t):
 *   links    U[V][4][3][3]            U_mu(x)[row][col], each exactly SU(3)
 *   spinor   psi[nrhs][V][4][3]       index 3*spin + colour
 *   clover   T[V][12][12]             the term T of C = 1 + T (export only)
 * Boundary conditions are periodic in all four directions for the links;
 * fermion fields are periodic too unless the lattice was created with
 * CS_ANTIPERIODIC_T (antiperiodic in time).  Gamma matrices
 * are those of the chiral basis with gamma5 = diag(1, 1, -1, -1):
 *   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = x, y, z),
 *   gamma_t = [[0, 1], [1, 0]].
 *
 * Streams: every call that takes a stream (a hipStream_t passed as void*,
 * NULL = the null stream) is asynchronous on it, except cs_gcr_solve, which
 * synchronises the stream for its convergence control and returns after the
 * solution is complete.  All pointers passed as field, link or result
 * arguments are device pointers unless stated otherwise.
 *
 * Precision (cs_prec) names the storage type of spinors and links in HBM:
 *   CS_F64   double spinors, links and clover; double arithmetic
 *   CS_F32   float spinors, links and clover; float arithmetic
 *   CS_F16   half spinors with one float scale per site, half links, float
 *            clover; float arithmetic
 *   CS_BF16  as CS_F16 with bfloat16 storage
 */
#ifndef CLOVERSAP_H
#define CLOVERSAP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CS_OK = 0,
    CS_ERR_INVALID = -1,    /* bad argument value                              */
    CS_ERR_GEOMETRY = -2,   /* dims not multiples of 4, or an odd block count  */
    CS_ERR_NULL = -3,       /* a required pointer or handle is NULL            */
    CS_ERR_PRECISION = -4,  /* precision not supported by this call            */
    CS_ERR_HIP = -5,        /* a HIP runtime call failed                       */
    CS_ERR_ALLOC = -6,      /* device memory allocation failed                 */
    CS_NOT_CONVERGED = 1,   /* solver stopped at max_iter                      */
    CS_BREAKDOWN = 2,       /* solver met a zero search direction              */
    CS_NONFINITE = 3        /* a NaN or Inf appeared in a residual norm        */
} cs_status;

typedef enum { CS_F64 = 0, CS_F32 = 1, CS_F16 = 2, CS_BF16 = 3 } cs_prec;

/* Lattice flags (cs_lattice_create). */
typedef enum {
    CS_PERIODIC = 0,       /* fermion fields periodic in all four directions */
    CS_ANTIPERIODIC_T = 1  /* fermion fields antiperiodic in time:
                              psi(x + Lt e_t) = -psi(x) */
} cs_lattice_flags;

typedef struct cs_lattice_s* cs_lattice;
typedef struct cs_gauge_s* cs_gauge;
typedef struct cs_clover_s* cs_clover;

/* Message for the last failing call on this thread ("" if none). */
const char* cs_last_error(void);
/* Short text for a status code. */
const char* cs_strerror(int status);

/* ---------------------------------------------------------------- geometry */

/* Lattice of dims[0..3] = (Lx, Ly, Lz, Lt) sites, cut into blocks of
 * block[0..3] sites.  The kernels require block = (4, 4, 4, 4) and every
 * extent a multiple of 4 (CS_ERR_GEOMETRY otherwise).  The red/black block
 * colouring of the SAP smoother (paper Section 2 and Section 3; colour of a
 * block = sum of its block coordinates mod 2) also needs an even number of
 * blocks in every direction; that is checked by the SAP and solver calls.
 * flags: CS_PERIODIC or CS_ANTIPERIODIC_T, the boundary condition of the
 * fermion fields in time (the paper does not state one).  With
 * CS_ANTIPERIODIC_T every hop of the operator of Eq. (1) that crosses the
 * time boundary changes sign, in D, D^dag, the smoothers, the solvers, the
 * multigrid operators and the force; the clover term is unaffected.  Other
 * flag bits: CS_ERR_INVALID. */
int cs_lattice_create(const int dims[4], const int block[4], int flags, cs_lattice* out);
int cs_lattice_destroy(cs_lattice lat);
/* Number of sites V. */
long long cs_lattice_volume(cs_lattice lat);
/* Bytes of one internal-layout spinor field of precision prec holding nrhs
 * right-hand sides (0 for an invalid precision). */
size_t cs_field_bytes(cs_lattice lat, cs_prec prec, int nrhs);

/* Canonical complex128 spinors (device) -> internal layout of precision prec
 * (device).  The nrhs fields are consecutive in both buffers. */
int cs_field_import(cs_lattice lat, cs_prec prec, void* dst_internal,
                    const void* src_canonical, int nrhs, void* stream);
/* Internal layout -> canonical complex128. */
int cs_field_export(cs_lattice lat, cs_prec prec, void* dst_canonical,
                    const void* src_internal, int nrhs, void* stream);

/* -------------------------------------------------------------- gauge field */

/* Copy the canonical links U (device, complex128 [V][4][3][3]) into the
 * library, compressed to rows 0 and 1 in every storage precision.  The third
 * row is rebuilt as conj(row0 x row1), which equals the stored row only for
 * exact SU(3) matrices: U must be SU(3) to rounding.  The input buffer is not
 * kept.  Completes on the stream before the call returns (the handle is then
 * usable on any stream). */
int cs_gauge_create(cs_lattice lat, const void* U_canonical, void* stream, cs_gauge* out);
int cs_gauge_destroy(cs_gauge g);

/* ----------------------------------------------------------- clover term */

/* Build C = 1 + T (paper Section 2, Eq. (1)) from the plaquette leaves, in
 * double precision, with
 *   T(x) = i kappa c_sw sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x),
 *   sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu],  F = (Q - Q^dag)/8,
 *   Q_{mu nu}(x) = the four counter-clockwise plaquettes at x in the plane.
 * Stored in double and float, together with the inverse C^-1 = (1 + T)^-1
 * (each 6x6 chirality block inverted in double precision; used by the
 * Jacobi form of the smoother).  Synchronises the stream before returning. */
int cs_clover_create(cs_gauge g, double kappa, double csw, void* stream, cs_clover* out);
int cs_clover_destroy(cs_clover c);
/* Write T (not 1 + T) in the canonical complex128 [V][12][12] layout. */
int cs_clover_export(cs_clover c, void* dst_canonical, void* stream);
/* Write (1 + T)^-1 (double precision) in the canonical complex128
 * [V][12][12] layout. */
int cs_clover_inverse_export(cs_clover c, void* dst_canonical, void* stream);

/* ---------------------------------------------------------------- operator */

/* out = D in for nrhs consecutive internal-layout fields of precision prec,
 * with D the clover-Wilson operator of the paper's Eq. (1) (Section 2):
 *   (D psi)(x) = (1 + T(x)) psi(x)
 *     - kappa sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu)
 *                     + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)].
 * out and in must not overlap. */
int cs_apply_D(cs_gauge g, cs_clover c, cs_prec prec, void* out, const void* in,
               int nrhs, void* stream);
/* out = D^dag in = gamma5 D gamma5 in. */
int cs_apply_Ddag(cs_gauge g, cs_clover c, cs_prec prec, void* out, const void* in,
                  int nrhs, void* stream);

/* ------------------------------------------------- multi-RHS launch shapes */

/* Launch shape of the multi-right-hand-side operator and SAP kernels:
 * rhs_tile right-hand sides per workgroup (the block's links and clover term
 * are read once per tile); when persistent_wgs > 0, a persistent launch of
 * that many workgroups striding over the (block, tile) work items; and
 * lanes_per_site of the FP32 / FP16 / BF16 SAP kernel: 1 (one lane per site),
 * 2 (a lane pair per site: forward and backward hops on separate lanes, one
 * chirality each), or 0 (the library chooses from the number of blocks).
 * Values other than 0, 1, 2 mean 0; the operator ignores lanes_per_site and
 * FP64 SAP always uses one lane per site. */
typedef struct {
    int rhs_tile;
    int persistent_wgs;
    int lanes_per_site;
} cs_launch_config;

/* Time the SAP half-sweep and the operator for rhs_tile in {1, 4, 8, 12}
 * (up to nrhs), for grid and persistent launches and (SAP below FP64) for
 * one and two lanes per site, on nrhs right-hand
 * sides of precision prec, and return the fastest shapes (either pointer may
 * be NULL).  The result is cached with the clover handle and used by
 * cs_gcr_solve when params.rhs_tile is 0.  Allocates and frees scratch
 * fields; synchronises the stream. */
int cs_autotune(cs_gauge g, cs_clover c, cs_prec prec, int nrhs, cs_launch_config* sap,
                cs_launch_config* dslash, void* stream);

/* -------------------------------------------------------------------- SAP */

/* Multiplicative Schwarz smoother (paper Section 2: domains updated in turn
 * with a fixed number of block-solver iterations; Section 3: used as the
 * post-smoother with a given start vector).  n_cy cycles, each a sweep over
 * the colour-0 blocks then the colour-1 blocks; on every block B of the
 * current colour
 *   r_B = b_B - (D x)_B,  delta = MR(D_BB, r_B, n_mr),  x_B += delta,
 * where D_BB drops every hopping term that leaves the block and MR is the
 * minimal-residual iteration delta += alpha rho, rho -= alpha D_BB rho,
 * alpha = <D_BB rho, rho> / |D_BB rho|^2, started from delta = 0, rho = r_B.
 * x holds x0 on entry (ignored when x0_is_zero != 0) and the result on exit.
 * b and x are nrhs consecutive internal fields of precision prec; they must
 * not overlap.  Needs an even number of blocks in every direction. */
int cs_sap_smooth(cs_gauge g, cs_clover c, cs_prec prec, void* x, const void* b,
                  int n_cy, int n_mr, int x0_is_zero, int nrhs, void* stream);

/* cs_sap_smooth and cs_apply_D with an explicit multi-right-hand-side launch
 * shape (cfg NULL: one right-hand side per workgroup).  Results are bitwise
 * identical to the untiled calls. */
int cs_sap_smooth_cfg(cs_gauge g, cs_clover c, cs_prec prec, void* x, const void* b,
                      int n_cy, int n_mr, int x0_is_zero, int nrhs,
                      const cs_launch_config* cfg, void* stream);
int cs_apply_D_cfg(cs_gauge g, cs_clover c, cs_prec prec, void* out, const void* in,
                   int nrhs, const cs_launch_config* cfg, void* stream);

/* The smoother in the form of the paper's QWS library (Section 2): the same
 * multiplicative red/black SAP, for the clover-preconditioned operator
 * A = C^-1 D = 1 + kappa C^-1 H, with every block system A_BB delta = rho
 * solved by n_jac Jacobi steps (A_BB has the identity on its diagonal, so
 * no inner products and no workgroup reductions are needed):
 *   rho = C^-1 (b - D x)_B,  delta = 0,  n_jac times: delta += rho - A_BB delta,
 *   x_B += delta.
 * For a right-hand side b of D x = b, A x = C^-1 b is the same system, so the
 * result smooths D x = b directly.  The Jacobi steps converge when the
 * spectral radius of kappa (C^-1 H)_BB is below one.  Arguments as
 * cs_sap_smooth_cfg (cfg may be NULL), n_jac >= 0. */
int cs_sap_smooth_jacobi(cs_gauge g, cs_clover c, cs_prec prec, void* x, const void* b,
                         int n_cy, int n_jac, int x0_is_zero, int nrhs,
                         const cs_launch_config* cfg, void* stream);

/* SAP whose block solves are even-odd preconditioned MR (the preconditioning
 * of DD-alphaAMG's solvers, which the paper's Section 3 compares its method
 * with, applied to SAP's block systems of Section 2): with the sites of a
 * block split by parity (x + y + z + t even / odd), the block system
 * D_BB delta = r_B is reduced to its Schur complement on the even sites,
 *   S = C_e - kappa^2 H_eo C_o^-1 H_oe,   S delta_e = r_e + kappa H_eo C_o^-1 r_o,
 * solved by n_mr MR steps from delta_e = 0, and the odd sites follow from
 * delta_o = C_o^-1 (r_o + kappa H_oe delta_e) (H_eo, H_oe the in-block hops,
 * C^-1 the inverse clover term of cs_clover_inverse_export).  One lane per
 * site (cfg->lanes_per_site is ignored).  Arguments, modes and errors as
 * cs_sap_smooth_cfg (cfg may be NULL). */
int cs_sap_smooth_eo(cs_gauge g, cs_clover c, cs_prec prec, void* x, const void* b,
                     int n_cy, int n_mr, int x0_is_zero, int nrhs,
                     const cs_launch_config* cfg, void* stream);

/* ------------------------------------------------------------------ solver */

typedef struct {
    int restart;          /* GCR restart length m (1..32)                        */
    int max_iter;         /* iteration cap                                       */
    int n_cy, n_mr;       /* SAP cycles and MR steps; n_cy = 0: no preconditioner */
    double tol;           /* stop when |b - D x| <= tol |b| (true FP64 residual)  */
    cs_prec inner_prec;   /* precision of the SAP preconditioner and of w = D z   */
    cs_prec basis_prec;   /* storage of the Krylov basis w_k: CS_F64, CS_F32, or
                             CS_F16 / CS_BF16 (one scale per site; inner_prec
                             CS_F32 or the same 16-bit type; not with the
                             multigrid preconditioner).  The orthogonalisation
                             arithmetic is FP64 whatever the storage          */
    double reliable_delta;/* restart early when |r_iter| < delta |r_true| (0: off) */
    int rhs_tile;         /* right-hand sides per workgroup in the batched SAP and
                             operator launches (0: autotuned, see cs_autotune)    */
    int use_graph;        /* 1: capture each iteration's kernels as a HIP graph
                             once and replay it (ignored while profiling)         */
    int block_solver;     /* SAP block solves: 0 = n_mr MR steps on D_BB; 1 =
                             n_mr Jacobi steps on (C^-1 D)_BB (the form of the
                             paper's QWS smoother, see cs_sap_smooth_jacobi); 2 =
                             n_mr even-odd preconditioned MR steps (see
                             cs_sap_smooth_eo)                                   */
    int rhs_groups;       /* 0 or 1: the nrhs right-hand sides advance as one
                             lock-step batch.  G > 1 (nrhs > 1, not with the
                             multigrid preconditioner): they are split into
                             min(G, nrhs) contiguous groups of near-equal size,
                             each solved as its own batch on its own workspace
                             (kept with the clover handle), private stream and
                             host thread, so the memory-bound level-1 kernels
                             of one group overlap the smoother of another.
                             Every column's result is bit-identical to its
                             single-right-hand-side solve either way.         */
} cs_solver_params;

typedef struct {
    int iters;            /* GCR iterations (= preconditioner applications)      */
    int restarts;         /* true-residual recomputations after the first        */
    double true_relres;   /* |b - D x| / |b| on exit, FP64                        */
    double seconds;       /* wall time of the call                               */
} cs_solver_stats;

/* Fill p with the defaults: restart 16, max_iter 2000, n_cy 2, n_mr 4,
 * tol 1e-10, inner CS_F32, basis CS_F32, reliable_delta 1e-5, rhs_tile 0,
 * use_graph 1, block_solver 0, rhs_groups 1. */
void cs_solver_params_default(cs_solver_params* p);

/* Solve D x = b by flexible GCR (outer arithmetic, reductions and the
 * residual recomputation in FP64), preconditioned by the SAP smoother in
 * p->inner_prec (the flexible outer iteration tolerates the nonlinear MR
 * preconditioner; mixed precision is recovered by recomputing the true
 * residual in FP64 at every restart, the iterative-refinement scheme of the
 * paper's Section 2).  x and b are nrhs consecutive CS_F64 internal fields;
 * x holds x0 on entry.  The right-hand sides advance together through
 * batched SAP and operator launches (links and clover read once per tile of
 * right-hand sides); each keeps its own scalars and stopping decisions, so
 * every column follows the iterations of a single-right-hand-side solve.
 * stats (host, may be NULL) has nrhs entries; seconds is the wall time of the
 * whole call.  Device workspace (2 m nrhs fields plus scalars) is allocated on
 * first use and kept with the clover handle.  The work runs on a private
 * stream after the caller's stream has been synchronised.  The host decides
 * after every iteration whether to go on; the next iteration is queued before
 * that decision, so the device may run one iteration past a stop, which
 * changes neither x nor the reported counts.  Returns CS_OK when every
 * right-hand side converged, else the first non-zero status. */
int cs_gcr_solve(cs_gauge g, cs_clover c, const cs_solver_params* p, void* x,
                 const void* b, int nrhs, cs_solver_stats* stats, void* stream);

/* Solve D^dag x = b (the adjoint system of the backward pass) with the same
 * method: D^dag = gamma5 D gamma5, so D (gamma5 x) = gamma5 b is solved by
 * cs_gcr_solve's algorithm.  Same arguments and ownership as cs_gcr_solve;
 * one extra FP64 field of workspace is kept with the clover handle. */
int cs_gcr_solve_dag(cs_gauge g, cs_clover c, const cs_solver_params* p, void* x,
                     const void* b, int nrhs, cs_solver_stats* stats, void* stream);

/* Solve D x = b with BiCGStab preconditioned on the right by SAP (the outer
 * solver of the paper's multigrid code is flexible BiCGStab, Section 3;
 * flexible because SAP with MR is not a fixed linear map).  Per iteration:
 * two SAP applications (n_cy cycles from zero, n_mr MR steps, in inner_prec;
 * none when n_cy = 0) and two operator applications in inner_prec; every
 * inner product is accumulated in FP64.  basis_prec selects the form:
 *   CS_F64  flexible BiCGStab with FP64 vectors.  The true FP64 residual is
 *           recomputed when the recursive one meets tol, drops below
 *           reliable_delta times the last true one (0 disables), or the
 *           iteration breaks down (<rh, v> = 0 or omega = 0); unless it meets
 *           tol the iteration restarts from x.
 *   CS_F32  the QWS scheme of the paper's Section 2: BiCGStab with FP32
 *           vectors solves D e = r / |r| to the relative tolerance
 *           reliable_delta (0 < reliable_delta < 1), inside an FP64
 *           Richardson iteration x += |r| e, r = b - D x.
 * Convergence is only declared on the true FP64 residual.
 *   params  tol, max_iter (BiCGStab iterations), n_cy, n_mr, inner_prec,
 *           basis_prec (CS_F64 or CS_F32; CS_F64 when inner_prec is CS_F64),
 *           reliable_delta, use_graph; restart and rhs_tile are ignored
 *   x, b    one CS_F64 internal field each (x holds the start vector)
 *   stats   optional; iters counts BiCGStab iterations, restarts the
 *           restarts (Richardson steps) after the first
 * Returns CS_OK, CS_NOT_CONVERGED (max_iter reached), CS_BREAKDOWN (a
 * restart without progress) or CS_NONFINITE; the same argument errors as
 * cs_gcr_solve, and CS_ERR_INVALID for reliable_delta outside (0, 1) with
 * CS_F32 vectors.  Synchronises the stream; the workspace (eleven or, with
 * CS_F32 vectors, fourteen fields) is kept with the clover handle. */
int cs_bicgstab_solve(cs_gauge g, cs_clover c, const cs_solver_params* p, void* x,
                      const void* b, cs_solver_stats* stats, void* stream);

/* --------------------------------------------------------------- multigrid */

/* Two-level multigrid preconditioner of the paper's Section 3 (adaptive
 * aggregation with SAP smoothing).  The aggregates are the 4^4 SAP blocks;
 * every aggregate carries nc = 2 nv coarse degrees of freedom, index
 * c = chi * nv + i with chi the chirality (spins 0, 1 / spins 2, 3), so that
 * the prolongator commutes with gamma5.  Everything runs in FP32 (coarse
 * reductions in FP64).
 *   setup       v_i = n_cy_setup SAP cycles on D v = eta_i from v = 0
 *               (i < nv); P = the columns p_{a,chi,i} obtained by modified
 *               Gram-Schmidt of v_0 .. v_{nv-1} restricted to aggregate a
 *               and chirality chi; D_c = P^dag D P.  Each of n_adapt passes
 *               then replaces every v_i by M_MG v_i and rebuilds P and D_c.
 *   M_MG r      r_c = P^dag r; e_c = BiCGStab on D_c e_c = r_c from zero,
 *               at most n_coarse iterations, stopping once the recursive
 *               residual is below tol_coarse |r_c| or on a breakdown;
 *               z = P e_c; then n_cy_post SAP cycles (MR block solves, n_mr
 *               steps) on D z = r started from z.
 * Storage: P as nv CS_F32 internal fields (field i holds p_{a,chi,i} for
 * every a and chi); coarse vectors float2[nblk][nc] with nblk the number of
 * 4^4 blocks in the lattice's block order (bx fastest); D_c as the 9-point
 * stencil float2[nblk][9][nc][nc], index [a][d][column][row] with d = 0 the
 * aggregate itself, d = 1 + 2 mu its +mu neighbour and d = 2 + 2 mu its -mu
 * neighbour (periodic), so that (D_c e)_a,row = sum_d sum_col
 * D_c[a][d][col][row] e_{n(a,d),col}. */
typedef struct cs_mg_s* cs_mg;

typedef struct {
    int nv;             /* null vectors (1..32)                                  */
    int n_cy_setup;     /* SAP cycles turning eta_i into v_i (>= 1)               */
    int n_mr;           /* MR steps per block solve in every SAP use (>= 1)       */
    int n_adapt;        /* adaptive passes (>= 0)                                 */
    int n_coarse;       /* coarse BiCGStab iteration cap per application (>= 1)   */
    int n_cy_post;      /* SAP post-smoothing cycles per application (>= 0)       */
    double tol_coarse;  /* relative coarse residual that ends the coarse solve    */
    cs_prec coarse_prec;/* storage of D_c read by the coarse solve and by
                           cs_mg_coarse_apply: CS_F32, or CS_F16 (an FP16 copy
                           made after every assembly; arithmetic stays FP32)  */
    cs_prec transfer_prec; /* storage of P read by restriction and
                           prolongation: CS_F32, or CS_F16 (an FP16 copy with
                           one FP32 scale per site, made after every rebuild;
                           D_c is still assembled from the FP32 P)            */
} cs_mg_params;

/* Defaults: nv 8, n_cy_setup 4, n_mr 4, n_adapt 1, n_coarse 50, n_cy_post 2,
 * tol_coarse 0.05, coarse_prec CS_F32, transfer_prec CS_F32. */
void cs_mg_params_default(cs_mg_params* p);

/* Build the hierarchy for operator (g, c).  etas: nv consecutive CS_F32
 * internal fields (device, caller-owned, read only; random vectors), so the
 * caller controls the random numbers.  Allocates 2 nv + 1 CS_F32 fields,
 * D_c (nblk * 9 * nc^2 float2, 288 nv^2 bytes per aggregate) and thirteen
 * coarse vectors of workspace (the coarse BiCGStab's vectors and the +mu
 * terms of a product), shared by every call on the handle, so calls on one
 * handle must be ordered (one stream); the handle refers to c, which must
 * outlive it.  Asynchronous on
 * the stream.  Errors: CS_ERR_NULL, CS_ERR_INVALID (parameters out of
 * range), CS_ERR_GEOMETRY (an odd number of blocks in some direction),
 * CS_ERR_ALLOC, CS_ERR_HIP. */
int cs_mg_create(cs_gauge g, cs_clover c, const cs_mg_params* p, const void* etas, void* stream,
                 cs_mg* out);
int cs_mg_destroy(cs_mg m);

/* Copies of P (nv CS_F32 internal fields) and D_c (layout above) into
 * caller-owned device buffers; either may be NULL.  Asynchronous. */
int cs_mg_export(cs_mg m, void* P, void* Dc, void* stream);

/* The pieces of M_MG on caller-owned device buffers (asynchronous):
 *   restrict      rc = P^dag r      (r a CS_F32 field, rc a coarse vector;
 *                                    P in transfer_prec)
 *   prolong       z = P ec          (ec a coarse vector, z a CS_F32 field)
 *   coarse_apply  y = D_c x         (coarse vectors, x != y)
 *   coarse_solve  ec = the coarse BiCGStab above from zero, with at most
 *                 n_iter iterations and relative tolerance tol
 *   apply         z = M_MG r        (CS_F32 fields, z != r) */
int cs_mg_restrict(cs_mg m, const void* r, void* rc, void* stream);
int cs_mg_prolong(cs_mg m, const void* ec, void* z, void* stream);
int cs_mg_coarse_apply(cs_mg m, const void* x, void* y, void* stream);
int cs_mg_coarse_solve(cs_mg m, const void* rc, void* ec, int n_iter, double tol, void* stream);
int cs_mg_apply(cs_mg m, void* z, const void* r, void* stream);

/* cs_gcr_solve with M_MG as the preconditioner (one right-hand side):
 * z_k = M_MG(r / |r_prev|) in FP32.  p->inner_prec must be CS_F32 (the
 * precision of w = D z); n_cy, n_mr and block_solver are not used (the
 * smoothing is the hierarchy's).  m must have been built for (g, c).  Same
 * stats, status codes and stream behaviour as cs_gcr_solve. */
int cs_gcr_solve_mg(cs_gauge g, cs_clover c, cs_mg m, const cs_solver_params* p, void* x,
                    const void* b, cs_solver_stats* stats, void* stream);

/* cs_bicgstab_solve with M_MG on the right in both preconditioner
 * applications of every iteration: the paper's method (Section 3), flexible
 * BiCGStab around the two-level multigrid preconditioner, in either vector
 * precision (p->basis_prec CS_F64: flexible BiCGStab with reliable restarts;
 * CS_F32: FP32 BiCGStab inner solves inside the FP64 Richardson iteration).
 * p->inner_prec must be CS_F32; n_cy, n_mr and block_solver are not used.  m
 * must have been built for (g, c).  Same stats, status codes and stream
 * behaviour as cs_bicgstab_solve. */
int cs_bicgstab_solve_mg(cs_gauge g, cs_clover c, cs_mg m, const cs_solver_params* p, void* x,
                         const void* b, cs_solver_stats* stats, void* stream);

/* ---------------------------------------------------------------- gradient */

/* Gradient with respect to the links of a real function L of x = D^{-1} b.
 * Given x (the solution) and y = D^{-dag} eta, where eta is dL/dx in the
 * convention dL = Re(eta^dag dx), every change dD of the operator changes L
 * by -Re(y^dag dD x).  With links varied as U_mu(x) -> exp(i w T^a) U_mu(x),
 * T^a = lambda^a / 2 (Gell-Mann), this computes g_{mu,a}(x) = dL/dw for the
 * hopping term and the clover term of the paper's Eq. (1) (Section 2; the
 * clover term through the derivative of every plaquette leaf of F).
 *   x, y     CS_F64 internal fields (one right-hand side each)
 *   g_lie    device, double [V][4][8] in canonical site order, or NULL
 *   grad_U   device, complex128 [V][4][3][3], or NULL: the tangent-space
 *            gradient G = 2 i (sum_a g_a T^a) U, which satisfies
 *            dL = Re tr(G^dag dU) for every dU = i X U, X Hermitian
 *            traceless (the gradient of any SU(3)-valued parametrisation).
 * Needs 864 bytes per site of device workspace (kept with the clover
 * handle).  Asynchronous on the stream. */
int cs_force(cs_gauge g, cs_clover c, const void* x, const void* y, double* g_lie,
             void* grad_U, void* stream);

/* cs_force for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid allocation): the same
 * kernels and results, with the insertion-matrix workspace taken from a
 * fixed 128 MiB device array of the library instead of memory allocated on
 * the first call.  No device memory is allocated or freed.  The lattice may
 * have at most 155,344 sites (864 bytes each; a 16^3 x 32 lattice fits,
 * 32^3 x 64 does not): larger lattices return CS_ERR_INVALID.  Every GPU
 * that runs it holds its own copy of the array until the process ends (its
 * address is looked up on the first call on that device).  The workspace is
 * written in full before it is read, and its contents are left from the last
 * call; calls that overlap in time on one GPU (on different streams, or from
 * different threads) share it and race. */
int cs_force_noalloc(cs_gauge g, cs_clover c, const void* x, const void* y, double* g_lie,
                     void* grad_U, void* stream);

/* -------------------------------------------------------------- profiling */

/* When enabled, every kernel launch of the library is bracketed by HIP
 * events on the stream it runs on.  cs_profile_query returns the number of
 * launches and their summed duration (ms) for a kernel family name (one of
 * "dslash", "sap_halfsweep", "blas", "convert", "clover_build"), after
 * synchronising the recorded events ("force" covers cs_force).
 * "copy" covers cs_device_copy; "sap_general" and "sap_from_zero" split the
 * "sap_halfsweep" launches into those with x nonzero everywhere and the two
 * half-sweeps of a cycle that start from x = 0.  cs_profile_reset clears the counters. */
int cs_profile_enable(int on);
int cs_profile_query(const char* name, long long* count, double* total_ms);
int cs_profile_reset(void);

/* Bandwidth reference (not part of the method): dst = src for `bytes` bytes
 * of device memory by a plain streaming-copy kernel, so that the field
 * kernels' HBM rates can be set beside what a copy reaches on the same GPU
 * in the same run.  bytes and both pointers must be multiples of 16 and the
 * buffers must not overlap (CS_ERR_INVALID); asynchronous on the stream. */
int cs_device_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Measurement probe (not part of the method), for the question whether the
 * product of a link with the half spinors of a tile of right-hand sides
 * pays on the matrix cores: per site V = U^reps H (the product chained reps
 * times), U a complex 3x3 matrix, H a complex 3 x 16 matrix (two spin
 * components for 8 right-hand sides).  kind 0: FP32 vector arithmetic, one
 * lane per site; kind 1: v_mfma_f32_16x16x16_bf16 on two sites at a time
 * (the real 6x6 forms of their links block-diagonal in one operand; four
 * independent pairs per wave), bfloat16 inputs and FP32 accumulation, each
 * step's result rounded to bfloat16 for the next.  Layouts (device, float):
 * U [nsites][9][2], H and V [nsites][16][3][2] (column, colour, re/im).
 * nsites must be a multiple of 8 for kind 1 (CS_ERR_INVALID).  Asynchronous
 * on the stream. */
int cs_probe_link_product(int kind, long long nsites, int reps, const float* U, const float* H, float* V,
                          void* stream);

#ifdef __cplusplus
}
#endif
#endif
