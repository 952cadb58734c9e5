/*
 * Plain FP64 CPU oracle for the clover-Wilson operator, the red/black SAP
 * smoother with MR block solves, flexible GCR, and the gauge-link gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the GPU path: the two meet
 * only through canonical arrays.
 *
 * Canonical layouts (all complex double, C order, site index x fastest:
 * s = x + Lx*(y + Ly*(z + Lz*t))):
 *   U   [V][4][3][3]   links U_mu(x), mu = 0..3 for x, y, z, t, [row][col]
 *   psi [V][4][3]      spinors, index 3*spin + colour
 *   T   [V][12][12]    clover term T(x) (so C = 1 + T, paper Section 2, Eq. (1))
 *   g   [V][4][8]      real gradient components g_{mu,a}(x)
 * Boundary conditions are periodic in all four directions.
 *
 * Parity status: every function below is pinned by a CPU test against a
 * property the mathematics fixes (tests/test_oracle_*.py).
 */
#ifndef CLOVERSAP_ORACLE_H
#define CLOVERSAP_ORACLE_H

#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef double _Complex ocplx;

/* OpenMP threads used by the site and block loops (1 = serial). */
void or_set_threads(int n);
int or_get_threads(void);

/* Gamma matrices of the chiral basis; mu = 0..3, mu = 4 gives gamma5. */
void or_gamma(int mu, ocplx g[16]);
/* sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu]. */
void or_sigma(int mu, int nu, ocplx s[16]);

/* Clover term T(x) = i kappa c_sw sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}(x). */
void or_clover_site(const int dims[4], const ocplx* U, double kappa, double csw,
                    long site, ocplx T[144]);
void or_clover_field(const int dims[4], const ocplx* U, double kappa, double csw,
                     ocplx* T);
/* Q_{mu nu}(x): sum of the four plaquette leaves, for the closed-form pin. */
void or_leaf_sum(const int dims[4], const ocplx* U, long site, int mu, int nu,
                 ocplx Q[9]);

/* out = D in, with D = 1 + T - kappa * hopping (T may be NULL: no clover). */
void or_apply_D(const int dims[4], const ocplx* U, const ocplx* T, double kappa,
                const ocplx* in, ocplx* out);
/* out = gamma5 D gamma5 in  (= D^dagger). */
void or_apply_Ddag(const int dims[4], const ocplx* U, const ocplx* T, double kappa,
                   const ocplx* in, ocplx* out);
/* D at selected sites only, clover built on the fly: out[n][12]. */
void or_apply_D_sites(const int dims[4], const ocplx* U, double kappa, double csw,
                      const ocplx* in, long nsites, const long* sites, ocplx* out);
/* |b - D x|_2 with the clover built on the fly (no T array). */
double or_residual_norm(const int dims[4], const ocplx* U, double kappa, double csw,
                        const ocplx* b, const ocplx* x);

/* Block geometry: block dims bdim[4] must divide dims.  Returns the number of
 * blocks; colour of block = (sum of block coordinates) mod 2. */
long or_num_blocks(const int dims[4], const int bdim[4]);
int or_block_colour(const int dims[4], const int bdim[4], long blk);
long or_block_of_site(const int dims[4], const int bdim[4], long site);

/* Dirichlet block operator D_BB: out = D restricted to block blk (every term
 * whose source site lies outside the block is dropped).  Reads in / writes out
 * at the sites of block blk only (full-lattice arrays). */
void or_apply_D_block(const int dims[4], const int bdim[4], long blk, const ocplx* U,
                      const ocplx* T, double kappa, const ocplx* in, ocplx* out);

/* n_mr minimal-residual steps on D_BB: delta ~ D_BB^{-1} r on block blk.
 * delta written at block sites; r read at block sites. */
void or_mr_block(const int dims[4], const int bdim[4], long blk, const ocplx* U,
                 const ocplx* T, double kappa, int n_mr, const ocplx* r, ocplx* delta);

/* Multiplicative red/black SAP: n_cy cycles of (colour 0, colour 1); x holds
 * x0 on entry and the smoothed result on exit. */
void or_sap(const int dims[4], const int bdim[4], const ocplx* U, const ocplx* T,
            double kappa, int n_cy, int n_mr, const ocplx* b, ocplx* x);

/* Flexible GCR(restart) with SAP(n_cy, n_mr) as the preconditioner
 * (n_cy = 0: no preconditioner).  x holds x0 on entry.  Stops when the true
 * residual |b - Dx|/|b| <= tol or after max_iter iterations.
 * hist (length max_iter + 1, may be NULL) receives the recursive relative
 * residual after each iteration (hist[0] = initial true residual).
 * Returns 0 on convergence, 1 if max_iter was reached, 2 on breakdown. */
/* C^-1 = (1 + T)^-1 per site (Gauss-Jordan); T NULL means T = 0. */
void or_clover_inverse_site(const ocplx* T, ocplx* Cinv);
void or_clover_inverse_field(const int dims[4], const ocplx* T, ocplx* Cinv);
/* Jacobi block solve of one block (rho = C^-1 r_B); see oracle.c. */
void or_jacobi_block(const int dims[4], const int bdim[4], long blk, const ocplx* U, const ocplx* T,
                     double kappa, int n_jac, const ocplx* r, ocplx* delta);
/* SAP on A = C^-1 D with n_jac Jacobi steps per block; see oracle.c. */
void or_sap_jacobi(const int dims[4], const int bdim[4], const ocplx* U, const ocplx* T,
                   double kappa, int n_cy, int n_jac, const ocplx* b, ocplx* x);
/* Even-odd preconditioned MR block solve (Schur complement on the even sites,
 * back-substitution on the odd ones) and SAP built on it. */
void or_mr_eo_block(const int dims[4], const int bdim[4], long blk, const ocplx* U, const ocplx* T,
                    double kappa, int n_mr, const ocplx* r, ocplx* delta);
void or_sap_eo(const int dims[4], const int bdim[4], const ocplx* U, const ocplx* T, double kappa,
               int n_cy, int n_mr, const ocplx* b, ocplx* x);

int or_fgcr(const int dims[4], const int bdim[4], const ocplx* U, const ocplx* T,
            double kappa, int n_cy, int n_mr, int restart, double tol, int max_iter,
            const ocplx* b, ocplx* x, int* iters, double* true_relres, double* hist);
/* Flexible BiCGStab, SAP preconditioner on the right; see oracle.c. */
int or_fbicgstab(const int dims[4], const int bdim[4], const ocplx* U, const ocplx* T,
                 double kappa, int n_cy, int n_mr, double tol, int max_iter, double delta,
                 const ocplx* b, ocplx* x, int* iters, int* restarts, double* relres,
                 double* hist);
/* FP64 Richardson iteration around inner BiCGStab solves; see oracle.c. */
int or_richardson_bicgstab(const int dims[4], const int bdim[4], const ocplx* U, const ocplx* T,
                           double kappa, int n_cy, int n_mr, double tol, int max_iter,
                           double inner_tol, const ocplx* b, ocplx* x, int* iters, int* outer,
                           double* relres);

/* Gradient of L = Re(eta^dag D^{-1} b) with respect to the left Lie-algebra
 * coordinates of every link, U -> exp(i w T^a) U, given x = D^{-1} b and
 * y = D^{-dag} eta:  g_{mu,a}(x) = -Re(y^dag (dD/dw) x).  T^a = lambda^a / 2.
 * hop and clover parts are written separately (either may be NULL). */
void or_force(const int dims[4], const ocplx* U, double kappa, double csw,
              const ocplx* x, const ocplx* y, double* g_hop, double* g_clov);
/* Gell-Mann generator T^a = lambda^a / 2, a = 0..7. */
void or_su3_generator(int a, ocplx t[9]);

#ifdef __cplusplus
}
#endif
#endif
