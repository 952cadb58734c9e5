/*
 * Plain FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Written for readability against the definitions, not for speed: every
 * matrix product is an explicit loop, gamma matrices act as full 4x4 spin
 * matrices (no spin projection), and the clover term is assembled from
 * explicit sigma_{mu nu} (x) F_{mu nu} products.  OpenMP only splits loops
 * whose iterations write disjoint outputs; every reduction is a serial sum,
 * so results do not depend on the thread count.
 *
 * Definitions followed (the paper: Section 2, Eq. (1) for D and C; Section 2
 * and Section 3 for the multiplicative SAP and the flexible outer solver):
 *   (D psi)(x) = psi(x) + T(x) psi(x)
 *                - kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
 *                               + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ]
 *   C = 1 + T,  T(x) = (i/2) kappa c_sw sum_{mu,nu} sigma_{mu nu} F_{mu nu}(x)
 *                    = i kappa c_sw sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x)
 *   sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu],  F = (Q - Q^dag) / 8,
 *   Q_{mu nu}(x) = sum of the four plaquette leaves around x in the
 *   (mu, nu) plane, each starting and ending at x.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define I_ _Complex_I

static int g_threads = 1;

void or_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int or_get_threads(void) { return g_threads; }

/* ------------------------------------------------------------------ geometry */

static long vol4(const int d[4]) { return (long)d[0] * d[1] * d[2] * d[3]; }

static void site_coords(const int d[4], long s, int c[4]) {
    c[0] = (int)(s % d[0]); s /= d[0];
    c[1] = (int)(s % d[1]); s /= d[1];
    c[2] = (int)(s % d[2]); s /= d[2];
    c[3] = (int)s;
}

static long site_index(const int d[4], const int c[4]) {
    return c[0] + (long)d[0] * (c[1] + (long)d[1] * (c[2] + (long)d[2] * c[3]));
}

/* site + off (periodic) */
static long site_displace(const int d[4], long s, const int off[4]) {
    int c[4];
    site_coords(d, s, c);
    for (int m = 0; m < 4; ++m) c[m] = ((c[m] + off[m]) % d[m] + d[m]) % d[m];
    return site_index(d, c);
}

static long site_step(const int d[4], long s, int mu, int step) {
    int off[4] = {0, 0, 0, 0};
    off[mu] = step;
    return site_displace(d, s, off);
}

long or_num_blocks(const int d[4], const int b[4]) {
    return (long)(d[0] / b[0]) * (d[1] / b[1]) * (d[2] / b[2]) * (d[3] / b[3]);
}

long or_block_of_site(const int d[4], const int b[4], long s) {
    int c[4], nb[4];
    site_coords(d, s, c);
    for (int m = 0; m < 4; ++m) { nb[m] = d[m] / b[m]; c[m] /= b[m]; }
    return c[0] + (long)nb[0] * (c[1] + (long)nb[1] * (c[2] + (long)nb[2] * c[3]));
}

static void block_coords(const int d[4], const int b[4], long blk, int bc[4]) {
    int nb[4];
    for (int m = 0; m < 4; ++m) nb[m] = d[m] / b[m];
    site_coords(nb, blk, bc);
}

int or_block_colour(const int d[4], const int b[4], long blk) {
    int bc[4];
    block_coords(d, b, blk, bc);
    return (bc[0] + bc[1] + bc[2] + bc[3]) % 2;
}

/* Global site of local index l (x fastest within the block). */
static long block_site(const int d[4], const int b[4], long blk, long l) {
    int bc[4], lc[4], c[4];
    block_coords(d, b, blk, bc);
    site_coords(b, l, lc);
    for (int m = 0; m < 4; ++m) c[m] = bc[m] * b[m] + lc[m];
    return site_index(d, c);
}

/* Local index of a site inside its own block. */
static long local_index(const int d[4], const int b[4], long s) {
    int c[4];
    site_coords(d, s, c);
    for (int m = 0; m < 4; ++m) c[m] %= b[m];
    return site_index(b, c);
}

/* ------------------------------------------------------- spin and colour algebra */

void or_gamma(int mu, ocplx g[16]) {
    memset(g, 0, 16 * sizeof(ocplx));
    switch (mu) {
    case 0: /* [[0, -i sigma1], [i sigma1, 0]] */
        g[0 * 4 + 3] = -I_; g[1 * 4 + 2] = -I_; g[2 * 4 + 1] = I_; g[3 * 4 + 0] = I_;
        break;
    case 1: /* [[0, -i sigma2], [i sigma2, 0]] */
        g[0 * 4 + 3] = -1; g[1 * 4 + 2] = 1; g[2 * 4 + 1] = 1; g[3 * 4 + 0] = -1;
        break;
    case 2: /* [[0, -i sigma3], [i sigma3, 0]] */
        g[0 * 4 + 2] = -I_; g[1 * 4 + 3] = I_; g[2 * 4 + 0] = I_; g[3 * 4 + 1] = -I_;
        break;
    case 3: /* [[0, 1], [1, 0]] */
        g[0 * 4 + 2] = 1; g[1 * 4 + 3] = 1; g[2 * 4 + 0] = 1; g[3 * 4 + 1] = 1;
        break;
    default: { /* gamma5 = gamma_x gamma_y gamma_z gamma_t */
        ocplx a[16], b[16], t[16];
        or_gamma(0, a);
        for (int m = 1; m < 4; ++m) {
            or_gamma(m, b);
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    ocplx s = 0;
                    for (int k = 0; k < 4; ++k) s += a[i * 4 + k] * b[k * 4 + j];
                    t[i * 4 + j] = s;
                }
            memcpy(a, t, sizeof t);
        }
        memcpy(g, a, sizeof a);
    }
    }
}

void or_sigma(int mu, int nu, ocplx s[16]) {
    ocplx a[16], b[16];
    or_gamma(mu, a);
    or_gamma(nu, b);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            ocplx ab = 0, ba = 0;
            for (int k = 0; k < 4; ++k) {
                ab += a[i * 4 + k] * b[k * 4 + j];
                ba += b[i * 4 + k] * a[k * 4 + j];
            }
            s[i * 4 + j] = 0.5 * I_ * (ab - ba);
        }
}

static void m3_mul(const ocplx* a, const ocplx* b, ocplx* c) {
    ocplx t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            ocplx s = 0;
            for (int k = 0; k < 3; ++k) s += a[i * 3 + k] * b[k * 3 + j];
            t[i * 3 + j] = s;
        }
    memcpy(c, t, sizeof t);
}

static void m3_dag(const ocplx* a, ocplx* c) {
    ocplx t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) t[i * 3 + j] = conj(a[j * 3 + i]);
    memcpy(c, t, sizeof t);
}

static void m3_unit(ocplx* c) {
    memset(c, 0, 9 * sizeof(ocplx));
    c[0] = c[4] = c[8] = 1;
}

void or_su3_generator(int a, ocplx t[9]) {
    /* Gell-Mann matrices lambda^a, halved. */
    memset(t, 0, 9 * sizeof(ocplx));
    switch (a) {
    case 0: t[1] = 1; t[3] = 1; break;
    case 1: t[1] = -I_; t[3] = I_; break;
    case 2: t[0] = 1; t[4] = -1; break;
    case 3: t[2] = 1; t[6] = 1; break;
    case 4: t[2] = -I_; t[6] = I_; break;
    case 5: t[5] = 1; t[7] = 1; break;
    case 6: t[5] = -I_; t[7] = I_; break;
    default: t[0] = 1 / sqrt(3.0); t[4] = 1 / sqrt(3.0); t[8] = -2 / sqrt(3.0); break;
    }
    for (int i = 0; i < 9; ++i) t[i] *= 0.5;
}

static const ocplx* link_at(const ocplx* U, long s, int mu) { return U + (s * 4 + mu) * 9; }

/* ------------------------------------------------------------ plaquette leaves */

/* One factor of a leaf: the link U_dir(x + a*mu_hat + b*nu_hat), daggered or
 * not; dir is mu (is_nu = 0) or nu (is_nu = 1).  The four leaves are the four
 * counter-clockwise plaquettes of the (mu, nu) plane that start and end at x:
 *   U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
 *   U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu)
 *   U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu)
 *   U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^dag                    */
typedef struct { int a, b, is_nu, dag; } leaf_factor;

static const leaf_factor LEAVES[4][4] = {
    {{0, 0, 0, 0}, {1, 0, 1, 0}, {0, 1, 0, 1}, {0, 0, 1, 1}},
    {{0, 0, 1, 0}, {-1, 1, 0, 1}, {-1, 0, 1, 1}, {-1, 0, 0, 0}},
    {{-1, 0, 0, 1}, {-1, -1, 1, 1}, {-1, -1, 0, 0}, {0, -1, 1, 0}},
    {{0, -1, 1, 1}, {0, -1, 0, 0}, {1, -1, 1, 0}, {0, 0, 0, 1}},
};

/* Site and direction of factor f of leaf l around site x in plane (mu, nu). */
static void leaf_link(const int d[4], long x, int mu, int nu, int l, int f, long* site,
                      int* dir) {
    const leaf_factor* F = &LEAVES[l][f];
    int off[4] = {0, 0, 0, 0};
    off[mu] += F->a;
    off[nu] += F->b;
    *site = site_displace(d, x, off);
    *dir = F->is_nu ? nu : mu;
}

/* The matrix of factor f (U or U^dag). */
static void leaf_factor_matrix(const int d[4], const ocplx* U, long x, int mu, int nu,
                               int l, int f, ocplx m[9]) {
    long s;
    int dir;
    leaf_link(d, x, mu, nu, l, f, &s, &dir);
    if (LEAVES[l][f].dag) m3_dag(link_at(U, s, dir), m);
    else memcpy(m, link_at(U, s, dir), 9 * sizeof(ocplx));
}

static void leaf_product(const int d[4], const ocplx* U, long x, int mu, int nu, int l,
                         ocplx P[9]) {
    ocplx m[9];
    m3_unit(P);
    for (int f = 0; f < 4; ++f) {
        leaf_factor_matrix(d, U, x, mu, nu, l, f, m);
        m3_mul(P, m, P);
    }
}

void or_leaf_sum(const int d[4], const ocplx* U, long x, int mu, int nu, ocplx Q[9]) {
    ocplx P[9];
    memset(Q, 0, 9 * sizeof(ocplx));
    for (int l = 0; l < 4; ++l) {
        leaf_product(d, U, x, mu, nu, l, P);
        for (int i = 0; i < 9; ++i) Q[i] += P[i];
    }
}

/* T += i kappa c_sw sigma_{mu nu} (x) F  (spin-colour index 3*spin + colour) */
static void add_sigma_F(int mu, int nu, const ocplx F[9], double kappa, double csw,
                        ocplx T[144]) {
    ocplx sg[16];
    or_sigma(mu, nu, sg);
    for (int s = 0; s < 4; ++s)
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    T[(3 * s + a) * 12 + 3 * sp + b] += I_ * kappa * csw * sg[s * 4 + sp] * F[a * 3 + b];
}

void or_clover_site(const int d[4], const ocplx* U, double kappa, double csw, long x,
                    ocplx T[144]) {
    memset(T, 0, 144 * sizeof(ocplx));
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu) {
            ocplx Q[9], F[9];
            or_leaf_sum(d, U, x, mu, nu, Q);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) F[a * 3 + b] = (Q[a * 3 + b] - conj(Q[b * 3 + a])) / 8.0;
            add_sigma_F(mu, nu, F, kappa, csw, T);
        }
}

void or_clover_field(const int d[4], const ocplx* U, double kappa, double csw, ocplx* T) {
    long V = vol4(d);
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (long x = 0; x < V; ++x) or_clover_site(d, U, kappa, csw, x, T + x * 144);
}

/* ------------------------------------------------------------------ operator */

/* hop(x) = sum_mu [ (1 - gamma_mu) U_mu(x) in(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dag in(x-mu) ]
 * keep(site) decides whether a source site contributes (NULL: all do). */
typedef int (*keep_fn)(const void* ctx, long site);

static void hop_site(const int d[4], const ocplx* U, const ocplx G[4][16],
                     const ocplx* in, long x, keep_fn keep, const void* ctx, ocplx acc[12]) {
    memset(acc, 0, 12 * sizeof(ocplx));
    for (int mu = 0; mu < 4; ++mu) {
        for (int dirn = 0; dirn < 2; ++dirn) {
            long y = site_step(d, x, mu, dirn == 0 ? +1 : -1);
            if (keep && !keep(ctx, y)) continue;
            ocplx v[12];
            if (dirn == 0) { /* U_mu(x) in(x+mu) */
                const ocplx* u = link_at(U, x, mu);
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) {
                        ocplx t = 0;
                        for (int b = 0; b < 3; ++b) t += u[a * 3 + b] * in[y * 12 + 3 * s + b];
                        v[3 * s + a] = t;
                    }
            } else { /* U_mu(x-mu)^dag in(x-mu) */
                const ocplx* u = link_at(U, y, mu);
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) {
                        ocplx t = 0;
                        for (int b = 0; b < 3; ++b) t += conj(u[b * 3 + a]) * in[y * 12 + 3 * s + b];
                        v[3 * s + a] = t;
                    }
            }
            double sgn = dirn == 0 ? -1.0 : +1.0; /* (1 - gamma) forward, (1 + gamma) backward */
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a) {
                    ocplx gv = 0;
                    for (int sp = 0; sp < 4; ++sp) gv += G[mu][s * 4 + sp] * v[3 * sp + a];
                    acc[3 * s + a] += v[3 * s + a] + sgn * gv;
                }
        }
    }
}

static void load_gammas(ocplx G[4][16]) {
    for (int m = 0; m < 4; ++m) or_gamma(m, G[m]);
}

/* out(x) = in(x) + T(x) in(x) - kappa hop(x) */
static void d_site(const ocplx* Tx, double kappa, const ocplx* in_x, const ocplx hop[12],
                   ocplx out[12]) {
    for (int i = 0; i < 12; ++i) {
        ocplx t = in_x[i];
        if (Tx)
            for (int j = 0; j < 12; ++j) t += Tx[i * 12 + j] * in_x[j];
        out[i] = t - kappa * hop[i];
    }
}

void or_apply_D(const int d[4], const ocplx* U, const ocplx* T, double kappa,
                const ocplx* in, ocplx* out) {
    long V = vol4(d);
    ocplx G[4][16];
    load_gammas(G);
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (long x = 0; x < V; ++x) {
        ocplx hop[12];
        hop_site(d, U, (const ocplx(*)[16])G, in, x, NULL, NULL, hop);
        d_site(T ? T + x * 144 : NULL, kappa, in + x * 12, hop, out + x * 12);
    }
}

static void apply_g5(long V, const ocplx* in, ocplx* out) {
    ocplx g5[16];
    or_gamma(4, g5);
    for (long x = 0; x < V; ++x)
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) {
                ocplx t = 0;
                for (int sp = 0; sp < 4; ++sp) t += g5[s * 4 + sp] * in[x * 12 + 3 * sp + a];
                out[x * 12 + 3 * s + a] = t;
            }
}

void or_apply_Ddag(const int d[4], const ocplx* U, const ocplx* T, double kappa,
                   const ocplx* in, ocplx* out) {
    long V = vol4(d);
    ocplx* tmp = malloc(sizeof(ocplx) * 12 * V);
    apply_g5(V, in, tmp);
    or_apply_D(d, U, T, kappa, tmp, out);
    apply_g5(V, out, tmp);
    memcpy(out, tmp, sizeof(ocplx) * 12 * V);
    free(tmp);
}

void or_apply_D_sites(const int d[4], const ocplx* U, double kappa, double csw,
                      const ocplx* in, long n, const long* sites, ocplx* out) {
    ocplx G[4][16];
    load_gammas(G);
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (long i = 0; i < n; ++i) {
        ocplx T[144], hop[12];
        long x = sites[i];
        or_clover_site(d, U, kappa, csw, x, T);
        hop_site(d, U, (const ocplx(*)[16])G, in, x, NULL, NULL, hop);
        d_site(T, kappa, in + x * 12, hop, out + i * 12);
    }
}

double or_residual_norm(const int d[4], const ocplx* U, double kappa, double csw,
                        const ocplx* b, const ocplx* x) {
    long V = vol4(d);
    double* part = malloc(sizeof(double) * V);
    ocplx G[4][16];
    load_gammas(G);
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (long s = 0; s < V; ++s) {
        ocplx T[144], hop[12], dx[12];
        or_clover_site(d, U, kappa, csw, s, T);
        hop_site(d, U, (const ocplx(*)[16])G, x, s, NULL, NULL, hop);
        d_site(T, kappa, x + s * 12, hop, dx);
        double acc = 0;
        for (int i = 0; i < 12; ++i) {
            ocplx r = b[s * 12 + i] - dx[i];
            acc += creal(r) * creal(r) + cimag(r) * cimag(r);
        }
        part[s] = acc;
    }
    double sum = 0;
    for (long s = 0; s < V; ++s) sum += part[s];
    free(part);
    return sqrt(sum);
}

/* -------------------------------------------------------------- block operator */

typedef struct { const int* d; const int* b; long blk; } block_ctx;

static int in_block(const void* ctx, long site) {
    const block_ctx* c = ctx;
    return or_block_of_site(c->d, c->b, site) == c->blk;
}

/* D_BB on block-local arrays: in_l / out_l indexed by local index.  The hop
 * reads a full-lattice view built from the local array. */
static void dbb_local(const int d[4], const int b[4], long blk, const ocplx* U,
                      const ocplx* T, double kappa, const ocplx G[4][16],
                      const ocplx* in_l, ocplx* out_l) {
    long bv = vol4(b);
    block_ctx ctx = {d, b, blk};
    for (long l = 0; l < bv; ++l) {
        long x = block_site(d, b, blk, l);
        ocplx acc[12];
        memset(acc, 0, sizeof acc);
        for (int mu = 0; mu < 4; ++mu)
            for (int dirn = 0; dirn < 2; ++dirn) {
                long y = site_step(d, x, mu, dirn == 0 ? +1 : -1);
                if (!in_block(&ctx, y)) continue;
                const ocplx* src = in_l + local_index(d, b, y) * 12;
                ocplx v[12];
                if (dirn == 0) {
                    const ocplx* u = link_at(U, x, mu);
                    for (int s = 0; s < 4; ++s)
                        for (int a = 0; a < 3; ++a) {
                            ocplx t = 0;
                            for (int c = 0; c < 3; ++c) t += u[a * 3 + c] * src[3 * s + c];
                            v[3 * s + a] = t;
                        }
                } else {
                    const ocplx* u = link_at(U, y, mu);
                    for (int s = 0; s < 4; ++s)
                        for (int a = 0; a < 3; ++a) {
                            ocplx t = 0;
                            for (int c = 0; c < 3; ++c) t += conj(u[c * 3 + a]) * src[3 * s + c];
                            v[3 * s + a] = t;
                        }
                }
                double sgn = dirn == 0 ? -1.0 : +1.0;
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) {
                        ocplx gv = 0;
                        for (int sp = 0; sp < 4; ++sp) gv += G[mu][s * 4 + sp] * v[3 * sp + a];
                        acc[3 * s + a] += v[3 * s + a] + sgn * gv;
                    }
            }
        d_site(T ? T + x * 144 : NULL, kappa, in_l + l * 12, acc, out_l + l * 12);
    }
}

void or_apply_D_block(const int d[4], const int b[4], long blk, const ocplx* U,
                      const ocplx* T, double kappa, const ocplx* in, ocplx* out) {
    long bv = vol4(b);
    ocplx G[4][16];
    load_gammas(G);
    ocplx* il = malloc(sizeof(ocplx) * 12 * bv);
    ocplx* ol = malloc(sizeof(ocplx) * 12 * bv);
    for (long l = 0; l < bv; ++l)
        memcpy(il + l * 12, in + block_site(d, b, blk, l) * 12, 12 * sizeof(ocplx));
    dbb_local(d, b, blk, U, T, kappa, (const ocplx(*)[16])G, il, ol);
    for (long l = 0; l < bv; ++l)
        memcpy(out + block_site(d, b, blk, l) * 12, ol + l * 12, 12 * sizeof(ocplx));
    free(il);
    free(ol);
}

static ocplx vdot(long n, const ocplx* a, const ocplx* b) { /* sum conj(a) b */
    ocplx s = 0;
    for (long i = 0; i < n; ++i) s += conj(a[i]) * b[i];
    return s;
}

static double vnorm2(long n, const ocplx* a) {
    double s = 0;
    for (long i = 0; i < n; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

/* Minimal residual on D_BB, local arrays: delta = 0, rho = r; repeat n_mr:
 * q = D_BB rho, alpha = <q, rho>/<q, q>, delta += alpha rho, rho -= alpha q. */
static void mr_local(const int d[4], const int b[4], long blk, const ocplx* U,
                     const ocplx* T, double kappa, const ocplx G[4][16], int n_mr,
                     const ocplx* r_l, ocplx* delta_l) {
    long n = vol4(b) * 12;
    ocplx* rho = malloc(sizeof(ocplx) * n);
    ocplx* q = malloc(sizeof(ocplx) * n);
    memcpy(rho, r_l, sizeof(ocplx) * n);
    memset(delta_l, 0, sizeof(ocplx) * n);
    for (int it = 0; it < n_mr; ++it) {
        dbb_local(d, b, blk, U, T, kappa, G, rho, q);
        double qq = vnorm2(n, q);
        if (qq == 0.0) break;
        ocplx alpha = vdot(n, q, rho) / qq;
        for (long i = 0; i < n; ++i) {
            delta_l[i] += alpha * rho[i];
            rho[i] -= alpha * q[i];
        }
    }
    free(rho);
    free(q);
}

void or_mr_block(const int d[4], const int b[4], long blk, const ocplx* U, const ocplx* T,
                 double kappa, int n_mr, const ocplx* r, ocplx* delta) {
    long bv = vol4(b);
    ocplx G[4][16];
    load_gammas(G);
    ocplx* rl = malloc(sizeof(ocplx) * 12 * bv);
    ocplx* dl = malloc(sizeof(ocplx) * 12 * bv);
    for (long l = 0; l < bv; ++l)
        memcpy(rl + l * 12, r + block_site(d, b, blk, l) * 12, 12 * sizeof(ocplx));
    mr_local(d, b, blk, U, T, kappa, (const ocplx(*)[16])G, n_mr, rl, dl);
    for (long l = 0; l < bv; ++l)
        memcpy(delta + block_site(d, b, blk, l) * 12, dl + l * 12, 12 * sizeof(ocplx));
    free(rl);
    free(dl);
}

/* --------------------------------------------------------------------- SAP */

/* For every block B of colour c (blocks of one colour share no hopping terms,
 * so their updates are independent):  r_B = b_B - (D x)_B with the full D,
 * delta = MR(D_BB, r_B, n_mr), x_B += delta.  Cycles alternate colour 0 then
 * colour 1 (multiplicative Schwarz, paper Section 2). */
void or_sap(const int d[4], const int b[4], const ocplx* U, const ocplx* T, double kappa,
            int n_cy, int n_mr, const ocplx* bsrc, ocplx* x) {
    long nblk = or_num_blocks(d, b), bv = vol4(b);
    ocplx G[4][16];
    load_gammas(G);
    for (int cy = 0; cy < n_cy; ++cy)
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for num_threads(g_threads) schedule(dynamic)
            for (long blk = 0; blk < nblk; ++blk) {
                if (or_block_colour(d, b, blk) != colour) continue;
                ocplx* rl = malloc(sizeof(ocplx) * 12 * bv);
                ocplx* dl = malloc(sizeof(ocplx) * 12 * bv);
                for (long l = 0; l < bv; ++l) {
                    long s = block_site(d, b, blk, l);
                    ocplx hop[12], dx[12];
                    hop_site(d, U, (const ocplx(*)[16])G, x, s, NULL, NULL, hop);
                    d_site(T ? T + s * 144 : NULL, kappa, x + s * 12, hop, dx);
                    for (int i = 0; i < 12; ++i) rl[l * 12 + i] = bsrc[s * 12 + i] - dx[i];
                }
                mr_local(d, b, blk, U, T, kappa, (const ocplx(*)[16])G, n_mr, rl, dl);
                for (long l = 0; l < bv; ++l) {
                    long s = block_site(d, b, blk, l);
                    for (int i = 0; i < 12; ++i) x[s * 12 + i] += dl[l * 12 + i];
                }
                free(rl);
                free(dl);
            }
        }
}

/* ------------------------------------------- SAP with Jacobi block solves */

/* Inverse of C = 1 + T(x) (12 x 12) by Gauss-Jordan elimination with
 * partial pivoting. */
void or_clover_inverse_site(const ocplx* Tx, ocplx* Cinv) {
    ocplx a[12][24];
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) {
            a[i][j] = (Tx ? Tx[i * 12 + j] : 0) + (i == j ? 1.0 : 0.0);
            a[i][12 + j] = i == j ? 1.0 : 0.0;
        }
    for (int c = 0; c < 12; ++c) {
        int piv = c;
        for (int i = c + 1; i < 12; ++i)
            if (cabs(a[i][c]) > cabs(a[piv][c])) piv = i;
        if (piv != c)
            for (int j = 0; j < 24; ++j) {
                ocplx t = a[c][j];
                a[c][j] = a[piv][j];
                a[piv][j] = t;
            }
        ocplx inv = 1.0 / a[c][c];
        for (int j = 0; j < 24; ++j) a[c][j] *= inv;
        for (int i = 0; i < 12; ++i) {
            if (i == c) continue;
            ocplx f = a[i][c];
            if (f == 0) continue;
            for (int j = 0; j < 24; ++j) a[i][j] -= f * a[c][j];
        }
    }
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) Cinv[i * 12 + j] = a[i][12 + j];
}

void or_clover_inverse_field(const int d[4], const ocplx* T, ocplx* Cinv) {
    long V = vol4(d);
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (long x = 0; x < V; ++x) or_clover_inverse_site(T ? T + x * 144 : NULL, Cinv + x * 144);
}

static void m12_apply(const ocplx* M, const ocplx* v, ocplx* out) {
    for (int i = 0; i < 12; ++i) {
        ocplx t = 0;
        for (int j = 0; j < 12; ++j) t += M[i * 12 + j] * v[j];
        out[i] = t;
    }
}

/* Jacobi on the block system A_BB delta = rho of A = C^-1 D (local arrays):
 * delta = 0, then n_jac times delta += rho - C^-1 D_BB delta.  ci holds
 * C^-1 of the block's sites. */
static void jacobi_local(const int d[4], const int b[4], long blk, const ocplx* U, const ocplx* T,
                         double kappa, const ocplx G[4][16], int n_jac, const ocplx* ci,
                         const ocplx* rho, ocplx* dl) {
    long bv = vol4(b);
    ocplx* q = malloc(sizeof(ocplx) * 12 * bv);
    memset(dl, 0, sizeof(ocplx) * 12 * bv);
    for (int it = 0; it < n_jac; ++it) {
        dbb_local(d, b, blk, U, T, kappa, G, dl, q);  /* D_BB delta */
        for (long l = 0; l < bv; ++l) {
            ocplx aq[12];
            m12_apply(ci + l * 144, q + l * 12, aq);   /* A_BB delta */
            for (int i = 0; i < 12; ++i) dl[l * 12 + i] += rho[l * 12 + i] - aq[i];
        }
    }
    free(q);
}

/* The block solve of the Jacobi smoother for one block: delta_B for the
 * block residual r_B of D (rho = C^-1 r_B), full-lattice arrays r, delta. */
void or_jacobi_block(const int d[4], const int b[4], long blk, const ocplx* U, const ocplx* T,
                     double kappa, int n_jac, const ocplx* r, ocplx* delta) {
    long bv = vol4(b);
    ocplx G[4][16];
    load_gammas(G);
    ocplx* ci = malloc(sizeof(ocplx) * 144 * bv);
    ocplx* rho = malloc(sizeof(ocplx) * 12 * bv);
    ocplx* dl = malloc(sizeof(ocplx) * 12 * bv);
    for (long l = 0; l < bv; ++l) {
        long s = block_site(d, b, blk, l);
        or_clover_inverse_site(T ? T + s * 144 : NULL, ci + l * 144);
        m12_apply(ci + l * 144, r + s * 12, rho + l * 12);
    }
    jacobi_local(d, b, blk, U, T, kappa, (const ocplx(*)[16])G, n_jac, ci, rho, dl);
    for (long l = 0; l < bv; ++l)
        memcpy(delta + block_site(d, b, blk, l) * 12, dl + l * 12, 12 * sizeof(ocplx));
    free(ci);
    free(rho);
    free(dl);
}

/* The smoother of QWS (paper Section 2): multiplicative SAP for the
 * clover-preconditioned operator A = C^-1 D, each block system A_BB delta =
 * rho solved by n_jac Jacobi steps (A_BB has the identity on its diagonal):
 * delta = 0, then n_jac times delta += rho - A_BB delta.  For a right-hand
 * side b of D x = b the block residual is rho = C^-1 (b - D x)_B (C is site
 * diagonal, so A x = C^-1 b is D x = b).  Same colouring and order as
 * or_sap. */
void or_sap_jacobi(const int d[4], const int b[4], const ocplx* U, const ocplx* T, double kappa,
                   int n_cy, int n_jac, const ocplx* bsrc, ocplx* x) {
    long nblk = or_num_blocks(d, b), bv = vol4(b);
    ocplx G[4][16];
    load_gammas(G);
    for (int cy = 0; cy < n_cy; ++cy)
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for num_threads(g_threads) schedule(dynamic)
            for (long blk = 0; blk < nblk; ++blk) {
                if (or_block_colour(d, b, blk) != colour) continue;
                ocplx* rho = malloc(sizeof(ocplx) * 12 * bv);
                ocplx* dl = malloc(sizeof(ocplx) * 12 * bv);
                ocplx* ci = malloc(sizeof(ocplx) * 144 * bv);
                for (long l = 0; l < bv; ++l) {
                    long s = block_site(d, b, blk, l);
                    ocplx hop[12], dx[12];
                    hop_site(d, U, (const ocplx(*)[16])G, x, s, NULL, NULL, hop);
                    d_site(T ? T + s * 144 : NULL, kappa, x + s * 12, hop, dx);
                    for (int i = 0; i < 12; ++i) dx[i] = bsrc[s * 12 + i] - dx[i];
                    or_clover_inverse_site(T ? T + s * 144 : NULL, ci + l * 144);
                    m12_apply(ci + l * 144, dx, rho + l * 12);
                }
                jacobi_local(d, b, blk, U, T, kappa, (const ocplx(*)[16])G, n_jac, ci, rho, dl);
                for (long l = 0; l < bv; ++l) {
                    long s = block_site(d, b, blk, l);
                    for (int i = 0; i < 12; ++i) x[s * 12 + i] += dl[l * 12 + i];
                }
                free(rho); free(dl); free(ci);
            }
        }
}

/* ------------------------------------------------- even-odd block MR (SAP) */

/* Global parity (x + y + z + t) mod 2 of site s; every hop joins opposite
 * parities. */
static int site_parity(const int d[4], long s) {
    int c[4];
    site_coords(d, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* Even-odd preconditioned MR on the Dirichlet block operator (local arrays).
 * With the block's sites split by parity, D_BB = [[C_e, -k H_eo],
 * [-k H_oe, C_o]] (C site diagonal); the Schur complement on the even sites
 * is S = C_e - k^2 H_eo C_o^-1 H_oe.  The block system D_BB delta = r becomes
 *   S delta_e = r_e + k H_eo C_o^-1 r_o,   delta_o = C_o^-1 (r_o + k H_oe delta_e),
 * and S delta_e = rhat_e is solved by n_mr MR steps from delta_e = 0 (as
 * mr_local, on vectors that vanish on the odd sites).  Every product with the
 * off-diagonal blocks is taken from D_BB itself: for u vanishing on the even
 * sites (D_BB u)_e = -k H_eo u_o; for v vanishing on the odd sites
 * (D_BB v)_o = -k H_oe v_e, so S v_e = [D_BB (v_e, -C_o^-1 (D_BB v)_o)]_e.
 * ci holds C^-1 of the block's sites, par their parities. */
static void eo_mr_local(const int d[4], const int b[4], long blk, const ocplx* U, const ocplx* T,
                        double kappa, const ocplx G[4][16], int n_mr, const ocplx* ci, const int* par,
                        const ocplx* r_l, ocplx* delta_l) {
    long bv = vol4(b), n = bv * 12;
    ocplx* rho = malloc(sizeof(ocplx) * n);
    ocplx* t = malloc(sizeof(ocplx) * n);
    ocplx* w = malloc(sizeof(ocplx) * n);
    ocplx* q = malloc(sizeof(ocplx) * n);
    /* rhat_e = r_e - (D_BB (0, C_o^-1 r_o))_e */
    for (long l = 0; l < bv; ++l) {
        if (par[l]) m12_apply(ci + l * 144, r_l + l * 12, t + l * 12);
        else memset(t + l * 12, 0, 12 * sizeof(ocplx));
    }
    dbb_local(d, b, blk, U, T, kappa, G, t, w);
    for (long l = 0; l < bv; ++l)
        for (int i = 0; i < 12; ++i) rho[l * 12 + i] = par[l] ? 0 : r_l[l * 12 + i] - w[l * 12 + i];
    memset(delta_l, 0, sizeof(ocplx) * n);
    for (int it = 0; it < n_mr; ++it) {
        /* q = S rho (rho vanishes on the odd sites) */
        dbb_local(d, b, blk, U, T, kappa, G, rho, w);
        for (long l = 0; l < bv; ++l) {
            if (par[l]) {
                ocplx u[12];
                m12_apply(ci + l * 144, w + l * 12, u);
                for (int i = 0; i < 12; ++i) t[l * 12 + i] = -u[i];
            } else {
                memcpy(t + l * 12, rho + l * 12, 12 * sizeof(ocplx));
            }
        }
        dbb_local(d, b, blk, U, T, kappa, G, t, q);
        for (long l = 0; l < bv; ++l)
            if (par[l]) memset(q + l * 12, 0, 12 * sizeof(ocplx));
        double qq = vnorm2(n, q);
        if (qq == 0.0) break;
        ocplx alpha = vdot(n, q, rho) / qq;
        for (long i = 0; i < n; ++i) {
            delta_l[i] += alpha * rho[i];
            rho[i] -= alpha * q[i];
        }
    }
    /* delta_o = C_o^-1 (r_o - (D_BB (delta_e, 0))_o) */
    dbb_local(d, b, blk, U, T, kappa, G, delta_l, w);
    for (long l = 0; l < bv; ++l)
        if (par[l]) {
            ocplx u[12];
            for (int i = 0; i < 12; ++i) u[i] = r_l[l * 12 + i] - w[l * 12 + i];
            m12_apply(ci + l * 144, u, delta_l + l * 12);
        }
    free(rho); free(t); free(w); free(q);
}

static void eo_block_tables(const int d[4], const int b[4], long blk, const ocplx* T, ocplx* ci, int* par) {
    for (long l = 0; l < vol4(b); ++l) {
        long s = block_site(d, b, blk, l);
        or_clover_inverse_site(T ? T + s * 144 : NULL, ci + l * 144);
        par[l] = site_parity(d, s);
    }
}

/* The even-odd block solve for one block: delta_B for the block residual r_B
 * (full-lattice arrays r, delta). */
void or_mr_eo_block(const int d[4], const int b[4], long blk, const ocplx* U, const ocplx* T,
                    double kappa, int n_mr, const ocplx* r, ocplx* delta) {
    long bv = vol4(b);
    ocplx G[4][16];
    load_gammas(G);
    ocplx* ci = malloc(sizeof(ocplx) * 144 * bv);
    int* par = malloc(sizeof(int) * bv);
    ocplx* rl = malloc(sizeof(ocplx) * 12 * bv);
    ocplx* dl = malloc(sizeof(ocplx) * 12 * bv);
    eo_block_tables(d, b, blk, T, ci, par);
    for (long l = 0; l < bv; ++l) memcpy(rl + l * 12, r + block_site(d, b, blk, l) * 12, 12 * sizeof(ocplx));
    eo_mr_local(d, b, blk, U, T, kappa, (const ocplx(*)[16])G, n_mr, ci, par, rl, dl);
    for (long l = 0; l < bv; ++l) memcpy(delta + block_site(d, b, blk, l) * 12, dl + l * 12, 12 * sizeof(ocplx));
    free(ci); free(par); free(rl); free(dl);
}

/* SAP as or_sap with the even-odd preconditioned block solve. */
void or_sap_eo(const int d[4], const int b[4], const ocplx* U, const ocplx* T, double kappa,
               int n_cy, int n_mr, const ocplx* bsrc, ocplx* x) {
    long nblk = or_num_blocks(d, b), bv = vol4(b);
    ocplx G[4][16];
    load_gammas(G);
    for (int cy = 0; cy < n_cy; ++cy)
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for num_threads(g_threads) schedule(dynamic)
            for (long blk = 0; blk < nblk; ++blk) {
                if (or_block_colour(d, b, blk) != colour) continue;
                ocplx* rl = malloc(sizeof(ocplx) * 12 * bv);
                ocplx* dl = malloc(sizeof(ocplx) * 12 * bv);
                ocplx* ci = malloc(sizeof(ocplx) * 144 * bv);
                int* par = malloc(sizeof(int) * bv);
                eo_block_tables(d, b, blk, T, ci, par);
                for (long l = 0; l < bv; ++l) {
                    long s = block_site(d, b, blk, l);
                    ocplx hop[12], dx[12];
                    hop_site(d, U, (const ocplx(*)[16])G, x, s, NULL, NULL, hop);
                    d_site(T ? T + s * 144 : NULL, kappa, x + s * 12, hop, dx);
                    for (int i = 0; i < 12; ++i) rl[l * 12 + i] = bsrc[s * 12 + i] - dx[i];
                }
                eo_mr_local(d, b, blk, U, T, kappa, (const ocplx(*)[16])G, n_mr, ci, par, rl, dl);
                for (long l = 0; l < bv; ++l) {
                    long s = block_site(d, b, blk, l);
                    for (int i = 0; i < 12; ++i) x[s * 12 + i] += dl[l * 12 + i];
                }
                free(rl); free(dl); free(ci); free(par);
            }
        }
}

/* -------------------------------------------------------------------- FGCR */

int or_fgcr(const int d[4], const int b[4], const ocplx* U, const ocplx* T, double kappa,
            int n_cy, int n_mr, int m, double tol, int max_iter, const ocplx* bsrc,
            ocplx* x, int* iters_out, double* relres_out, double* hist) {
    long V = vol4(d), n = V * 12;
    ocplx* r = malloc(sizeof(ocplx) * n);
    ocplx* t = malloc(sizeof(ocplx) * n);
    ocplx* Z = malloc(sizeof(ocplx) * n * m);
    ocplx* W = malloc(sizeof(ocplx) * n * m);
    ocplx* R = calloc((size_t)m * m, sizeof(ocplx));
    ocplx* c = calloc((size_t)m, sizeof(ocplx));
    ocplx* gam = calloc((size_t)m, sizeof(ocplx));
    int status = 1, iters = 0;
    double bnorm = sqrt(vnorm2(n, bsrc)), rel = 0;

    if (bnorm == 0.0) { /* D x = 0 has the unique solution x = 0 */
        memset(x, 0, sizeof(ocplx) * n);
        status = 0;
        if (hist) hist[0] = 0;
        goto done;
    }
    or_apply_D(d, U, T, kappa, x, t);
    for (long i = 0; i < n; ++i) r[i] = bsrc[i] - t[i];
    rel = sqrt(vnorm2(n, r)) / bnorm;
    if (hist) hist[0] = rel;
    for (;;) {
        if (rel <= tol) { status = 0; break; }
        if (iters >= max_iter) { status = 1; break; }
        int k_used = 0;
        for (int k = 0; k < m; ++k) {
            ocplx* z = Z + (long)k * n;
            ocplx* w = W + (long)k * n;
            if (n_cy > 0) {
                memset(z, 0, sizeof(ocplx) * n);
                or_sap(d, b, U, T, kappa, n_cy, n_mr, r, z);
            } else {
                memcpy(z, r, sizeof(ocplx) * n);
            }
            or_apply_D(d, U, T, kappa, z, w);
            /* modified Gram-Schmidt against the previous normalised w_j */
            for (int j = 0; j < k; ++j) {
                const ocplx* wj = W + (long)j * n;
                ocplx beta = vdot(n, wj, w);
                R[j * m + k] = beta;
                for (long i = 0; i < n; ++i) w[i] -= beta * wj[i];
            }
            double nu = sqrt(vnorm2(n, w));
            if (nu == 0.0) { status = 2; goto done; }
            R[k * m + k] = nu;
            for (long i = 0; i < n; ++i) w[i] /= nu;
            c[k] = vdot(n, w, r);
            for (long i = 0; i < n; ++i) r[i] -= c[k] * w[i];
            ++iters;
            k_used = k + 1;
            double rr = sqrt(vnorm2(n, r)) / bnorm;
            if (hist) hist[iters] = rr;
            if (rr <= tol || iters >= max_iter) break;
        }
        /* back substitution R gamma = c, then x += sum gamma_k z_k */
        for (int k = k_used - 1; k >= 0; --k) {
            ocplx s = c[k];
            for (int j = k + 1; j < k_used; ++j) s -= R[k * m + j] * gam[j];
            gam[k] = s / R[k * m + k];
        }
        for (int k = 0; k < k_used; ++k) {
            const ocplx* z = Z + (long)k * n;
            for (long i = 0; i < n; ++i) x[i] += gam[k] * z[i];
        }
        /* true residual */
        or_apply_D(d, U, T, kappa, x, t);
        for (long i = 0; i < n; ++i) r[i] = bsrc[i] - t[i];
        rel = sqrt(vnorm2(n, r)) / bnorm;
    }
done:
    if (iters_out) *iters_out = iters;
    if (relres_out) *relres_out = rel;
    free(r); free(t); free(Z); free(W); free(R); free(c); free(gam);
    return status;
}

/* --------------------------------------------------------------- BiCGStab */

/* Flexible BiCGStab with the SAP preconditioner on the right (the outer
 * solver of the paper's multigrid code, Section 3; flexible because SAP with
 * MR is not a fixed linear map), FP64.  z = M v means n_cy SAP cycles from
 * zero on v (z = v when n_cy = 0).  One iteration:
 *   rho' = <rh, r>;  beta = (rho' / rho)(alpha / omega);  p = r + beta (p - omega v)
 *   ph = M p;  v = D ph;  alpha = rho' / <rh, v>;  s = r - alpha v
 *   sh = M s;  t = D sh;  omega = <t, s> / <t, t>
 *   x += alpha ph + omega sh;  r = s - omega t;  rho = rho'
 * The recursive residual r stops the iteration at tol ||b|| or, when delta >
 * 0, once it falls below delta times the last true residual; then the true
 * residual b - D x is recomputed and, unless it meets tol, the iteration
 * restarts from the current x with rh = r, p = v = 0, rho = alpha = omega = 1.
 * A zero <rh, v>, <t, t> or omega also restarts; a restart whose true
 * residual has not decreased since the previous one is a breakdown.
 * hist[k] = recursive relative residual after iteration k (hist[0] the
 * initial true one).  Returns 0 converged, 1 iteration cap, 2 breakdown. */
int or_fbicgstab(const int d[4], const int b[4], const ocplx* U, const ocplx* T, double kappa,
                 int n_cy, int n_mr, double tol, int max_iter, double delta, const ocplx* bsrc,
                 ocplx* x, int* iters_out, int* restarts_out, double* relres_out, double* hist) {
    long n = vol4(d) * 12;
    ocplx *r = malloc(sizeof(ocplx) * n), *rh = malloc(sizeof(ocplx) * n);
    ocplx *p = malloc(sizeof(ocplx) * n), *v = malloc(sizeof(ocplx) * n);
    ocplx *s = malloc(sizeof(ocplx) * n), *t = malloc(sizeof(ocplx) * n);
    ocplx *ph = malloc(sizeof(ocplx) * n), *sh = malloc(sizeof(ocplx) * n);
    int status = 1, iters = 0, restarts = 0;
    double bnorm = sqrt(vnorm2(n, bsrc)), rel = 0, last_true = 0;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(ocplx) * n);
        status = 0;
        if (hist) hist[0] = 0;
        goto done;
    }
    for (;;) {
        /* (re)start: true residual */
        or_apply_D(d, U, T, kappa, x, t);
        for (long i = 0; i < n; ++i) r[i] = bsrc[i] - t[i];
        double rt = sqrt(vnorm2(n, r));
        rel = rt / bnorm;
        if (iters == 0 && hist) hist[0] = rel;
        if (rel <= tol) { status = 0; break; }
        if (iters >= max_iter) { status = 1; break; }
        if (iters > 0 && !(rt < last_true)) { status = 2; break; }
        if (iters > 0) ++restarts;
        last_true = rt;
        memcpy(rh, r, sizeof(ocplx) * n);
        memset(p, 0, sizeof(ocplx) * n);
        memset(v, 0, sizeof(ocplx) * n);
        ocplx rho = 1, alpha = 1, omega = 1;
        while (iters < max_iter) {
            ocplx rho_new = vdot(n, rh, r);
            ocplx beta = (rho_new / rho) * (alpha / omega);
            for (long i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            if (n_cy > 0) {
                memset(ph, 0, sizeof(ocplx) * n);
                or_sap(d, b, U, T, kappa, n_cy, n_mr, p, ph);
            } else {
                memcpy(ph, p, sizeof(ocplx) * n);
            }
            or_apply_D(d, U, T, kappa, ph, v);
            ocplx rv = vdot(n, rh, v);
            if (rv == 0) break;
            alpha = rho_new / rv;
            for (long i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
            if (n_cy > 0) {
                memset(sh, 0, sizeof(ocplx) * n);
                or_sap(d, b, U, T, kappa, n_cy, n_mr, s, sh);
            } else {
                memcpy(sh, s, sizeof(ocplx) * n);
            }
            or_apply_D(d, U, T, kappa, sh, t);
            double tt = vnorm2(n, t);
            omega = tt > 0 ? vdot(n, t, s) / tt : 0;
            for (long i = 0; i < n; ++i) {
                x[i] += alpha * ph[i] + omega * sh[i];
                r[i] = s[i] - omega * t[i];
            }
            rho = rho_new;
            ++iters;
            double rr = sqrt(vnorm2(n, r));
            if (hist) hist[iters] = rr / bnorm;
            if (rr <= tol * bnorm || omega == 0 || (delta > 0 && rr < delta * last_true)) break;
        }
    }
done:
    if (iters_out) *iters_out = iters;
    if (restarts_out) *restarts_out = restarts;
    if (relres_out) *relres_out = rel;
    free(r); free(rh); free(p); free(v); free(s); free(t); free(ph); free(sh);
    return status;
}

/* The scheme the paper's Section 2 describes for QWS: a Richardson
 * iteration in double precision around an inner BiCGStab solve.  Each outer
 * step recomputes r = b - D x, solves D e = r / |r| with the flexible
 * BiCGStab above to the relative tolerance inner_tol (from e = 0, no
 * reliable restarts), and sets x += |r| e.  Stops when the true residual
 * meets tol; an outer step without progress is a breakdown.  iters counts
 * inner BiCGStab iterations, outer the Richardson steps taken. */
int or_richardson_bicgstab(const int d[4], const int b[4], const ocplx* U, const ocplx* T, double kappa,
                           int n_cy, int n_mr, double tol, int max_iter, double inner_tol,
                           const ocplx* bsrc, ocplx* x, int* iters_out, int* outer_out,
                           double* relres_out) {
    long n = vol4(d) * 12;
    ocplx *r = malloc(sizeof(ocplx) * n), *e = malloc(sizeof(ocplx) * n);
    int status = 1, iters = 0, outer = 0;
    double bnorm = sqrt(vnorm2(n, bsrc)), rel = 0, last = 0;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(ocplx) * n);
        status = 0;
        goto done;
    }
    for (;;) {
        or_apply_D(d, U, T, kappa, x, r);
        for (long i = 0; i < n; ++i) r[i] = bsrc[i] - r[i];
        double rt = sqrt(vnorm2(n, r));
        rel = rt / bnorm;
        if (rel <= tol) { status = 0; break; }
        if (iters >= max_iter) { status = 1; break; }
        if (outer > 0 && !(rt < last)) { status = 2; break; }
        last = rt;
        for (long i = 0; i < n; ++i) r[i] /= rt;
        memset(e, 0, sizeof(ocplx) * n);
        int it = 0, rs = 0;
        double rr = 0;
        or_fbicgstab(d, b, U, T, kappa, n_cy, n_mr, inner_tol, max_iter - iters, 0.0, r, e, &it, &rs, &rr,
                     NULL);
        iters += it;
        ++outer;
        for (long i = 0; i < n; ++i) x[i] += rt * e[i];
    }
done:
    if (iters_out) *iters_out = iters;
    if (outer_out) *outer_out = outer;
    if (relres_out) *relres_out = rel;
    free(r);
    free(e);
    return status;
}

/* -------------------------------------------------------------------- force */

/* tr(A B) for 3x3 */
static ocplx m3_trace_prod(const ocplx* a, const ocplx* b) {
    ocplx s = 0;
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) s += a[i * 3 + k] * b[k * 3 + i];
    return s;
}

/* y^dag (sigma (x) F) x summed over spin and colour, with x, y one site. */
static ocplx sandwich(const ocplx sg[16], const ocplx F[9], const ocplx* y, const ocplx* x) {
    ocplx s = 0;
    for (int si = 0; si < 4; ++si)
        for (int sj = 0; sj < 4; ++sj) {
            if (sg[si * 4 + sj] == 0) continue;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    s += conj(y[3 * si + a]) * sg[si * 4 + sj] * F[a * 3 + b] * x[3 * sj + b];
        }
    return s;
}

void or_force(const int d[4], const ocplx* U, double kappa, double csw, const ocplx* x,
              const ocplx* y, double* g_hop, double* g_clov) {
    long V = vol4(d);
    ocplx G[4][16], Ta[8][9];
    load_gammas(G);
    for (int a = 0; a < 8; ++a) or_su3_generator(a, Ta[a]);

    if (g_hop) {
        /* The link U_mu(x) enters D at row x (forward hop, (1 - gamma_mu)) and at
         * row x+mu (backward hop, (1 + gamma_mu), as U^dag).  With
         * dU = i w T^a U and dU^dag = -i w U^dag T^a:
         *   dL/dw = -Re(y^dag dD x)
         *         = -kappa Im tr[T^a (U X1 - X2 U^dag)],
         *   X1 = sum_spin [(1 - gamma_mu) x(x+mu)] (x) y(x)^dag,
         *   X2 = sum_spin [(1 + gamma_mu) x(x)] (x) y(x+mu)^dag. */
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (long s = 0; s < V; ++s)
            for (int mu = 0; mu < 4; ++mu) {
                long sp = site_step(d, s, mu, +1);
                ocplx pm[12], pp[12];
                for (int si = 0; si < 4; ++si)
                    for (int a = 0; a < 3; ++a) {
                        ocplx gm = 0, gp = 0;
                        for (int sj = 0; sj < 4; ++sj) {
                            gm += G[mu][si * 4 + sj] * x[sp * 12 + 3 * sj + a];
                            gp += G[mu][si * 4 + sj] * x[s * 12 + 3 * sj + a];
                        }
                        pm[3 * si + a] = x[sp * 12 + 3 * si + a] - gm;
                        pp[3 * si + a] = x[s * 12 + 3 * si + a] + gp;
                    }
                ocplx X1[9], X2[9], A[9], B[9], Ud[9], M[9];
                for (int a = 0; a < 3; ++a)
                    for (int bb = 0; bb < 3; ++bb) {
                        ocplx s1 = 0, s2 = 0;
                        for (int si = 0; si < 4; ++si) {
                            s1 += pm[3 * si + a] * conj(y[s * 12 + 3 * si + bb]);
                            s2 += pp[3 * si + a] * conj(y[sp * 12 + 3 * si + bb]);
                        }
                        X1[a * 3 + bb] = s1;
                        X2[a * 3 + bb] = s2;
                    }
                m3_mul(link_at(U, s, mu), X1, A);
                m3_dag(link_at(U, s, mu), Ud);
                m3_mul(X2, Ud, B);
                for (int i = 0; i < 9; ++i) M[i] = A[i] - B[i];
                for (int a = 0; a < 8; ++a)
                    g_hop[(s * 4 + mu) * 8 + a] = -kappa * cimag(m3_trace_prod(Ta[a], M));
            }
    }

    if (g_clov) {
        /* dL/dw = -Re sum_z y(z)^dag (dT(z)/dw) x(z), with
         * dT = i kappa c_sw sigma_{mu nu} (x) (dQ - dQ^dag)/8 and dQ the leaf
         * sum with one factor differentiated (product rule): U -> i T^a U,
         * U^dag -> -i U^dag T^a.  Literal loop over sites z, planes, leaves,
         * factors; every (leaf, factor) adds to the link it names.  The
         * contributions are accumulated per site z and scattered serially. */
        memset(g_clov, 0, sizeof(double) * V * 32);
        double* contrib = malloc(sizeof(double) * V * 6 * 4 * 4 * 8);
        long* target = malloc(sizeof(long) * V * 6 * 4 * 4);
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (long z = 0; z < V; ++z) {
            int plane = 0;
            for (int mu = 0; mu < 4; ++mu)
                for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
                    ocplx sg[16];
                    or_sigma(mu, nu, sg);
                    for (int l = 0; l < 4; ++l) {
                        ocplx fac[4][9];
                        for (int f = 0; f < 4; ++f) leaf_factor_matrix(d, U, z, mu, nu, l, f, fac[f]);
                        for (int f = 0; f < 4; ++f) {
                            long ls;
                            int ldir;
                            leaf_link(d, z, mu, nu, l, f, &ls, &ldir);
                            long slot = ((z * 6 + plane) * 4 + l) * 4 + f;
                            target[slot] = ls * 4 + ldir;
                            for (int a = 0; a < 8; ++a) {
                                ocplx dfac[9], P[9], dF[9];
                                if (LEAVES[l][f].dag) { /* -i U^dag T^a */
                                    m3_mul(fac[f], Ta[a], dfac);
                                    for (int i = 0; i < 9; ++i) dfac[i] *= -I_;
                                } else { /* i T^a U */
                                    m3_mul(Ta[a], fac[f], dfac);
                                    for (int i = 0; i < 9; ++i) dfac[i] *= I_;
                                }
                                m3_unit(P);
                                for (int g = 0; g < 4; ++g) m3_mul(P, g == f ? dfac : fac[g], P);
                                for (int i = 0; i < 3; ++i)
                                    for (int j = 0; j < 3; ++j)
                                        dF[i * 3 + j] = (P[i * 3 + j] - conj(P[j * 3 + i])) / 8.0;
                                ocplx v = I_ * kappa * csw * sandwich(sg, dF, y + z * 12, x + z * 12);
                                contrib[slot * 8 + a] = -creal(v);
                            }
                        }
                    }
                }
        }
        for (long slot = 0; slot < V * 96; ++slot)
            for (int a = 0; a < 8; ++a) g_clov[target[slot] * 8 + a] += contrib[slot * 8 + a];
        free(contrib);
        free(target);
    }
}
