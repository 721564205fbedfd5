/*
 * oracle.c -- plain, slow, FP64 CPU reference for the Wilson hopping matrix,
 * the even-odd preconditioned twisted-mass operator and CG on it.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP path under paper_1311_4521_amd/.
 *
 * The paper (Deuzeman, Jansen, Kostrzewa, Urbach, "Experiences with OpenMP in
 * tmLQCD", LATTICE 2013) names the operator -- the hopping matrix
 * Hopping_Matrix between the two checkerboards (Section 2, "Performance
 * Measurements" and the introduction) and the twisted-mass Wilson fermions it
 * is used for (introduction) -- but never writes it down.  Every formula below
 * is the standard definition, taken in the readings listed here:
 *
 *   Lattice   Z_T x Z_LX x Z_LY x Z_LZ, mu = 0..3 = t,x,y,z, all extents even
 *             and >= 2.  lex = ((t*LX + x)*LY + y)*LZ + z, parity
 *             (t+x+y+z) mod 2.  The even-odd index of a site is the number of
 *             sites of the same parity that precede it in lex order; this file
 *             builds that map by enumeration.
 *   Gammas    chiral basis, written out as 4x4 tables below; gamma_5 is formed
 *             here as the product gamma_0 gamma_1 gamma_2 gamma_3.
 *   Hopping   (H psi)(x) = kappa sum_mu [ eta+ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                       + eta- (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *             eta+ = exp(+i pi theta_mu) when the forward hop wraps from
 *             L_mu - 1 to 0, eta- = exp(-i pi theta_mu) when the backward hop
 *             wraps from 0 to L_mu - 1, 1 otherwise.  H_eo: odd -> even,
 *             H_oe: even -> odd.  When L_mu = 2 both terms reach the same site
 *             and both are added.
 *   Twisted   A(s) = 1 + i s mt gamma_5 with mt = 2 kappa mu, s = +-1;
 *   mass      Mhat(s) = A(s) - H_oe A(s)^-1 H_eo on odd fields,
 *             Qhat(s) = gamma_5 Mhat(s).  A(s)^-1 = (1 - i s mt gamma_5)/(1 + mt^2)
 *             (gamma_5^2 = 1).
 *   Force     for L = Re <X, H Y>, a link varied as U -> exp(t Z) U with Z
 *             anti-Hermitian traceless changes L by t tr(Z TA(M)), where
 *             L = Re tr(U W) over the terms containing the link and M is the
 *             derivative matrix of each term (see link_matrix below);
 *             TA(M) = (M - M^+)/2 - tr(M - M^+)/6.  The Euclidean gradient
 *             G with dL = Re sum conj(G) dU, for U taken as a free complex
 *             matrix, is W^+ for a forward and W for a backward term.  The
 *             paper only names the "fermionic derivative" (Section 2, race
 *             conditions).
 *   CG        conjugate gradient on Qhat(+)^dagger Qhat(+) = Qhat(-) Qhat(+),
 *             stopped when |r|^2 <= tol^2 |b|^2, then the true residual
 *             b - A x is recomputed; if it is above tol, CG restarts from x
 *             (at most three restarts).
 *
 * Spin products use the dense 4x4 gamma matrices (no half-spinor projection).
 * Reductions use compensated (Kahan) summation.  Build: -O2 -ffp-contract=off.
 *
 * Layouts (all complex128, interleaved re/im):
 *   gauge   [4][V][3][3]   (mu, lex, row, column)
 *   spinor  [Vh][4][3]     (even-odd index, spin, colour) on one parity, or
 *           [V][4][3]      (lex, spin, colour) for the full-lattice routines.
 *
 * Return value of every entry point: 0 on success, -1 on bad arguments,
 * -2 on allocation failure, 1 from orc_cg when it did not converge.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

/* ------------------------------------------------------------------ gammas */

static cplx GAM[5][4][4]; /* gamma_0..gamma_3, gamma_5 */
static int gam_ready = 0;

static void gam_init(void)
{
    if (gam_ready) return;
    const cplx i = I;
    const cplx g0[4][4] = {{0, 0, -1, 0}, {0, 0, 0, -1}, {-1, 0, 0, 0}, {0, -1, 0, 0}};
    const cplx g1[4][4] = {{0, 0, 0, -i}, {0, 0, -i, 0}, {0, i, 0, 0}, {i, 0, 0, 0}};
    const cplx g2[4][4] = {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}};
    const cplx g3[4][4] = {{0, 0, -i, 0}, {0, 0, 0, i}, {i, 0, 0, 0}, {0, -i, 0, 0}};
    memcpy(GAM[0], g0, sizeof g0);
    memcpy(GAM[1], g1, sizeof g1);
    memcpy(GAM[2], g2, sizeof g2);
    memcpy(GAM[3], g3, sizeof g3);
    /* gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3 */
    cplx a[4][4], b[4][4];
    memcpy(a, GAM[0], sizeof a);
    for (int m = 1; m < 4; ++m) {
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                cplx s = 0;
                for (int k = 0; k < 4; ++k) s += a[r][k] * GAM[m][k][c];
                b[r][c] = s;
            }
        memcpy(a, b, sizeof a);
    }
    memcpy(GAM[4], a, sizeof a);
    gam_ready = 1;
}

/* Copies a gamma matrix out (index 0..3, or 4 for gamma_5); used by tests. */
void orc_gamma(int m, double* out)
{
    gam_init();
    if (m < 0 || m > 4) return;
    memcpy(out, GAM[m], sizeof(cplx) * 16);
}

/* ---------------------------------------------------------------- geometry */

typedef struct {
    int L[4];
    int64_t V, Vh;
    int32_t* eo_of_lex;   /* [V] even-odd index of each site            */
    int32_t* lex_of_eo;   /* [2][Vh] lex index of the i-th site of parity p */
} geom;

static int geom_init(geom* g, const int dims[4])
{
    memset(g, 0, sizeof *g);
    for (int m = 0; m < 4; ++m) {
        if (dims[m] < 2 || (dims[m] & 1)) return -1;
        g->L[m] = dims[m];
    }
    g->V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    g->Vh = g->V / 2;
    if (g->V > INT32_MAX) return -1;
    g->eo_of_lex = malloc(sizeof(int32_t) * g->V);
    g->lex_of_eo = malloc(sizeof(int32_t) * g->V);
    if (!g->eo_of_lex || !g->lex_of_eo) {
        free(g->eo_of_lex);
        free(g->lex_of_eo);
        return -2;
    }
    int64_t count[2] = {0, 0};
    int64_t lex = 0;
    for (int t = 0; t < g->L[0]; ++t)
        for (int x = 0; x < g->L[1]; ++x)
            for (int y = 0; y < g->L[2]; ++y)
                for (int z = 0; z < g->L[3]; ++z, ++lex) {
                    int p = (t + x + y + z) & 1;
                    g->eo_of_lex[lex] = (int32_t)count[p];
                    g->lex_of_eo[p * g->Vh + count[p]] = (int32_t)lex;
                    ++count[p];
                }
    return 0;
}

static void geom_free(geom* g)
{
    free(g->eo_of_lex);
    free(g->lex_of_eo);
}

static void coords(const geom* g, int64_t lex, int c[4])
{
    c[3] = (int)(lex % g->L[3]);
    lex /= g->L[3];
    c[2] = (int)(lex % g->L[2]);
    lex /= g->L[2];
    c[1] = (int)(lex % g->L[1]);
    c[0] = (int)(lex / g->L[1]);
}

static int64_t lex_at(const geom* g, const int c[4])
{
    return (((int64_t)c[0] * g->L[1] + c[1]) * g->L[2] + c[2]) * g->L[3] + c[3];
}

/* Neighbour of x in direction mu (dir = +1 forward, -1 backward); *wrapped is
 * set when the step crosses the lattice boundary. */
static int64_t neighbour(const geom* g, const int c[4], int mu, int dir, int* wrapped)
{
    int d[4] = {c[0], c[1], c[2], c[3]};
    d[mu] += dir;
    *wrapped = 0;
    if (d[mu] == g->L[mu]) { d[mu] = 0; *wrapped = 1; }
    if (d[mu] < 0) { d[mu] = g->L[mu] - 1; *wrapped = 1; }
    return lex_at(g, d);
}

/* ------------------------------------------------------------ hopping term */

/* The hopping term at one output site x (lex index), written into out[4][3].
 * psi(y) is found at in + 12*idx(y), with idx the even-odd map or identity. */
static void hop_site(const geom* g, int64_t x, cplx* out, const cplx* U, const cplx* in,
                     const int32_t* idx, double kappa, const double theta[4])
{
    int c[4];
    coords(g, x, c);
    cplx acc[4][3];
    memset(acc, 0, sizeof acc);
    for (int mu = 0; mu < 4; ++mu) {
        for (int dir = +1; dir >= -1; dir -= 2) {
            int wrapped;
            int64_t y = neighbour(g, c, mu, dir, &wrapped);
            cplx eta = 1.0;
            if (wrapped) eta = cexp(I * (dir * M_PI * theta[mu]));
            const cplx* psi = in + 12 * (idx ? (int64_t)idx[y] : y);
            /* forward: U_mu(x); backward: U_mu(x - mu)^dagger */
            const cplx* u = U + 9 * (mu * g->V + (dir > 0 ? x : y));
            cplx chi[4][3];
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a) {
                    cplx sum = 0;
                    for (int b = 0; b < 3; ++b) {
                        cplx ub = dir > 0 ? u[3 * a + b] : conj(u[3 * b + a]);
                        sum += ub * psi[3 * s + b];
                    }
                    chi[s][a] = sum;
                }
            /* (1 - gamma_mu) for the forward, (1 + gamma_mu) for the backward term */
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a) {
                    cplx sum = 0;
                    for (int r = 0; r < 4; ++r) {
                        cplx p = (s == r ? 1.0 : 0.0) - dir * GAM[mu][s][r];
                        sum += p * chi[r][a];
                    }
                    acc[s][a] += eta * sum;
                }
        }
    }
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) out[3 * s + a] = kappa * acc[s][a];
}

/* Hopping matrix between checkerboards.  dir = 0: H_eo (odd input, even
 * output); dir = 1: H_oe (even input, odd output). */
int orc_hop(const int dims[4], int dir, double* out, const double* gauge, const double* in,
            double kappa, const double theta[4])
{
    if (dir != 0 && dir != 1) return -1;
    gam_init();
    geom g;
    int st = geom_init(&g, dims);
    if (st) return st;
    const int pout = dir == 0 ? 0 : 1;
    const int32_t* lexs = g.lex_of_eo + pout * g.Vh;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g.Vh; ++i)
        hop_site(&g, lexs[i], (cplx*)out + 12 * i, (const cplx*)gauge, (const cplx*)in,
                 g.eo_of_lex, kappa, theta);
    geom_free(&g);
    return 0;
}

/* The same operator evaluated only at the listed output sites (even-odd
 * indices on the output parity); out has n*12 complex entries. */
int orc_hop_sites(const int dims[4], int dir, const int64_t* sites, int64_t n, double* out,
                  const double* gauge, const double* in, double kappa, const double theta[4])
{
    if (dir != 0 && dir != 1) return -1;
    gam_init();
    geom g;
    int st = geom_init(&g, dims);
    if (st) return st;
    const int pout = dir == 0 ? 0 : 1;
    for (int64_t k = 0; k < n; ++k)
        if (sites[k] < 0 || sites[k] >= g.Vh) { geom_free(&g); return -1; }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k)
        hop_site(&g, g.lex_of_eo[pout * g.Vh + sites[k]], (cplx*)out + 12 * k,
                 (const cplx*)gauge, (const cplx*)in, g.eo_of_lex, kappa, theta);
    geom_free(&g);
    return 0;
}

/* Full-lattice hopping term (lex-ordered spinors on all V sites). */
int orc_hop_full(const int dims[4], double* out, const double* gauge, const double* in,
                 double kappa, const double theta[4])
{
    gam_init();
    geom g;
    int st = geom_init(&g, dims);
    if (st) return st;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < g.V; ++x)
        hop_site(&g, x, (cplx*)out + 12 * x, (const cplx*)gauge, (const cplx*)in, NULL, kappa,
                 theta);
    geom_free(&g);
    return 0;
}

/* Lex index of each site of parity p, in even-odd order (n = Vh entries). */
int orc_eo_sites(const int dims[4], int p, int64_t* lex_out)
{
    geom g;
    int st = geom_init(&g, dims);
    if (st) return st;
    for (int64_t i = 0; i < g.Vh; ++i) lex_out[i] = g.lex_of_eo[(p & 1) * g.Vh + i];
    geom_free(&g);
    return 0;
}

/* ------------------------------------------------------------ twisted mass */

/* out = (c1 + c5 gamma_5) in, site by site, dense 4x4 spin product. */
static void spin_lincomb_g5(cplx* out, const cplx* in, int64_t nsites, cplx c1, cplx c5)
{
    gam_init();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nsites; ++i) {
        cplx tmp[12];
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) {
                cplx sum = c1 * in[12 * i + 3 * s + a];
                for (int r = 0; r < 4; ++r) sum += c5 * GAM[4][s][r] * in[12 * i + 3 * r + a];
                tmp[3 * s + a] = sum;
            }
        memcpy(out + 12 * i, tmp, sizeof tmp);
    }
}

/* Qhat(sign) in = gamma_5 [ A in - H_oe A^-1 H_eo in ] on odd fields. */
int orc_qtm(const int dims[4], double* out, const double* gauge, const double* in, double kappa,
            double mu, const double theta[4], int sign)
{
    if (sign != 1 && sign != -1) return -1;
    geom g;
    int st = geom_init(&g, dims);
    if (st) return st;
    const int64_t Vh = g.Vh;
    geom_free(&g);
    cplx* te = malloc(sizeof(cplx) * 12 * Vh);
    cplx* w = malloc(sizeof(cplx) * 12 * Vh);
    if (!te || !w) { free(te); free(w); return -2; }
    const double mt = 2.0 * kappa * mu * sign;
    const double D = 1.0 + mt * mt;
    st = orc_hop(dims, 0, (double*)te, gauge, in, kappa, theta);
    if (!st) {
        spin_lincomb_g5(te, te, Vh, 1.0 / D, -I * mt / D);         /* A^-1 */
        st = orc_hop(dims, 1, (double*)w, gauge, (const double*)te, kappa, theta);
    }
    if (!st) {
        const cplx* x = (const cplx*)in;
        spin_lincomb_g5(te, x, Vh, 1.0, I * mt);                      /* A in */
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < 12 * Vh; ++k) w[k] = te[k] - w[k];
        spin_lincomb_g5((cplx*)out, w, Vh, 0.0, 1.0);                 /* gamma_5 */
    }
    free(te);
    free(w);
    return st;
}

/* Full-lattice twisted-mass Wilson operator on lex-ordered spinors [V][4][3]:
 * out = (1 + i sign mt gamma_5) in - H in, the matrix whose even-odd Schur
 * complement is Mhat. */
int orc_full_operator(const int dims[4], double* out, const double* gauge, const double* in,
                      double kappa, double mu, const double theta[4], int sign)
{
    if (sign != 1 && sign != -1) return -1;
    geom g;
    int st = geom_init(&g, dims);
    if (st) return st;
    const int64_t V = g.V;
    geom_free(&g);
    cplx* h = malloc(sizeof(cplx) * 12 * V);
    if (!h) return -2;
    st = orc_hop_full(dims, (double*)h, gauge, in, kappa, theta);
    if (!st) {
        spin_lincomb_g5((cplx*)out, (const cplx*)in, V, 1.0, I * (2.0 * kappa * mu * sign));
        for (int64_t k = 0; k < 12 * V; ++k) ((cplx*)out)[k] -= h[k];
    }
    free(h);
    return st;
}

/* ----------------------------------------------------------- linear algebra */

/* Re <a, b> = Re sum conj(a_k) b_k, Kahan-compensated, serial. */
static double kahan_re_dot(const cplx* a, const cplx* b, int64_t n)
{
    double s = 0.0, c = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double term = creal(a[k]) * creal(b[k]) + cimag(a[k]) * cimag(b[k]);
        double y = term - c;
        double t = s + y;
        c = (t - s) - y;
        s = t;
    }
    return s;
}

double orc_re_dot(const double* a, const double* b, int64_t ncomplex)
{
    return kahan_re_dot((const cplx*)a, (const cplx*)b, ncomplex);
}

typedef struct {
    const int* dims;
    const double* gauge;
    double kappa, mu;
    const double* theta;
    cplx* tmp;
} normal_op;

/* y = Qhat(-) Qhat(+) x */
static int apply_normal(const normal_op* op, cplx* y, const cplx* x)
{
    int st = orc_qtm(op->dims, (double*)op->tmp, op->gauge, (const double*)x, op->kappa, op->mu,
                     op->theta, +1);
    if (st) return st;
    return orc_qtm(op->dims, (double*)y, op->gauge, (const double*)op->tmp, op->kappa, op->mu,
                   op->theta, -1);
}

/* CG on Qhat(+)^dagger Qhat(+) x = b.  x holds the initial guess on entry
 * (pass zeros for x0 = 0) and the solution on return.  iters counts the
 * operator applications inside the CG recursions. */
int orc_cg(const int dims[4], double* xd, const double* bd, const double* gauge, double kappa,
           double mu, const double theta[4], double tol, int max_iter, int* iters,
           double* true_rel_res)
{
    geom g;
    int st = geom_init(&g, dims);
    if (st) return st;
    const int64_t n = 12 * g.Vh;
    geom_free(&g);
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n),
         *q = malloc(sizeof(cplx) * n), *tmp = malloc(sizeof(cplx) * n);
    if (!r || !p || !q || !tmp) { free(r); free(p); free(q); free(tmp); return -2; }
    normal_op op = {dims, gauge, kappa, mu, theta, tmp};
    cplx* x = (cplx*)xd;
    const cplx* b = (const cplx*)bd;
    const double bb = kahan_re_dot(b, b, n);
    int it = 0, converged = 0;
    double rel = 0.0;
    if (bb == 0.0) {
        memset(x, 0, sizeof(cplx) * n);
        converged = 1;
    }
    for (int restart = 0; restart < 4 && !converged && !st; ++restart) {
        /* r = b - A x, p = r */
        st = apply_normal(&op, q, x);
        if (st) break;
        for (int64_t k = 0; k < n; ++k) { r[k] = b[k] - q[k]; p[k] = r[k]; }
        double rr = kahan_re_dot(r, r, n);
        while (rr > tol * tol * bb && it < max_iter) {
            st = apply_normal(&op, q, p);
            if (st) break;
            ++it;
            const double pq = kahan_re_dot(p, q, n);
            const double alpha = rr / pq;
            for (int64_t k = 0; k < n; ++k) {
                x[k] += alpha * p[k];
                r[k] -= alpha * q[k];
            }
            const double rr_new = kahan_re_dot(r, r, n);
            const double beta = rr_new / rr;
            rr = rr_new;
            for (int64_t k = 0; k < n; ++k) p[k] = r[k] + beta * p[k];
        }
        if (st) break;
        /* true residual */
        st = apply_normal(&op, q, x);
        if (st) break;
        for (int64_t k = 0; k < n; ++k) r[k] = b[k] - q[k];
        rel = sqrt(kahan_re_dot(r, r, n) / bb);
        if (rel <= tol) converged = 1;
        if (it >= max_iter) break;
    }
    if (iters) *iters = it;
    if (true_rel_res) *true_rel_res = rel;
    free(r); free(p); free(q); free(tmp);
    if (st) return st;
    return converged ? 0 : 1;
}

/* ---------------------------------------------------------------- force */

/* The derivative matrix of the one term of L = Re <X, H Y> that contains
 * the link U_mu(l).  H holds each link in exactly one term:
 *   l on the output parity: the forward term at x = l,
 *     Re X(x)^+ kappa eta+ (1 - gamma_mu) U Y(x+mu) = Re tr(U W),
 *     W = kappa eta+ sum_s phi_s X(x)_s^+, phi = (1 - gamma_mu) Y(x+mu);
 *     with U -> exp(tZ) U:  dL/dt = Re tr(Z U W)       -> M = U W;
 *     as a function of the free complex U, dL = Re sum conj(W^+) dU.
 *   l on the input parity: the backward term at x = l + mu,
 *     Re X(x)^+ kappa eta- (1 + gamma_mu) U^+ Y(l) = Re tr(U^+ W),
 *     W = kappa eta- sum_s phi_s X(x)_s^+, phi = (1 + gamma_mu) Y(l);
 *     U^+ -> U^+ exp(-tZ): dL/dt = -Re tr(Z W U^+)     -> M = -W U^+;
 *     as a function of the free complex U, dL = Re sum conj(W) dU.
 * X and Y are even-odd fields.  Returns 1 for a forward term. */
static int link_matrix(const geom* g, int64_t l, int mu, int pout, cplx M[3][3], cplx W[3][3],
                       const cplx* U, const cplx* X, const cplx* Y, double kappa,
                       const double theta[4])
{
    int c[4];
    coords(g, l, c);
    const int p = (c[0] + c[1] + c[2] + c[3]) & 1;
    const int forward = p == pout;
    int wrapped;
    const int64_t nb = neighbour(g, c, mu, +1, &wrapped); /* both cases: the site l + mu */
    cplx eta = 1.0;
    if (wrapped) eta = cexp(I * ((forward ? 1 : -1) * M_PI * theta[mu]));
    const cplx* xs = X + 12 * (int64_t)g->eo_of_lex[forward ? l : nb];
    const cplx* ys = Y + 12 * (int64_t)g->eo_of_lex[forward ? nb : l];
    const double sg = forward ? -1.0 : 1.0; /* 1 - gamma or 1 + gamma */
    cplx phi[4][3];
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx sum = 0;
            for (int r = 0; r < 4; ++r) sum += ((s == r ? 1.0 : 0.0) + sg * GAM[mu][s][r]) * ys[3 * r + a];
            phi[s][a] = sum;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            cplx sum = 0;
            for (int s = 0; s < 4; ++s) sum += phi[s][a] * conj(xs[3 * s + b]);
            W[a][b] = kappa * eta * sum;
        }
    const cplx* u = U + 9 * (mu * g->V + l);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            cplx sum = 0;
            for (int k = 0; k < 3; ++k)
                sum += forward ? u[3 * a + k] * W[k][b] : -W[a][k] * conj(u[3 * b + k]);
            M[a][b] = sum;
        }
    return forward;
}

/* Adds to out[mu][l]: kind 0: coeff * TA(M) (the su(3) force); kind 1:
 * coeff * (W^+ or W) (the Euclidean gradient of a forward or backward term). */
static void add_projected(const geom* g, int64_t l, int mu, cplx M[3][3], cplx W[3][3], int forward,
                          cplx* out, double coeff, int kind)
{
    cplx* f = out + 9 * (mu * g->V + l);
    if (kind == 0) {
        cplx A[3][3];
        cplx tr = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A[a][b] = 0.5 * (M[a][b] - conj(M[b][a]));
        for (int a = 0; a < 3; ++a) tr += A[a][a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) f[3 * a + b] += coeff * (A[a][b] - (a == b ? tr / 3.0 : 0.0));
    } else {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) f[3 * a + b] += coeff * (forward ? conj(W[b][a]) : W[a][b]);
    }
}

/* out[4][V][3][3] += coeff * P(dL/dU) for L = Re <X, H Y>; dir 0: H_eo
 * (X even, Y odd), dir 1: H_oe (X odd, Y even); kind as for add_projected. */
int orc_hop_force(const int dims[4], int dir, double* out, const double* gauge, const double* X,
                  const double* Y, double kappa, const double theta[4], double coeff, int kind)
{
    if ((dir != 0 && dir != 1) || (kind != 0 && kind != 1)) return -1;
    gam_init();
    geom g;
    int st = geom_init(&g, dims);
    if (st) return st;
    const int pout = dir == 0 ? 0 : 1;
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < g.V; ++l)
        for (int mu = 0; mu < 4; ++mu) {
            cplx M[3][3], W[3][3];
            const int fwd = link_matrix(&g, l, mu, pout, M, W, (const cplx*)gauge, (const cplx*)X,
                                        (const cplx*)Y, kappa, theta);
            add_projected(&g, l, mu, M, W, fwd, (cplx*)out, coeff, kind);
        }
    geom_free(&g);
    return 0;
}

/* out += coeff * P(dL/dU) for L = Re <chi, Qhat(sign) psi>.  With
 * Qhat = gamma_5 [A - H_oe A^-1 H_eo],
 *   dL = -Re <gamma_5 chi, dH_oe A^-1 H_eo psi> - Re <X2, dH_eo psi>,
 *   X2 = (A^-1)^+ H_oe^+ gamma_5 chi = (A^+)^-1 gamma_5 H_eo chi
 * (gamma_5-hermiticity H_oe^+ = gamma_5 H_eo gamma_5). */
int orc_qtm_force(const int dims[4], double* out, const double* gauge, const double* chi,
                  const double* psi, double kappa, double mu, const double theta[4], int sign,
                  double coeff, int kind)
{
    if (sign != 1 && sign != -1) return -1;
    geom g;
    int st = geom_init(&g, dims);
    if (st) return st;
    const int64_t Vh = g.Vh;
    geom_free(&g);
    cplx* te = malloc(sizeof(cplx) * 12 * Vh);
    cplx* x1 = malloc(sizeof(cplx) * 12 * Vh);
    if (!te || !x1) { free(te); free(x1); return -2; }
    const double mt = 2.0 * kappa * mu * sign;
    const double D = 1.0 + mt * mt;
    /* first term: X = gamma_5 chi (odd), Y = A^-1 H_eo psi (even), through H_oe */
    st = orc_hop(dims, 0, (double*)te, gauge, psi, kappa, theta);
    if (!st) {
        spin_lincomb_g5(te, te, Vh, 1.0 / D, -I * mt / D);
        spin_lincomb_g5(x1, (const cplx*)chi, Vh, 0.0, 1.0);
        st = orc_hop_force(dims, 1, out, gauge, (const double*)x1, (const double*)te, kappa, theta,
                           -coeff, kind);
    }
    /* second term: X = (A^+)^-1 gamma_5 H_eo chi (even), Y = psi (odd), through H_eo;
     * (A^+)^-1 = (1 + i mt gamma_5)/D */
    if (!st) st = orc_hop(dims, 0, (double*)te, gauge, chi, kappa, theta);
    if (!st) {
        spin_lincomb_g5(te, te, Vh, 0.0, 1.0);
        spin_lincomb_g5(te, te, Vh, 1.0 / D, I * mt / D);
        st = orc_hop_force(dims, 0, out, gauge, (const double*)te, psi, kappa, theta, -coeff, kind);
    }
    free(te);
    free(x1);
    return st;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the thread count of the parallel loops that follow (n >= 1). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
