/*
 * fade_oracle.c -- ORACLE.  Test infrastructure only.
 *
 * A plain, scalar, double-precision CPU implementation of the lattice
 * Boltzmann (LB) scheme for the space-fractional advection-diffusion
 * equation (FADE) of Cartalade, Younsi and Neel, "Multiple-Relaxation-Time
 * Lattice Boltzmann scheme for Fractional Advection-Diffusion Equation"
 * (arXiv:1706.09161).  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library; the GPU library neither
 * links nor calls it, and the two share no code, header or table.
 *
 * The method is an explicit iteration, so this file executes the steps of
 * the paper's Algorithm 1 in the paper's order and notation: the discrete
 * fractional integrals are direct sums with the trapezoidal product-rule
 * coefficients evaluated exactly as printed (Sec. 2.4), the collision is the
 * literal matrix product M^-1 Lambda M (f - f^eq) (Sec. 2.3) with M^-1 and
 * Lambda obtained by Gauss-Jordan inversion, and streaming and the Dirichlet
 * rule are applied node by node (Sec. 2.2, Sec. 2.5).  No blocking, fusion
 * or reordering is done beyond what those definitions state.
 *
 * Readings taken where the paper is silent or ambiguous (each one is also
 * repeated at its point of use):
 *   - grid size n[mu] counts nodes per axis INCLUDING both wall nodes, so the
 *     paper's N_mu = n[mu] - 1 and node indices run 0..N_mu (Sec. 2.4);
 *   - c+_{00} and c-_{NN} (integrals over an empty interval): 0^gamma, the value
 *     the exactness rule for constants gives at n = 0 (Sec. 2.4);
 *   - a wall node with several unknown populations (2D corners, 3D edges and
 *     corners) shares the Dirichlet deficit equally among them (Sec. 2.5);
 *   - initial populations are the equilibrium of the initial concentration,
 *     after the wall nodes have been overwritten with the wall value;
 *   - the D2Q5 relaxation matrix is blockdiag(tau0, lambda-bar (2x2),
 *     tau_free[0], tau_free[1]) for moment rows 3 and 4 of M (Sec. 2.3);
 *   - the "relaxation rates" lambda of the paper are relaxation TIMES: the
 *     collision uses 1/lambda (Sec. 2.2) and D = e^2 (lambda - 1/2) dx^2/dt;
 *   - the source enters after collision with weight w_i S dt (Sec. 2.2).
 *
 * Layout: node index x + nx*(y + ny*z) (x fastest); populations
 * f[i*nodes + node]; fractional terms Phi[mu*nodes + node].
 * Threads (OpenMP) only split independent nodes or lines: every value is
 * summed by one thread in a fixed order, so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FO_OK 0
#define FO_EINVAL (-1)
#define FO_ENOMEM (-2)

typedef struct {
    int32_t dim;        /* 2 (D2Q5) or 3 (D3Q7) */
    int32_t n[3];       /* nodes per axis, both wall nodes included */
    int32_t collision;  /* 0 = BGK, 1 = MRT */
    int32_t flux_form;  /* 0 = equation (Fg), 1 = the Caputo-type variant (Fg2) */
    double dx, dt;
    double alpha[3];    /* in (1, 2] */
    double p[3];        /* in [0, 1] */
    double g[3];        /* > 0 */
    double D[9];        /* d x d, row-major */
    double u[3];
    double tau_free[4]; /* relaxation times of the moments beyond the fluxes (MRT) */
    double tau0;        /* relaxation time of the mass moment (no effect) */
    double c_wall;      /* Dirichlet value on every wall node */
} fo_problem;

/* ------------------------------------------------------------------------ */
/* Lattices D2Q5 and D3Q7 (Sec. 2.1 and the caption of the lattice figure):
 * e_0 = 0, e_{2mu-1} = +b_mu, e_{2mu} = -b_mu; D2Q5: w0 = 1/3, w_i = 1/6,
 * e^2 = 1/3; D3Q7: w0 = 1/4, w_i = 1/8, e^2 = 1/4. */
typedef struct {
    int Q;
    int e[7][3];
    double w[7];
    double e2;
} fo_lattice_t;

static int lattice_of(int dim, fo_lattice_t* L)
{
    if (dim != 2 && dim != 3) return FO_EINVAL;
    memset(L, 0, sizeof(*L));
    L->Q = 2 * dim + 1;
    for (int mu = 0; mu < dim; ++mu) {
        L->e[2 * mu + 1][mu] = 1;
        L->e[2 * mu + 2][mu] = -1;
    }
    if (dim == 2) {
        L->w[0] = 1.0 / 3.0;
        for (int i = 1; i < 5; ++i) L->w[i] = 1.0 / 6.0;
        L->e2 = 1.0 / 3.0;
    } else {
        L->w[0] = 1.0 / 4.0;
        for (int i = 1; i < 7; ++i) L->w[i] = 1.0 / 8.0;
        L->e2 = 1.0 / 4.0;
    }
    return FO_OK;
}

int fo_lattice(int32_t dim, int32_t* Q, int32_t* e /* 7x3 */, double* w /* 7 */, double* e2)
{
    fo_lattice_t L;
    if (lattice_of(dim, &L) != FO_OK) return FO_EINVAL;
    *Q = L.Q;
    for (int i = 0; i < 7; ++i)
        for (int c = 0; c < 3; ++c) e[3 * i + c] = L.e[i][c];
    for (int i = 0; i < 7; ++i) w[i] = L.w[i];
    *e2 = L.e2;
    return FO_OK;
}

/* ------------------------------------------------------------------------ */
/* Trapezoidal product-rule coefficients for the left fractional integral,
 * equation (c+) of Sec. 2.4 (after Diethelm et al.).  Defined for 0 <= l <= n;
 * zero outside the summation range.  Reading at l = n = 0, where the printed
 * branches do not apply (the l = 0 branch needs (n - 1)^(gamma+1) at n = 0):
 * the integral over the empty interval [x_0, x_0] vanishes, and the weights
 * integrate constants exactly, sum_l c+_{ln} = (1 + gamma) n^gamma, which at
 * n = 0 gives c+_{00} = 0^gamma: 0 for gamma > 0, 1 for gamma = 0 (the
 * identity operator of alpha = 2). */
double fo_cplus(int64_t l, int64_t n, double gamma)
{
    if (l < 0 || l > n) return 0.0;
    if (n == 0) return pow(0.0, gamma);
    if (l == n) return 1.0;
    const double gp1 = gamma + 1.0;
    if (l == 0)
        return (1.0 + gamma) * pow((double)n, gamma) - pow((double)n, gp1) + pow((double)(n - 1), gp1);
    return pow((double)(n - l + 1), gp1) - 2.0 * pow((double)(n - l), gp1) + pow((double)(n - l - 1), gp1);
}

/* Coefficients for the right fractional integral, equation (c-) of Sec. 2.4.
 * Defined for n <= l <= N; zero outside.  Same reading at l = n = N:
 * c-_{NN} = 0^gamma. */
double fo_cminus(int64_t l, int64_t n, int64_t N, double gamma)
{
    if (l < n || l > N) return 0.0;
    if (n == N) return pow(0.0, gamma);
    if (l == n) return 1.0;
    const double gp1 = gamma + 1.0;
    if (l == N)
        return (1.0 + gamma) * pow((double)(N - n), gamma) - pow((double)(N - n), gp1) + pow((double)(N - n - 1), gp1);
    return pow((double)(l - n + 1), gp1) - 2.0 * pow((double)(l - n), gp1) + pow((double)(l - n - 1), gp1);
}

/* ------------------------------------------------------------------------ */
static int64_t nodes_of(const fo_problem* P)
{
    int64_t m = 1;
    for (int mu = 0; mu < P->dim; ++mu) m *= P->n[mu];
    return m;
}

static int64_t stride_of(const fo_problem* P, int mu)
{
    int64_t s = 1;
    for (int nu = 0; nu < mu; ++nu) s *= P->n[nu];
    return s;
}

static void coords_of(const fo_problem* P, int64_t node, int64_t x[3])
{
    x[0] = x[1] = x[2] = 0;
    for (int mu = 0; mu < P->dim; ++mu) {
        x[mu] = node % P->n[mu];
        node /= P->n[mu];
    }
}

static int validate(const fo_problem* P)
{
    if (P->dim != 2 && P->dim != 3) return FO_EINVAL;
    if (!(P->dx > 0.0) || !(P->dt > 0.0)) return FO_EINVAL;
    for (int mu = 0; mu < P->dim; ++mu) {
        if (P->n[mu] < 3) return FO_EINVAL;
        if (!(P->alpha[mu] > 1.0 && P->alpha[mu] <= 2.0)) return FO_EINVAL;
        if (!(P->p[mu] >= 0.0 && P->p[mu] <= 1.0)) return FO_EINVAL;
        if (!(P->g[mu] > 0.0)) return FO_EINVAL;
    }
    if (P->collision != 0 && P->collision != 1) return FO_EINVAL;
    if (P->flux_form != 0 && P->flux_form != 1) return FO_EINVAL;
    return FO_OK;
}

/* ------------------------------------------------------------------------ */
/* The fractional term of Algorithm 1 (time loop, first stage), for every node
 * and axis, by the discrete integrals of equation (XXminus_discret), Sec. 2.4:
 *   Phi_mu(x) = p_mu I+^{gamma_mu}(g_mu C)(x) + (1 - p_mu) I-^{gamma_mu}(g_mu C)(x),
 *   I+ = dx^gamma / Gamma(2+gamma) * sum_{l=0}^{n} c+_{ln} g C(y_l),
 *   I- = dx^gamma / Gamma(2+gamma) * sum_{l=n}^{N} c-_{ln} g C(y_l),
 * with gamma_mu = 2 - alpha_mu, y_l the node of the same line with index l
 * along mu, and the sums running over every node of the line, wall nodes
 * included.  The coefficients c+-_{ln} are tabulated once per axis from the
 * printed formulas; each sum is then taken term by term in increasing l. */
typedef struct {
    int64_t N;
    double* cp; /* (N+1)^2, cp[n*(N+1) + l] = c+_{ln} */
    double* cm; /* (N+1)^2, cm[n*(N+1) + l] = c-_{ln} */
} coeff_table;

/* A one-sided operator (p = 1 or p = 0) weighs one of the two integrals by
 * exactly zero: the forward term then builds no table for that integral and
 * forms no sum with it (for finite C, adding 0 * sum changes no value).  The
 * adjoint needs both tables for the p-derivative. */
static int make_table(int64_t N, double gamma, int need_plus, int need_minus, coeff_table* T)
{
    const int64_t m = N + 1;
    T->N = N;
    T->cp = need_plus ? (double*)malloc(sizeof(double) * m * m) : NULL;
    T->cm = need_minus ? (double*)malloc(sizeof(double) * m * m) : NULL;
    if ((need_plus && !T->cp) || (need_minus && !T->cm)) {
        free(T->cp);
        free(T->cm);
        return FO_ENOMEM;
    }
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < m; ++n)
        for (int64_t l = 0; l < m; ++l) {
            if (T->cp) T->cp[n * m + l] = fo_cplus(l, n, gamma);
            if (T->cm) T->cm[n * m + l] = fo_cminus(l, n, N, gamma);
        }
    return FO_OK;
}

static void free_table(coeff_table* T)
{
    free(T->cp);
    free(T->cm);
    T->cp = T->cm = NULL;
}

/* Phi_mu at index n of one line whose concentrations are line[0..N]. */
static double phi_on_line(const coeff_table* T, const double* line, int64_t n,
                          double p, double g, double pref)
{
    const int64_t m = T->N + 1;
    double splus = 0.0, sminus = 0.0;
    if (T->cp)
        for (int64_t l = 0; l <= n; ++l) splus += T->cp[n * m + l] * (g * line[l]);
    if (T->cm)
        for (int64_t l = n; l <= T->N; ++l) sminus += T->cm[n * m + l] * (g * line[l]);
    return p * (pref * splus) + (1.0 - p) * (pref * sminus);
}

/* The Caputo-type variant of the flux, equation (Fg2) of Sec. 3.5, puts the
 * derivative inside the fractional integrals.  Integration by parts
 * (equations (PSRLdD-a), (PSRLdD-b)) turns its equilibrium term, equation
 * (CoeffA_FADE3DPS), into the term of (Fg) minus the boundary values of the
 * line (the ends of the integration intervals on the box boundary):
 *   p g C(y_0) (x_n - x_0)^(2-alpha) / Gamma(3-alpha)
 *     + (1 - p) g C(y_N) (x_N - x_n)^(2-alpha) / Gamma(3-alpha),
 * with x_n - x_0 = n dx and x_N - x_n = (N - n) dx.  0^0 = 1 (alpha = 2). */
static double variant_boundary_term(double c0, double cN, int64_t n, int64_t N, double p, double g, double alpha,
                                    double dx)
{
    const double G = tgamma(3.0 - alpha);
    return p * g * c0 * pow((double)n * dx, 2.0 - alpha) / G +
           (1.0 - p) * g * cN * pow((double)(N - n) * dx, 2.0 - alpha) / G;
}

int fo_phi(const fo_problem* P, const double* C, double* Phi)
{
    int rc = validate(P);
    if (rc) return rc;
    const int64_t nodes = nodes_of(P);
    for (int mu = 0; mu < P->dim; ++mu) {
        const int64_t len = P->n[mu], N = len - 1, s = stride_of(P, mu);
        const int64_t lines = nodes / len;
        const double gamma = 2.0 - P->alpha[mu];
        const double pref = pow(P->dx, gamma) / tgamma(2.0 + gamma);
        coeff_table T;
        if (make_table(N, gamma, P->p[mu] != 0.0, P->p[mu] != 1.0, &T)) return FO_ENOMEM;
        double* out = Phi + (int64_t)mu * nodes;
        int failed = 0;
#pragma omp parallel
        {
            double* line = (double*)malloc(sizeof(double) * len);
            if (!line) {
#pragma omp atomic write
                failed = 1;
            } else {
#pragma omp for schedule(static)
                for (int64_t q = 0; q < lines; ++q) {
                    /* first node of line q: split q into the index below mu
                     * (stride < s) and the index above mu */
                    const int64_t base = (q % s) + (q / s) * s * len;
                    for (int64_t l = 0; l < len; ++l) line[l] = C[base + l * s];
                    for (int64_t n = 0; n < len; ++n) {
                        double v = phi_on_line(&T, line, n, P->p[mu], P->g[mu], pref);
                        if (P->flux_form == 1)
                            v -= variant_boundary_term(line[0], line[N], n, N, P->p[mu], P->g[mu], P->alpha[mu],
                                                       P->dx);
                        out[base + n * s] = v;
                    }
                }
                free(line);
            }
        }
        free_table(&T);
        if (failed) return FO_ENOMEM;
    }
    return FO_OK;
}

/* Same sums, evaluated only at the listed nodes: Phi[mu*count + k]. */
int fo_phi_at(const fo_problem* P, const double* C, const int64_t* which, int64_t count, double* Phi)
{
    int rc = validate(P);
    if (rc) return rc;
    const int64_t nodes = nodes_of(P);
    for (int64_t k = 0; k < count; ++k)
        if (which[k] < 0 || which[k] >= nodes) return FO_EINVAL;
    for (int mu = 0; mu < P->dim; ++mu) {
        const int64_t len = P->n[mu], N = len - 1, s = stride_of(P, mu);
        const double gamma = 2.0 - P->alpha[mu];
        const double pref = pow(P->dx, gamma) / tgamma(2.0 + gamma);
        const double p = P->p[mu], g = P->g[mu];
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t k = 0; k < count; ++k) {
            const int64_t node = which[k];
            const int64_t n = (node / s) % len;
            const int64_t base = node - n * s;
            double splus = 0.0, sminus = 0.0;
            for (int64_t l = 0; l <= n; ++l) splus += fo_cplus(l, n, gamma) * (g * C[base + l * s]);
            for (int64_t l = n; l <= N; ++l) sminus += fo_cminus(l, n, N, gamma) * (g * C[base + l * s]);
            double v = p * (pref * splus) + (1.0 - p) * (pref * sminus);
            if (P->flux_form == 1)
                v -= variant_boundary_term(C[base], C[base + N * s], n, N, p, g, P->alpha[mu], P->dx);
            Phi[(int64_t)mu * count + k] = v;
        }
    }
    return FO_OK;
}

/* ------------------------------------------------------------------------ */
/* Gauss-Jordan inversion with partial pivoting of an m x m row-major matrix. */
static int invert(int m, const double* A, double* Ainv)
{
    double W[7][14];
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < 2 * m; ++c) W[r][c] = (c < m) ? A[r * m + c] : (c - m == r ? 1.0 : 0.0);
    for (int c = 0; c < m; ++c) {
        int piv = c;
        for (int r = c + 1; r < m; ++r)
            if (fabs(W[r][c]) > fabs(W[piv][c])) piv = r;
        if (W[piv][c] == 0.0) return FO_EINVAL;
        if (piv != c)
            for (int k = 0; k < 2 * m; ++k) {
                double t = W[c][k];
                W[c][k] = W[piv][k];
                W[piv][k] = t;
            }
        const double d = W[c][c];
        for (int k = 0; k < 2 * m; ++k) W[c][k] /= d;
        for (int r = 0; r < m; ++r)
            if (r != c) {
                const double fct = W[r][c];
                if (fct != 0.0)
                    for (int k = 0; k < 2 * m; ++k) W[r][k] -= fct * W[c][k];
            }
    }
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) Ainv[r * m + c] = W[r][m + c];
    return FO_OK;
}

/* Collision operator data.  MRT (Sec. 2.3): M of equation (MatrixD2); Lambda
 * is the inverse of equation (MatrixS), whose flux block lambda-bar follows
 * from equation (D_ab): D = e^2 (lambda-bar - Id/2) dx^2/dt.  BGK (Sec. 2.2):
 * one relaxation time lambda from equation (Diffusion_Coefficient_3D), which
 * needs an isotropic D. */
typedef struct {
    int Q, dim, collision;
    double M[49], Minv[49], Lam[49], Laminv[49];
    double lambda_bgk;
} fo_collision;

static const double M_D2Q5[25] = {
    1, 1, 1, 1, 1,
    0, 1, -1, 0, 0,
    0, 0, 0, 1, -1,
    4, -1, -1, -1, -1,
    0, 1, 1, -1, -1,
};
static const double M_D3Q7[49] = {
    1, 1, 1, 1, 1, 1, 1,
    0, 1, -1, 0, 0, 0, 0,
    0, 0, 0, 1, -1, 0, 0,
    0, 0, 0, 0, 0, 1, -1,
    6, -1, -1, -1, -1, -1, -1,
    0, 2, 2, -1, -1, -1, -1,
    0, 0, 0, 1, 1, -1, -1,
};

static int make_collision(const fo_problem* P, fo_collision* K)
{
    fo_lattice_t L;
    int rc = validate(P);
    if (rc) return rc;
    lattice_of(P->dim, &L);
    const int d = P->dim, Q = L.Q;
    const double scale = P->dt / (L.e2 * P->dx * P->dx);
    memset(K, 0, sizeof(*K));
    K->Q = Q;
    K->dim = d;
    K->collision = P->collision;
    if (P->collision == 0) {
        /* BGK: D must be D*Id */
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                const double v = P->D[a * d + b];
                if (a != b && v != 0.0) return FO_EINVAL;
                if (a == b && v != P->D[0]) return FO_EINVAL;
            }
        K->lambda_bgk = P->D[0] * scale + 0.5;
        if (!(K->lambda_bgk > 0.5)) return FO_EINVAL;
        return FO_OK;
    }
    memcpy(K->M, d == 2 ? M_D2Q5 : M_D3Q7, sizeof(double) * Q * Q);
    rc = invert(Q, K->M, K->Minv);
    if (rc) return rc;
    /* Lambda^{-1} = blockdiag(tau0, lambda-bar, tau_free...) */
    K->Laminv[0] = P->tau0;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b)
            K->Laminv[(1 + a) * Q + (1 + b)] = P->D[a * d + b] * scale + (a == b ? 0.5 : 0.0);
    for (int k = d + 1; k < Q; ++k) K->Laminv[k * Q + k] = P->tau_free[k - d - 1];
    /* lambda-bar - Id/2 must be symmetric positive definite (D SPD): check
     * symmetry and leading principal minors of D. */
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < a; ++b)
            if (P->D[a * d + b] != P->D[b * d + a]) return FO_EINVAL;
    {
        const double* D = P->D;
        double m1 = D[0], m2, m3;
        if (!(m1 > 0.0)) return FO_EINVAL;
        m2 = D[0] * D[d + 1] - D[1] * D[d];
        if (!(m2 > 0.0)) return FO_EINVAL;
        if (d == 3) {
            m3 = D[0] * (D[4] * D[8] - D[5] * D[7]) - D[1] * (D[3] * D[8] - D[5] * D[6]) +
                 D[2] * (D[3] * D[7] - D[4] * D[6]);
            if (!(m3 > 0.0)) return FO_EINVAL;
        }
    }
    if (!(P->tau0 > 0.0)) return FO_EINVAL;
    for (int k = d + 1; k < Q; ++k)
        if (!(P->tau_free[k - d - 1] > 0.5)) return FO_EINVAL;
    return invert(Q, K->Laminv, K->Lam);
}

int fo_collision_matrices(const fo_problem* P, double* M, double* Minv, double* Lam, double* lambda_bgk)
{
    fo_collision K;
    int rc = make_collision(P, &K);
    if (rc) return rc;
    const int Q = 2 * P->dim + 1;
    if (P->collision == 1) {
        memcpy(M, K.M, sizeof(double) * Q * Q);
        memcpy(Minv, K.Minv, sizeof(double) * Q * Q);
        memcpy(Lam, K.Lam, sizeof(double) * Q * Q);
    }
    *lambda_bgk = K.lambda_bgk;
    return FO_OK;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium, equations (Feq) and (CoeffA_FADE3D), Sec. 2.2:
 *   f^eq_0 = C - w0 sum_mu Phi_mu,
 *   f^eq_i = w_i Phi_{mu(i)} + (C / e^2)(dt/dx) sum_mu u_mu e_{i,mu} w_i,
 * where mu(i) is the axis of e_i (i = 2mu-1, 2mu). */
static void equilibrium(const fo_problem* P, const fo_lattice_t* L, double C, const double* phi, double* feq)
{
    double sphi = 0.0;
    for (int mu = 0; mu < P->dim; ++mu) sphi += phi[mu];
    feq[0] = C - L->w[0] * sphi;
    for (int i = 1; i < L->Q; ++i) {
        const int mu = (i - 1) / 2;
        double adv = 0.0;
        for (int nu = 0; nu < P->dim; ++nu) adv += P->u[nu] * L->e[i][nu] * L->w[i];
        feq[i] = L->w[i] * phi[mu] + (C / L->e2) * (P->dt / P->dx) * adv;
    }
}

int fo_equilibrium(const fo_problem* P, double C, const double* phi, double* feq)
{
    fo_lattice_t L;
    int rc = validate(P);
    if (rc) return rc;
    lattice_of(P->dim, &L);
    equilibrium(P, &L, C, phi, feq);
    return FO_OK;
}

/* Collision with source at one node, equation (MRT-Coll) (or (LBE_FADE) for
 * BGK): f* = f - M^-1 Lambda M (f - f^eq) + w S dt.  Lam is the relaxation
 * matrix of this node (K->Lam unless the diffusion tensor varies in space). */
static void collide(const fo_problem* P, const fo_lattice_t* L, const fo_collision* K, const double* Lam,
                    const double* f, const double* feq, double S, double* fstar)
{
    const int Q = L->Q;
    if (K->collision == 0) {
        for (int i = 0; i < Q; ++i)
            fstar[i] = f[i] - (1.0 / K->lambda_bgk) * (f[i] - feq[i]) + L->w[i] * S * P->dt;
        return;
    }
    double dev[7], m[7], lm[7];
    for (int i = 0; i < Q; ++i) dev[i] = f[i] - feq[i];
    for (int r = 0; r < Q; ++r) {
        double s = 0.0;
        for (int c = 0; c < Q; ++c) s += K->M[r * Q + c] * dev[c];
        m[r] = s;
    }
    for (int r = 0; r < Q; ++r) {
        double s = 0.0;
        for (int c = 0; c < Q; ++c) s += Lam[r * Q + c] * m[c];
        lm[r] = s;
    }
    for (int r = 0; r < Q; ++r) {
        double s = 0.0;
        for (int c = 0; c < Q; ++c) s += K->Minv[r * Q + c] * lm[c];
        fstar[r] = f[r] - s + L->w[r] * S * P->dt;
    }
}

int fo_collide_node(const fo_problem* P, const double* f, double C, const double* phi, double S, double* fstar)
{
    fo_lattice_t L;
    fo_collision K;
    double feq[7];
    int rc = make_collision(P, &K);
    if (rc) return rc;
    lattice_of(P->dim, &L);
    equilibrium(P, &L, C, phi, feq);
    collide(P, &L, &K, K.Lam, f, feq, S, fstar);
    return FO_OK;
}

/* ------------------------------------------------------------------------ */
/* Moment C = <1|f> (Algorithm 1, last stage of the time loop). */
int fo_moment(const fo_problem* P, const double* f, double* C)
{
    int rc = validate(P);
    if (rc) return rc;
    const int64_t nodes = nodes_of(P);
    const int Q = 2 * P->dim + 1;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < nodes; ++x) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += f[(int64_t)i * nodes + x];
        C[x] = s;
    }
    return FO_OK;
}

static int on_wall(const fo_problem* P, const int64_t x[3])
{
    for (int mu = 0; mu < P->dim; ++mu)
        if (x[mu] == 0 || x[mu] == P->n[mu] - 1) return 1;
    return 0;
}

/* Streaming, equation (Def_Translation): f_i(x + e_i dx, t + dt) = f*_i(x, t),
 * taken as a pull f_i(y) = f*_i(y - e_i); a population whose source lies
 * outside the domain is unknown.  Then the Dirichlet rule, equation
 * (Dirichlet_BC) of Sec. 2.5: at a wall node with unknown set U,
 * f_b = (C_wall - sum_{i not in U} f_i) / |U| for b in U (|U| = 1 on faces;
 * the equal share at edges and corners is this implementation's reading).
 * c_wall is the Dirichlet value of node y. */
static void stream_node(const fo_problem* P, const fo_lattice_t* L, const double* fstar,
                        int64_t nodes, int64_t y, double c_wall, double* fy /* Q */)
{
    int64_t c[3];
    coords_of(P, y, c);
    int unknown[7] = {0}, nu_known = 0;
    double known = 0.0;
    for (int i = 0; i < L->Q; ++i) {
        int inside = 1;
        int64_t src = 0, mul = 1;
        for (int mu = 0; mu < P->dim; ++mu) {
            const int64_t s = c[mu] - L->e[i][mu];
            if (s < 0 || s >= P->n[mu]) inside = 0;
            src += s * mul;
            mul *= P->n[mu];
        }
        if (inside) {
            fy[i] = fstar[(int64_t)i * nodes + src];
            known += fy[i];
        } else {
            unknown[i] = 1;
            ++nu_known;
        }
    }
    if (nu_known > 0) {
        const double share = (c_wall - known) / (double)nu_known;
        for (int i = 0; i < L->Q; ++i)
            if (unknown[i]) fy[i] = share;
    }
}

/* Initial state (Algorithm 1, initialisations; reading: f(x, 0) is the
 * equilibrium of the initial concentration whose wall nodes carry the
 * Dirichlet value).  Cw (nullable) gives a Dirichlet value per node (only its
 * wall entries are read); NULL means P->c_wall on every wall node. */
int fo_init_var(const fo_problem* P, const double* C0, const double* Cw, double* f)
{
    fo_lattice_t L;
    int rc = validate(P);
    if (rc) return rc;
    lattice_of(P->dim, &L);
    const int64_t nodes = nodes_of(P);
    double* C = (double*)malloc(sizeof(double) * nodes);
    double* Phi = (double*)malloc(sizeof(double) * nodes * P->dim);
    if (!C || !Phi) {
        free(C);
        free(Phi);
        return FO_ENOMEM;
    }
    for (int64_t x = 0; x < nodes; ++x) {
        int64_t c[3];
        coords_of(P, x, c);
        C[x] = on_wall(P, c) ? (Cw ? Cw[x] : P->c_wall) : C0[x];
    }
    rc = fo_phi(P, C, Phi);
    if (!rc) {
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < nodes; ++x) {
            double phi[3], feq[7];
            for (int mu = 0; mu < P->dim; ++mu) phi[mu] = Phi[(int64_t)mu * nodes + x];
            equilibrium(P, &L, C[x], phi, feq);
            for (int i = 0; i < L.Q; ++i) f[(int64_t)i * nodes + x] = feq[i];
        }
    }
    free(C);
    free(Phi);
    return rc;
}

int fo_init(const fo_problem* P, const double* C0, double* f) { return fo_init_var(P, C0, NULL, f); }

/* Relaxation matrix of one node whose diffusion tensor is Dn (d x d,
 * row-major): the paper lets D, hence lambda-bar and Lambda, depend on x
 * (Sec. 2.3, and the exact-solution test of Sec. 3.4).  Lambda^{-1} is K's
 * blockdiag(tau0, lambda-bar, tau_free) with the flux block replaced by
 * lambda-bar(x) = Dn dt / (e^2 dx^2) + Id/2, inverted by Gauss-Jordan.
 * Dn must be symmetric positive SEMI-definite (every principal minor >= 0):
 * D(x) vanishes where x_mu = 0 in that test, and lambda-bar = Id/2 is still
 * invertible there. */
static int node_relaxation(const fo_problem* P, const fo_lattice_t* L, const fo_collision* K, const double* Dn,
                           double* Lam /* Q x Q */)
{
    const int d = P->dim, Q = L->Q;
    const double scale = P->dt / (L->e2 * P->dx * P->dx);
    double Li[49];
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < a; ++b)
            if (Dn[a * d + b] != Dn[b * d + a]) return FO_EINVAL;
    for (int a = 0; a < d; ++a) {
        if (!(Dn[a * d + a] >= 0.0)) return FO_EINVAL;
        for (int b = a + 1; b < d; ++b)
            if (!(Dn[a * d + a] * Dn[b * d + b] - Dn[a * d + b] * Dn[b * d + a] >= 0.0)) return FO_EINVAL;
    }
    if (d == 3) {
        const double m3 = Dn[0] * (Dn[4] * Dn[8] - Dn[5] * Dn[7]) - Dn[1] * (Dn[3] * Dn[8] - Dn[5] * Dn[6]) +
                          Dn[2] * (Dn[3] * Dn[7] - Dn[4] * Dn[6]);
        if (!(m3 >= 0.0)) return FO_EINVAL;
    }
    memcpy(Li, K->Laminv, sizeof(double) * Q * Q);
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) Li[(1 + a) * Q + (1 + b)] = Dn[a * d + b] * scale + (a == b ? 0.5 : 0.0);
    return invert(Q, Li, Lam);
}

/* Collision at every node: f -> f* (stages 1-2 of the time loop plus the
 * right-hand side of (MRT-Coll)).  C is the moment of f at the start of the
 * step.  LamN (nullable): relaxation matrix of every node, LamN[x*Q*Q + ...];
 * NULL means K->Lam everywhere. */
static int collide_all(const fo_problem* P, const fo_lattice_t* L, const fo_collision* K, const double* LamN,
                       const double* f, const double* S, double* fstar)
{
    const int64_t nodes = nodes_of(P);
    const int64_t QQ = (int64_t)L->Q * L->Q;
    double* C = (double*)malloc(sizeof(double) * nodes);
    double* Phi = (double*)malloc(sizeof(double) * nodes * P->dim);
    int rc = FO_ENOMEM;
    if (C && Phi) {
        fo_moment(P, f, C);
        rc = fo_phi(P, C, Phi);
        if (!rc) {
#pragma omp parallel for schedule(static)
            for (int64_t x = 0; x < nodes; ++x) {
                double fx[7], phi[3], feq[7], fs[7];
                for (int i = 0; i < L->Q; ++i) fx[i] = f[(int64_t)i * nodes + x];
                for (int mu = 0; mu < P->dim; ++mu) phi[mu] = Phi[(int64_t)mu * nodes + x];
                equilibrium(P, L, C[x], phi, feq);
                collide(P, L, K, LamN ? LamN + x * QQ : K->Lam, fx, feq, S ? S[x] : 0.0, fs);
                for (int i = 0; i < L->Q; ++i) fstar[(int64_t)i * nodes + x] = fs[i];
            }
        }
    }
    free(C);
    free(Phi);
    return rc;
}

/* nsteps iterations of the time loop of Algorithm 1 on f in place, with
 * optional space-dependent coefficients:
 *   S     (nullable) source field, constant over the nsteps;
 *   Dfld  (nullable) diffusion tensor of every node, Dfld[(a*d + b)*nodes + x]
 *         (MRT only: BGK has one relaxation time for every moment);
 *   Cw    (nullable) Dirichlet value of every node (wall entries are read).
 * NULL takes the constant P->D / P->c_wall.  A time-dependent source or wall
 * value is applied by calling this once per step with the fields of that
 * step. */
int fo_step_var(const fo_problem* P, double* f, const double* S, const double* Dfld, const double* Cw,
                int64_t nsteps)
{
    fo_lattice_t L;
    fo_collision K;
    int rc = make_collision(P, &K);
    if (rc) return rc;
    if (nsteps < 0) return FO_EINVAL;
    if (Dfld && P->collision != 1) return FO_EINVAL;
    lattice_of(P->dim, &L);
    const int64_t nodes = nodes_of(P);
    const int d = P->dim;
    const int64_t QQ = (int64_t)L.Q * L.Q;
    double* fstar = (double*)malloc(sizeof(double) * nodes * L.Q);
    double* LamN = Dfld ? (double*)malloc(sizeof(double) * nodes * QQ) : NULL;
    if (!fstar || (Dfld && !LamN)) {
        free(fstar);
        free(LamN);
        return FO_ENOMEM;
    }
    if (Dfld) {
        for (int64_t x = 0; x < nodes && !rc; ++x) {
            double Dn[9];
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) Dn[a * d + b] = Dfld[(int64_t)(a * d + b) * nodes + x];
            rc = node_relaxation(P, &L, &K, Dn, LamN + x * QQ);
        }
    }
    for (int64_t m = 0; m < nsteps && !rc; ++m) {
        rc = collide_all(P, &L, &K, LamN, f, S, fstar);
        if (rc) break;
#pragma omp parallel for schedule(static)
        for (int64_t y = 0; y < nodes; ++y) {
            double fy[7];
            stream_node(P, &L, fstar, nodes, y, Cw ? Cw[y] : P->c_wall, fy);
            for (int i = 0; i < L.Q; ++i) f[(int64_t)i * nodes + y] = fy[i];
        }
    }
    free(fstar);
    free(LamN);
    return rc;
}

int fo_step(const fo_problem* P, double* f, const double* S, int64_t nsteps)
{
    return fo_step_var(P, f, S, NULL, NULL, nsteps);
}

/* One iteration of the time loop evaluated only at the listed nodes: given
 * the full state f at time t, returns f(t + dt) at those nodes,
 * fnew[i*count + k].  Needs C(t) everywhere (cheap) but Phi only at the
 * listed nodes and their lattice neighbours. */
int fo_step_sampled(const fo_problem* P, const double* f, const double* S,
                    const int64_t* which, int64_t count, double* fnew)
{
    fo_lattice_t L;
    fo_collision K;
    int rc = make_collision(P, &K);
    if (rc) return rc;
    lattice_of(P->dim, &L);
    const int64_t nodes = nodes_of(P);
    const int Q = L.Q;
    for (int64_t k = 0; k < count; ++k)
        if (which[k] < 0 || which[k] >= nodes) return FO_EINVAL;
    double* C = (double*)malloc(sizeof(double) * nodes);
    int64_t* src = (int64_t*)malloc(sizeof(int64_t) * count * Q);
    double* phi = (double*)malloc(sizeof(double) * count * Q * P->dim);
    if (!C || !src || !phi) {
        free(C);
        free(src);
        free(phi);
        return FO_ENOMEM;
    }
    fo_moment(P, f, C);
    /* source node of every population of every listed node (or -1) */
    for (int64_t k = 0; k < count; ++k) {
        int64_t c[3];
        coords_of(P, which[k], c);
        for (int i = 0; i < Q; ++i) {
            int inside = 1;
            int64_t s_idx = 0, mul = 1;
            for (int mu = 0; mu < P->dim; ++mu) {
                const int64_t s = c[mu] - L.e[i][mu];
                if (s < 0 || s >= P->n[mu]) inside = 0;
                s_idx += s * mul;
                mul *= P->n[mu];
            }
            src[k * Q + i] = inside ? s_idx : -1;
        }
    }
    /* Phi at the source nodes (an outside source gets a dummy index 0) */
    {
        int64_t* at = (int64_t*)malloc(sizeof(int64_t) * count * Q);
        if (!at) rc = FO_ENOMEM;
        else {
            for (int64_t j = 0; j < count * Q; ++j) at[j] = src[j] >= 0 ? src[j] : 0;
            rc = fo_phi_at(P, C, at, count * Q, phi);
            free(at);
        }
    }
    if (!rc) {
        for (int64_t k = 0; k < count; ++k) {
            int unknown[7] = {0}, nu = 0;
            double known = 0.0, fy[7];
            for (int i = 0; i < Q; ++i) {
                const int64_t s = src[k * Q + i];
                if (s < 0) {
                    unknown[i] = 1;
                    ++nu;
                    continue;
                }
                double fs[7], ph[3], feq[7], fst[7];
                for (int j = 0; j < Q; ++j) fs[j] = f[(int64_t)j * nodes + s];
                for (int mu = 0; mu < P->dim; ++mu) ph[mu] = phi[(int64_t)mu * count * Q + k * Q + i];
                equilibrium(P, &L, C[s], ph, feq);
                collide(P, &L, &K, K.Lam, fs, feq, S ? S[s] : 0.0, fst);
                fy[i] = fst[i];
                known += fy[i];
            }
            if (nu > 0) {
                const double share = (P->c_wall - known) / (double)nu;
                for (int i = 0; i < Q; ++i)
                    if (unknown[i]) fy[i] = share;
            }
            for (int i = 0; i < Q; ++i) fnew[(int64_t)i * count + k] = fy[i];
        }
    }
    free(C);
    free(src);
    free(phi);
    return rc;
}

/* Number of threads the parallel loops above use. */
#ifdef _OPENMP
#include <omp.h>
#endif
int fo_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Subnormal operands read as zero and subnormal results written as zero (the
 * x86 MXCSR bits DAZ and FTZ), in the calling thread and every thread of the
 * OpenMP pool.  Off by default.  A long run whose field spreads through the
 * fractional tails fills many nodes with values below 2.2e-308, and x86
 * arithmetic on subnormals is slow enough to stall the dense sums; flushing
 * them changes the result by less than 1e-300 per value.  Returns 0, or -1
 * where the bits do not exist (then nothing changes). */
#if defined(__SSE2__)
#include <xmmintrin.h>
#endif
int fo_flush_subnormals(int on)
{
#if defined(__SSE2__)
    const unsigned bits = 0x8040u; /* FTZ (bit 15) | DAZ (bit 6) */
    int ok = 1;
#ifdef _OPENMP
#pragma omp parallel reduction(& : ok)
#endif
    {
        const unsigned m = _mm_getcsr();
        _mm_setcsr(on ? (m | bits) : (m & ~bits));
        ok = ok & (((_mm_getcsr() & bits) == bits) == (on != 0));
    }
    {
        const unsigned m = _mm_getcsr();
        _mm_setcsr(on ? (m | bits) : (m & ~bits));
    }
    return ok ? 0 : -1;
#else
    (void)on;
    return -1;
#endif
}

/* ======================================================================== */
/* Adjoint (vector-Jacobian product) of n time steps, FP64.  The paper has no
 * adjoint; this is the literal reverse of every sub-step above, in reverse
 * order, with every forward state stored (no checkpointing).  For
 * L = <gC, C_n>, C_n = <1|f^n>, f^0 = f^eq(C0', Phi(C0')) (C0' = C0 with the
 * wall nodes set to c_wall) it returns dL/dC0 (zero on wall nodes), dL/dS
 * (constant source), dL/dD (symmetrised: dL = sum_ab dD_ab deltaD_ab for a
 * symmetric perturbation; BGK: (dL/dD0 / d) Id), dL/du and dL/dp. */

/* Fractional-term data of one axis for the adjoint: coefficient tables and scalars. */
typedef struct {
    coeff_table T;
    double pref, p, g, alpha, dx;
    int flux_form;
    int64_t len, s;
} axis_data;

static int axis_prepare(const fo_problem* P, int mu, axis_data* A)
{
    A->len = P->n[mu];
    A->s = stride_of(P, mu);
    const double gamma = 2.0 - P->alpha[mu];
    A->pref = pow(P->dx, gamma) / tgamma(2.0 + gamma);
    A->p = P->p[mu];
    A->g = P->g[mu];
    A->alpha = P->alpha[mu];
    A->dx = P->dx;
    A->flux_form = P->flux_form;
    return make_table(A->len - 1, gamma, 1, 1, &A->T);
}

/* Adjoint of Phi_mu = K_mu C along every line of axis mu: Cbar += K^T Phibar,
 * and dL/dp_mu += <Phibar, pref g (W+ C - W- C)>; with the Caputo-type
 * variant also the transposed boundary terms (they reach the two wall nodes
 * of the line) and their p-derivative. */
static int phi_adjoint_axis(const fo_problem* P, const axis_data* A, int mu, const double* C, const double* Phibar,
                            double* Cbar, double* pbar)
{
    const int64_t nodes = nodes_of(P), len = A->len, N = len - 1, s = A->s, lines = nodes / len;
    const int64_t m = N + 1;
    double acc_p = 0.0;
    int failed = 0;
#pragma omp parallel reduction(+ : acc_p)
    {
        double* c = (double*)malloc(sizeof(double) * len);
        double* pb = (double*)malloc(sizeof(double) * len);
        double* cb = (double*)malloc(sizeof(double) * len);
        if (!c || !pb || !cb) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t q = 0; q < lines; ++q) {
                const int64_t base = (q % s) + (q / s) * s * len;
                for (int64_t l = 0; l < len; ++l) {
                    c[l] = C[base + l * s];
                    pb[l] = Phibar[(int64_t)mu * nodes + base + l * s];
                    cb[l] = 0.0;
                }
                double line_p = 0.0;
                for (int64_t n = 0; n < len; ++n) {
                    double splus = 0.0, sminus = 0.0;
                    for (int64_t l = 0; l <= n; ++l) {
                        cb[l] += pb[n] * A->pref * A->p * A->T.cp[n * m + l] * A->g;
                        splus += A->T.cp[n * m + l] * (A->g * c[l]);
                    }
                    for (int64_t l = n; l <= N; ++l) {
                        cb[l] += pb[n] * A->pref * (1.0 - A->p) * A->T.cm[n * m + l] * A->g;
                        sminus += A->T.cm[n * m + l] * (A->g * c[l]);
                    }
                    line_p += pb[n] * A->pref * (splus - sminus);
                    if (A->flux_form == 1) {
                        const double bp = variant_boundary_term(1.0, 0.0, n, N, 1.0, A->g, A->alpha, A->dx);
                        const double bm = variant_boundary_term(0.0, 1.0, n, N, 0.0, A->g, A->alpha, A->dx);
                        cb[0] -= pb[n] * A->p * bp;
                        cb[N] -= pb[n] * (1.0 - A->p) * bm;
                        line_p -= pb[n] * (bp * c[0] - bm * c[N]);
                    }
                }
                acc_p += line_p;
                for (int64_t l = 0; l < len; ++l) Cbar[base + l * s] += cb[l];
            }
        }
        free(c);
        free(pb);
        free(cb);
    }
    if (failed) return FO_ENOMEM;
    *pbar += acc_p;
    return FO_OK;
}

/* Adjoint of the equilibrium at one node: given febar, adds to *Cbar, phibar[mu]
 * and ubar[nu]. */
static void equilibrium_adjoint(const fo_problem* P, const fo_lattice_t* L, double C, const double* febar,
                                double* Cbar, double* phibar, double* ubar)
{
    *Cbar += febar[0];
    for (int mu = 0; mu < P->dim; ++mu) phibar[mu] += -L->w[0] * febar[0];
    for (int i = 1; i < L->Q; ++i) {
        const int mu = (i - 1) / 2;
        phibar[mu] += L->w[i] * febar[i];
        double adv = 0.0;
        for (int nu = 0; nu < P->dim; ++nu) {
            adv += P->u[nu] * L->e[i][nu] * L->w[i];
            ubar[nu] += febar[i] * (C / L->e2) * (P->dt / P->dx) * L->e[i][nu] * L->w[i];
        }
        *Cbar += febar[i] * (1.0 / L->e2) * (P->dt / P->dx) * adv;
    }
}

int fo_adjoint(const fo_problem* P, const double* C0, const double* S, int64_t nsteps, const double* gC,
               double* dC0, double* dS, double* dD, double* du, double* dp)
{
    fo_lattice_t L;
    fo_collision K;
    int rc = make_collision(P, &K);
    if (rc) return rc;
    if (nsteps < 0) return FO_EINVAL;
    lattice_of(P->dim, &L);
    const int Q = L.Q, d = P->dim;
    const int64_t nodes = nodes_of(P);
    double* fs = (double*)malloc(sizeof(double) * Q * nodes * (nsteps + 1)); /* f^0 .. f^n */
    double* C = (double*)malloc(sizeof(double) * nodes);
    double* Phi = (double*)malloc(sizeof(double) * nodes * d);
    double* fbar = (double*)malloc(sizeof(double) * Q * nodes);
    double* fsbar = (double*)malloc(sizeof(double) * Q * nodes);
    double* Cbar = (double*)malloc(sizeof(double) * nodes);
    double* Phibar = (double*)malloc(sizeof(double) * nodes * d);
    axis_data AX[3];
    int nax = 0;
    double Lambar[49] = {0}, lambar_bgk = 0.0, ubar[3] = {0, 0, 0}, pbar[3] = {0, 0, 0};
    if (!fs || !C || !Phi || !fbar || !fsbar || !Cbar || !Phibar) {
        rc = FO_ENOMEM;
        goto done;
    }
    for (nax = 0; nax < d; ++nax)
        if (axis_prepare(P, nax, &AX[nax])) {
            rc = FO_ENOMEM;
            goto done;
        }
    /* forward, storing every state */
    rc = fo_init(P, C0, fs);
    for (int64_t t = 0; t < nsteps && !rc; ++t) {
        memcpy(fs + (t + 1) * Q * nodes, fs + t * Q * nodes, sizeof(double) * Q * nodes);
        rc = fo_step(P, fs + (t + 1) * Q * nodes, S, 1);
    }
    if (rc) goto done;
    /* L = <gC, sum_i f^n_i> */
    for (int64_t x = 0; x < nodes; ++x)
        for (int i = 0; i < Q; ++i) fbar[(int64_t)i * nodes + x] = gC[x];
    for (int64_t x = 0; x < nodes; ++x) dS[x] = 0.0;

    for (int64_t t = nsteps - 1; t >= 0; --t) {
        const double* f = fs + t * Q * nodes;
        /* reverse of the Dirichlet rule and the streaming: fbar -> fsbar */
        memset(fsbar, 0, sizeof(double) * Q * nodes);
        for (int64_t y = 0; y < nodes; ++y) {
            int64_t c[3];
            coords_of(P, y, c);
            int unknown[7] = {0}, nu = 0;
            int64_t src[7];
            for (int i = 0; i < Q; ++i) {
                int inside = 1;
                int64_t s_idx = 0, mul = 1;
                for (int mu = 0; mu < d; ++mu) {
                    const int64_t sc = c[mu] - L.e[i][mu];
                    if (sc < 0 || sc >= P->n[mu]) inside = 0;
                    s_idx += sc * mul;
                    mul *= P->n[mu];
                }
                src[i] = s_idx;
                if (!inside) {
                    unknown[i] = 1;
                    ++nu;
                }
            }
            double avg = 0.0;
            if (nu > 0) {
                for (int i = 0; i < Q; ++i)
                    if (unknown[i]) avg += fbar[(int64_t)i * nodes + y];
                avg /= (double)nu;
            }
            for (int i = 0; i < Q; ++i)
                if (!unknown[i]) fsbar[(int64_t)i * nodes + src[i]] += fbar[(int64_t)i * nodes + y] - avg;
        }
        /* reverse of the collision and the equilibrium at every node */
        fo_moment(P, f, C);
        rc = fo_phi(P, C, Phi);
        if (rc) goto done;
        memset(Phibar, 0, sizeof(double) * nodes * d);
        double lam_acc[49] = {0}, lb_acc = 0.0, u_acc[3] = {0, 0, 0};
        for (int64_t x = 0; x < nodes; ++x) {
            double fx[7], phi[3], feq[7], fb[7], feqbar[7], phib[3] = {0, 0, 0}, cb = 0.0;
            for (int i = 0; i < Q; ++i) {
                fx[i] = f[(int64_t)i * nodes + x];
                fb[i] = fsbar[(int64_t)i * nodes + x];
            }
            for (int mu = 0; mu < d; ++mu) phi[mu] = Phi[(int64_t)mu * nodes + x];
            equilibrium(P, &L, C[x], phi, feq);
            double sb = 0.0;
            for (int i = 0; i < Q; ++i) sb += L.w[i] * P->dt * fb[i];
            dS[x] += sb;
            double fdir[7];
            if (K.collision == 0) {
                const double r = 1.0 / K.lambda_bgk;
                for (int i = 0; i < Q; ++i) {
                    fdir[i] = (1.0 - r) * fb[i];
                    feqbar[i] = r * fb[i];
                    lb_acc += fb[i] * (fx[i] - feq[i]) / (K.lambda_bgk * K.lambda_bgk);
                }
            } else {
                double dev[7], m[7], lmbar[7], mbar[7], devbar[7];
                for (int i = 0; i < Q; ++i) dev[i] = fx[i] - feq[i];
                for (int r = 0; r < Q; ++r) {
                    double s = 0.0;
                    for (int cc = 0; cc < Q; ++cc) s += K.M[r * Q + cc] * dev[cc];
                    m[r] = s;
                }
                for (int r = 0; r < Q; ++r) { /* lmbar = -Minv^T fb */
                    double s = 0.0;
                    for (int cc = 0; cc < Q; ++cc) s += K.Minv[cc * Q + r] * fb[cc];
                    lmbar[r] = -s;
                }
                for (int r = 0; r < Q; ++r)
                    for (int cc = 0; cc < Q; ++cc) lam_acc[r * Q + cc] += lmbar[r] * m[cc];
                for (int r = 0; r < Q; ++r) { /* mbar = Lam^T lmbar */
                    double s = 0.0;
                    for (int cc = 0; cc < Q; ++cc) s += K.Lam[cc * Q + r] * lmbar[cc];
                    mbar[r] = s;
                }
                for (int r = 0; r < Q; ++r) { /* devbar = M^T mbar */
                    double s = 0.0;
                    for (int cc = 0; cc < Q; ++cc) s += K.M[cc * Q + r] * mbar[cc];
                    devbar[r] = s;
                }
                for (int i = 0; i < Q; ++i) {
                    fdir[i] = fb[i] + devbar[i];
                    feqbar[i] = -devbar[i];
                }
            }
            equilibrium_adjoint(P, &L, C[x], feqbar, &cb, phib, u_acc);
            for (int mu = 0; mu < d; ++mu) Phibar[(int64_t)mu * nodes + x] = phib[mu];
            Cbar[x] = cb;
            for (int i = 0; i < Q; ++i) fbar[(int64_t)i * nodes + x] = fdir[i];
        }
        for (int k = 0; k < Q * Q; ++k) Lambar[k] += lam_acc[k];
        lambar_bgk += lb_acc;
        for (int mu = 0; mu < d; ++mu) ubar[mu] += u_acc[mu];
        /* reverse of the fractional term, then of the moment */
        for (int mu = 0; mu < d; ++mu) {
            rc = phi_adjoint_axis(P, &AX[mu], mu, C, Phibar, Cbar, &pbar[mu]);
            if (rc) goto done;
        }
        for (int64_t x = 0; x < nodes; ++x)
            for (int i = 0; i < Q; ++i) fbar[(int64_t)i * nodes + x] += Cbar[x];
    }
    /* reverse of the initial state f^0 = f^eq(C0', Phi(C0')) */
    for (int64_t x = 0; x < nodes; ++x) {
        int64_t c[3];
        coords_of(P, x, c);
        C[x] = on_wall(P, c) ? P->c_wall : C0[x];
    }
    rc = fo_phi(P, C, Phi);
    if (rc) goto done;
    for (int64_t x = 0; x < nodes; ++x) {
        double feqbar[7], phib[3] = {0, 0, 0}, cb = 0.0;
        for (int i = 0; i < Q; ++i) feqbar[i] = fbar[(int64_t)i * nodes + x];
        equilibrium_adjoint(P, &L, C[x], feqbar, &cb, phib, ubar);
        for (int mu = 0; mu < d; ++mu) Phibar[(int64_t)mu * nodes + x] = phib[mu];
        Cbar[x] = cb;
    }
    for (int mu = 0; mu < d; ++mu) {
        rc = phi_adjoint_axis(P, &AX[mu], mu, C, Phibar, Cbar, &pbar[mu]);
        if (rc) goto done;
    }
    for (int64_t x = 0; x < nodes; ++x) {
        int64_t c[3];
        coords_of(P, x, c);
        dC0[x] = on_wall(P, c) ? 0.0 : Cbar[x];
    }
    /* relaxation gradients -> D */
    {
        const double scale = P->dt / (L.e2 * P->dx * P->dx);
        double G[9] = {0};
        if (K.collision == 0) {
            for (int a = 0; a < d; ++a) G[a * d + a] = lambar_bgk * scale / d;
        } else {
            /* Lambda = (Lambda^-1)^-1: d(Lambda^-1) bar = -Lambda^T Lambar Lambda^T */
            double T1[49], T2[49];
            for (int r = 0; r < Q; ++r)
                for (int cc = 0; cc < Q; ++cc) {
                    double s = 0.0;
                    for (int k = 0; k < Q; ++k) s += K.Lam[k * Q + r] * Lambar[k * Q + cc];
                    T1[r * Q + cc] = s;
                }
            for (int r = 0; r < Q; ++r)
                for (int cc = 0; cc < Q; ++cc) {
                    double s = 0.0;
                    for (int k = 0; k < Q; ++k) s += T1[r * Q + k] * K.Lam[cc * Q + k];
                    T2[r * Q + cc] = -s;
                }
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) G[a * d + b] = T2[(1 + a) * Q + (1 + b)] * scale;
        }
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) dD[a * d + b] = 0.5 * (G[a * d + b] + G[b * d + a]);
    }
    for (int mu = 0; mu < d; ++mu) {
        du[mu] = ubar[mu];
        dp[mu] = pbar[mu];
    }
done:
    for (int k = 0; k < nax; ++k) free_table(&AX[k].T);
    free(fs);
    free(C);
    free(Phi);
    free(fbar);
    free(fsbar);
    free(Cbar);
    free(Phibar);
    return rc;
}
