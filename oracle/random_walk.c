/*
 * random_walk.c -- ORACLE.  Test infrastructure only.
 *
 * Plain FP64 CPU version of the paper's Levy-stable random walk (Sec. 3.1,
 * "Equation (FADE_moreGeneral) and random walks", equations (RW_STABLE) and
 * (distri); bounded domains by killing at the first exit time), the
 * statistical check the paper compares its LB results with.  Like the rest of
 * the oracle it shares no code with the GPU library; both implement the same
 * counter-based generator from its published definition, so a particle's
 * path is a function of (seed, particle index, step) on either side.
 *
 * Random numbers: Philox-4x32-10 of Salmon, Moraes, Dror and Shaw ("Parallel
 * random numbers: as easy as 1, 2, 3", SC 2011): a 128-bit counter and a
 * 64-bit key, ten rounds; a round multiplies counter words 0 and 2 by
 * 0xD2511F53 and 0xCD9E8D57 (32 x 32 -> 64 bits) and mixes the high halves
 * with the other two words and the key; the key is bumped by the Weyl
 * constants 0x9E3779B9 and 0xBB67AE85 between rounds.  Counter of a draw:
 * (particle index low word, high word, step, purpose), key = the seed; two
 * output words make one FP64 uniform in the open interval (0, 1):
 * (k + 1/2) / 2^53 with k the top 53 bits of the pair.
 *
 * Stable variables: Weron's algebraic formula (after Chambers, Mallows and
 * Stuck) for S(alpha, beta) with characteristic function
 * exp(-|k|^alpha (1 - j beta sign(k) tan(pi alpha / 2))) (equations (stb),
 * (stbb)), alpha != 1, from V uniform on (-pi/2, pi/2) and W exponential of
 * mean 1:
 *   t = beta tan(pi alpha / 2), B = atan(t) / alpha, S = (1 + t^2)^(1/(2 alpha)),
 *   X = S sin(alpha (V + B)) / cos(V)^(1/alpha) (cos(V - alpha (V + B)) / W)^((1 - alpha)/alpha).
 *
 * Step of particle X along axis mu (equation (RW_STABLE) with (distri)):
 *   X_mu += u_mu dt + (D_mumu g_mu)^(1/alpha_mu) (-cos(pi alpha_mu / 2) dt)^(1/alpha_mu) S(alpha_mu, beta_mu),
 * beta = 2 p - 1; a particle is killed (and stays dead) once it is not
 * strictly inside the box after a step (killing at the first exit time,
 * observed at the step times).  Initial positions: the Gaussian hill
 * (Gaussian_IC_3D) by the Box-Muller transform.
 *
 * Positions are stored field-major: x[mu * n + k].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define RW_PI 3.14159265358979323846
#define RW_OK 0
#define RW_EINVAL (-1)

typedef struct {
    int32_t dim;
    int32_t reserved;
    double lo[3], hi[3]; /* the open box ]lo, hi[ */
    double alpha[3];     /* in (1, 2] */
    double p[3];         /* skewness weight; beta = 2 p - 1 */
    double D[3];         /* diagonal of the diffusion tensor */
    double g[3];
    double u[3];
    double dt;
    uint64_t seed;
} fo_rw_params;

/* Purposes (counter word 3): 0..2 the step draws of axis mu, 8..10 the
 * initial Gaussian of axis mu. */
#define PURPOSE_STEP 0u
#define PURPOSE_INIT 8u

void fo_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        const uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        if (r < 9) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* FP64 uniform in (0, 1) from two words: the top 27 bits of a and 26 of b. */
static double uniform53(uint32_t a, uint32_t b)
{
    const uint64_t k = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)k + 0.5) / 9007199254740992.0; /* 2^53 */
}

/* Two uniforms of the draw (seed, particle, step, purpose). */
static void draw2(uint64_t seed, int64_t particle, uint32_t step, uint32_t purpose, double* u1, double* u2)
{
    const uint32_t ctr[4] = {(uint32_t)(uint64_t)particle, (uint32_t)((uint64_t)particle >> 32), step, purpose};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    fo_philox4x32_10(ctr, key, o);
    *u1 = uniform53(o[0], o[1]);
    *u2 = uniform53(o[2], o[3]);
}

void fo_rw_uniforms(uint64_t seed, int64_t particle, uint32_t step, uint32_t purpose, double* u /* 2 */)
{
    draw2(seed, particle, step, purpose, &u[0], &u[1]);
}

/* S(alpha, beta) from V in (-pi/2, pi/2) and W > 0 (Weron's formula). */
double fo_stable_from(double alpha, double beta, double V, double W)
{
    const double t = beta * tan(RW_PI * alpha / 2.0);
    const double B = atan(t) / alpha;
    const double S = pow(1.0 + t * t, 1.0 / (2.0 * alpha));
    return S * sin(alpha * (V + B)) / pow(cos(V), 1.0 / alpha) *
           pow(cos(V - alpha * (V + B)) / W, (1.0 - alpha) / alpha);
}

/* S(alpha, beta) of the draw (seed, particle, step, purpose). */
double fo_stable_draw(double alpha, double beta, uint64_t seed, int64_t particle, uint32_t step, uint32_t purpose)
{
    double u1, u2;
    draw2(seed, particle, step, purpose, &u1, &u2);
    const double V = RW_PI * (u1 - 0.5);
    const double W = -log(u2);
    return fo_stable_from(alpha, beta, V, W);
}

static int check(const fo_rw_params* P)
{
    if (P->dim < 1 || P->dim > 3) return RW_EINVAL;
    if (!(P->dt > 0.0)) return RW_EINVAL;
    for (int mu = 0; mu < P->dim; ++mu) {
        if (!(P->alpha[mu] > 1.0 && P->alpha[mu] <= 2.0)) return RW_EINVAL;
        if (!(P->p[mu] >= 0.0 && P->p[mu] <= 1.0)) return RW_EINVAL;
        if (!(P->D[mu] >= 0.0) || !(P->g[mu] > 0.0)) return RW_EINVAL;
        if (!(P->lo[mu] < P->hi[mu])) return RW_EINVAL;
    }
    return RW_OK;
}

static int inside(const fo_rw_params* P, const double* x, int64_t n, int64_t k)
{
    for (int mu = 0; mu < P->dim; ++mu) {
        const double v = x[mu * n + k];
        if (!(v > P->lo[mu] && v < P->hi[mu])) return 0;
    }
    return 1;
}

/* Initial positions of particles first .. first + n - 1: the Gaussian hill of
 * standard deviation sigma0 around center (Box-Muller: sqrt(-2 log u2)
 * cos(2 pi u1)).  alive[k] = 1 if the position is inside the box. */
int fo_rw_init_gaussian(const fo_rw_params* P, const double* center, double sigma0, int64_t n, int64_t first,
                        double* x, uint8_t* alive)
{
    if (check(P) || n < 0 || !(sigma0 >= 0.0)) return RW_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        for (int mu = 0; mu < P->dim; ++mu) {
            double u1, u2;
            draw2(P->seed, first + k, 0u, PURPOSE_INIT + (uint32_t)mu, &u1, &u2);
            x[mu * n + k] = center[mu] + sigma0 * sqrt(-2.0 * log(u2)) * cos(2.0 * RW_PI * u1);
        }
        alive[k] = (uint8_t)inside(P, x, n, k);
    }
    return RW_OK;
}

/* Steps step0 + 1 .. step0 + nsteps of particles first .. first + n - 1 (x
 * and alive in place; dead particles do not move). */
int fo_rw_walk(const fo_rw_params* P, double* x, uint8_t* alive, int64_t n, int64_t first, int64_t step0,
               int64_t nsteps)
{
    if (check(P) || n < 0 || nsteps < 0 || step0 < 0 || step0 + nsteps > 0xFFFFFFFFll) return RW_EINVAL;
    double scale[3], beta[3];
    for (int mu = 0; mu < P->dim; ++mu) {
        const double a = P->alpha[mu];
        scale[mu] = pow(P->D[mu] * P->g[mu], 1.0 / a) * pow(-cos(RW_PI * a / 2.0) * P->dt, 1.0 / a);
        beta[mu] = 2.0 * P->p[mu] - 1.0;
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        if (!alive[k]) continue;
        for (int64_t s = step0 + 1; s <= step0 + nsteps; ++s) {
            for (int mu = 0; mu < P->dim; ++mu) {
                const double S = fo_stable_draw(P->alpha[mu], beta[mu], P->seed, first + k, (uint32_t)s,
                                                PURPOSE_STEP + (uint32_t)mu);
                x[mu * n + k] += P->u[mu] * P->dt + scale[mu] * S;
            }
            if (!inside(P, x, n, k)) {
                alive[k] = 0;
                break;
            }
        }
    }
    return RW_OK;
}

/* Counts of the living particles per node of a grid of n_mu nodes per axis
 * from lo with spacing dx (node j covers [lo + (j - 1/2) dx, lo + (j + 1/2) dx),
 * index x fastest); particles outside every cell are not counted. */
int fo_rw_histogram(const fo_rw_params* P, const double* x, const uint8_t* alive, int64_t n, const int32_t* nodes,
                    double dx, uint32_t* counts)
{
    if (check(P) || !(dx > 0.0)) return RW_EINVAL;
    int64_t total = 1;
    for (int mu = 0; mu < P->dim; ++mu) total *= nodes[mu];
    for (int64_t i = 0; i < total; ++i) counts[i] = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (!alive[k]) continue;
        int64_t idx = 0, mul = 1;
        int ok = 1;
        for (int mu = 0; mu < P->dim; ++mu) {
            const double j = floor((x[mu * n + k] - P->lo[mu]) / dx + 0.5);
            if (j < 0.0 || j >= (double)nodes[mu]) ok = 0;
            idx += (int64_t)j * mul;
            mul *= nodes[mu];
        }
        if (ok) counts[idx] += 1;
    }
    return RW_OK;
}
