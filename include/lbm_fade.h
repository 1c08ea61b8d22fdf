/*
 * lbm_fade.h -- C ABI of the MI355X (gfx950) library that runs the time step
 * of the lattice Boltzmann (LB) scheme for the space-fractional
 * advection-diffusion equation (FADE) of Cartalade, Younsi and Neel,
 * "Multiple-Relaxation-Time Lattice Boltzmann scheme for Fractional
 * Advection-Diffusion Equation" (arXiv:1706.09161).
 *
 * One step (Algorithm 1, time loop) is, on device:
 *   Phi_mu = p_mu I+^{2-alpha_mu}(g_mu C) + (1-p_mu) I-^{2-alpha_mu}(g_mu C) along every
 *            grid line of every axis (Sec. 2.4, trapezoidal product rule), run as
 *            a Toeplitz-plus-boundary-column GEMM on the matrix cores;
 *   f^eq(C, Phi, u) (Sec. 2.2, equations (Feq), (CoeffA_FADE3D));
 *   BGK or MRT collision with source (equations (LBE_FADE), (MRT-Coll));
 *   streaming (equation (Def_Translation)) and the Dirichlet rule
 *   (equation (Dirichlet_BC)); the new moment C = <1|f>.
 *
 * Conventions
 *   - Every call returns 0 (LBM_OK) or a negative LBM_E* code and never throws.
 *     lbm_fade_last_error() gives a message for the calling thread's last failure.
 *   - Grids count nodes per axis INCLUDING both wall nodes (the paper's N_mu + 1).
 *     Node fields are dense, x fastest: index x + nx*(y + ny*z).  Populations are
 *     structure-of-arrays: f[i*nodes + node], i = 0..Q-1 in the paper's order
 *     (e_0 = 0, e_{2mu-1} = +b_mu, e_{2mu} = -b_mu).
 *   - Pointers marked "host or device" are device pointers when on_device != 0
 *     (they must be on the handle's device and ordered on `stream`), else host
 *     pointers.  They are only borrowed for the duration of the call.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls are
 *     asynchronous on it unless stated otherwise; a call that reads into host
 *     memory synchronises the stream before returning.
 *   - The library owns all device state (populations, C, Phi, weights,
 *     checkpoints).  A handle is not thread-safe; distinct handles are.
 *   - On error the handle's state is unchanged unless stated otherwise.
 */
#ifndef LBM_FADE_H
#define LBM_FADE_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define LBM_API __attribute__((visibility("default")))
#else
#define LBM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_fade* lbm_fade_t;

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument or parameter */
    LBM_ENOMEM = -2,     /* device or host allocation failed */
    LBM_EDEVICE = -3,    /* HIP runtime error, or no usable gfx950 device */
    LBM_ENONFINITE = -4, /* non-finite value found by the optional guard */
    LBM_ESTATE = -5      /* call out of order (e.g. step before set_C) */
};

enum { LBM_D2Q5 = 5, LBM_D3Q7 = 7 };
enum { LBM_BGK = 0, LBM_MRT = 1 };

/* Arithmetic of the fractional-term GEMM.  Weights are always generated in FP64.
 *   LBM_FP32   FP32 operands on FP32 MFMA, FP32 accumulation;
 *   LBM_BF16X3 3-term split BF16: W = W_hi + W_lo, C = C_hi + C_lo (round to
 *              nearest even), W_hi C_hi + W_hi C_lo + W_lo C_hi on BF16 MFMA with
 *              FP32 accumulation (the lo*lo term is dropped);
 *   LBM_FP32_SIMT  FP32 fused multiply-add on the vector units (no MFMA); a
 *              plain kernel kept as a second implementation of the operator. */
enum { LBM_FP32 = 0, LBM_BF16X3 = 1, LBM_FP32_SIMT = 2 };

typedef struct {
    int32_t dim;   /* 2 or 3 */
    int32_t n[3];  /* nodes per axis incl. both walls (>= 3); n[2] ignored in 2D */
    double dx, dt; /* lattice spacing and time step (> 0) */
} lbm_grid;

typedef struct {
    double alpha[3];    /* fractional orders, in (1, 2]; gamma_mu = 2 - alpha_mu (Sec. 1) */
    double p[3];        /* skewness weights, in [0, 1] */
    double g[3];        /* positive factors g_mu (uniform per axis) */
    double D[9];        /* d x d diffusion tensor, row-major, symmetric positive definite */
    double u[3];        /* uniform velocity */
    double tau_free[4]; /* MRT relaxation TIMES of the moments beyond the fluxes (> 1/2):
                           D2Q5 rows 3,4 of M; D3Q7 rows 4,5,6 (Sec. 2.3).  Ignored for BGK. */
    double tau0;        /* relaxation time of the mass moment (> 0; no effect, Sec. 2.3) */
    double c_wall;      /* Dirichlet value on every wall node (Sec. 2.5) */
    int32_t collision;  /* LBM_BGK (needs isotropic D) or LBM_MRT */
    int32_t precision;  /* LBM_FP32, LBM_BF16X3 or LBM_FP32_SIMT */
    int32_t nonfinite_check_every; /* 0 = off; else check C every k steps inside lbm_fade_step */
    int32_t flux_form;  /* LBM_FLUX_RL: the dispersive flux of equation (Fg) (derivative of the
                           fractional integrals); LBM_FLUX_CAPUTO: the Caputo-type flux of equation
                           (Fg2), Sec. 3.5 (fractional integrals of the derivative), whose
                           equilibrium (CoeffA_FADE3DPS) subtracts, per axis, p g C(x_0)
                           (x - x_0)^(2-alpha) / Gamma(3-alpha) and (1-p) g C(x_N)
                           (x_N - x)^(2-alpha) / Gamma(3-alpha) from the fractional term, with
                           x_0, x_N the wall nodes ending the line (uniform C is then an
                           equilibrium) */
} lbm_params;

enum { LBM_FLUX_RL = 0, LBM_FLUX_CAPUTO = 1 };

/* Create a solver on the current HIP device.  Computes in FP64 on the host:
 * the relaxation times lambda-bar = D dt/(e^2 dx^2) + Id/2 (equation (D_ab);
 * for BGK equation (Diffusion_Coefficient_3D)) and the collision matrix
 * M^-1 Lambda M (equations (MatrixD2), (MatrixS)); the product-rule weights
 * c+-_{ln}(gamma_mu) of equations (c+), (c-) scaled by dx^gamma/Gamma(2+gamma),
 * as one Toeplitz generator per axis plus two boundary columns.
 * Allocates the device state (two population buffers, C, Phi, weights).
 * The product-rule integrals over the empty intervals at the ends of a line
 * (c+_{00}, c-_{NN}) are 0^gamma (constants stay integrated exactly there).
 * Errors: LBM_EINVAL for alpha outside (1,2], p outside [0,1], g <= 0, D not SPD
 * (or not isotropic for BGK), tau_free <= 1/2, tau0 <= 0, n < 3, lattice != 2*dim+1,
 * unknown collision/precision/flux_form; LBM_EDEVICE if the current device is not gfx950.
 * On error *out is set to NULL. */
LBM_API int lbm_fade_create(const lbm_grid* grid, int32_t lattice, const lbm_params* params, lbm_fade_t* out);

/* Destroy a handle and free its device memory (NULL-safe; synchronises the device). */
LBM_API void lbm_fade_destroy(lbm_fade_t h);

/* Set the initial concentration (host or device, nodes floats).  Wall nodes are
 * overwritten with c_wall (or the values of lbm_fade_set_wall), Phi(C0) is computed, and f := f^eq(C0, Phi(C0))
 * (reading of Algorithm 1's initialisations: the paper does not fix f(x, 0)). */
LBM_API int lbm_fade_set_C(lbm_fade_t h, const float* C0, int32_t on_device, void* stream);

/* Set the source field S (host or device, nodes floats), added as w_i S dt
 * after collision (equation (LBE_FADE)) by every later step until the next
 * call (a time-dependent source is set before every step); NULL removes it. */
LBM_API int lbm_fade_set_source(lbm_fade_t h, const float* S, int32_t on_device, void* stream);

/* Space-dependent diffusion tensor D(x) (Sec. 2.3: lambda-bar and Lambda may
 * depend on x; the exact-solution test of Sec. 3.4 uses D_mumu(x) proportional
 * to x_mu^alpha_mu).  D is host or device, d*d node fields, field-major:
 * D[(a*d + b)*nodes + node], FP32, each node's tensor symmetric and positive
 * SEMI-definite (it may vanish, e.g. on the x_mu = 0 walls).  Computes on the
 * host in FP64, once per call, lambda-bar(x) = D(x) dt/(e^2 dx^2) + Id/2 and
 * stores the difference lambda-bar(x)^-1 - lambda-bar^-1 from the flux block
 * of the handle's constant tensor (d(d+1)/2 FP32 fields on the device), which
 * the collision adds to its flux block at every node; the constant D of
 * create stays the reference (any SPD choice).  NULL goes back to the constant
 * D.  MRT only (LBM_EINVAL for BGK, whose single relaxation time covers every
 * moment).  Errors: LBM_EINVAL naming the first node whose tensor is not
 * finite, symmetric (relative 1e-6) or positive semi-definite (principal
 * minors >= -1e-6 times the product of their diagonal entries); the handle is
 * then unchanged.  Synchronises `stream` (device input is staged through the
 * host).  Adds 4 d(d+1)/2 bytes per node to the collide kernel's traffic.  The
 * adjoint refuses a handle with a space-dependent D or wall values. */
LBM_API int lbm_fade_set_diffusion(lbm_fade_t h, const float* D, int32_t on_device, void* stream);

/* Non-homogeneous Dirichlet values (Sec. 2.5 with a value per wall node):
 * Cw is host or device, one node field; the Dirichlet rule of every later
 * step, and the wall overwrite of set_C, use Cw[node] at wall nodes (interior
 * entries are ignored) instead of c_wall.  Time-dependent walls (Sec. 3.4) are
 * set before every step; the value written by a step is read when that step
 * runs.  NULL goes back to c_wall.  Host input synchronises `stream`. */
LBM_API int lbm_fade_set_wall(lbm_fade_t h, const float* Cw, int32_t on_device, void* stream);

/* Advance n >= 0 time steps.  Asynchronous; the launches of one step are: the
 * fractional-term GEMM of every axis, then the fused collide-stream-boundary-
 * moment kernel.  Returns LBM_ESTATE before set_C/set_f. */
LBM_API int lbm_fade_step(lbm_fade_t h, int64_t n, void* stream);

/* Copy C (nodes floats) to host or device memory. */
LBM_API int lbm_fade_get_C(lbm_fade_t h, float* dst, int32_t on_device, void* stream);

/* Copy / replace the populations (Q*nodes floats, structure of arrays) of the
 * current state (after streaming and the Dirichlet rule).  set_f recomputes C. */
LBM_API int lbm_fade_get_f(lbm_fade_t h, float* dst, int32_t on_device, void* stream);
LBM_API int lbm_fade_set_f(lbm_fade_t h, const float* src, int32_t on_device, void* stream);

/* Apply the fractional operator of Sec. 2.4 to a given field:
 * Phi[mu*nodes + node] = p_mu I+(g_mu C) + (1-p_mu) I-(g_mu C) for every axis,
 * with the handle's precision.  C and Phi are host or device (same on_device).
 * C = NULL applies it to the solver's current concentration (device Phi only;
 * LBM_ESTATE before set_C/set_f): exactly the GEMM launch of a step.
 * Does not touch the solver state. */
LBM_API int lbm_fade_apply_phi(lbm_fade_t h, const float* C, float* Phi, int32_t on_device, void* stream);

/* The operator of lbm_fade_apply_phi without a handle and without any device
 * allocation, for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, hosts that forbid hipMalloc).
 * grid and params are as for lbm_fade_create (same checks, same FP64 weight
 * generation, same kernels: the result equals lbm_fade_apply_phi on a handle
 * created with them, bit for bit).  C (nodes floats) and Phi (dim * nodes
 * floats, Phi[mu*nodes + node]) are device pointers on the current device,
 * ordered on `stream`; they are only borrowed.  The operator data (the
 * Toeplitz generator, boundary columns and BF16 splits of every axis) are
 * placed in a fixed device array of LBM_NOALLOC_SCRATCH_BYTES bytes that the
 * library holds on every device it runs on until the process ends: the call
 * needs about 40 n bytes per axis of n nodes and returns LBM_EINVAL, naming
 * the size, for a grid beyond that.  Every call on a device uses that
 * device's one array, so calls that overlap on one device (other host
 * threads, or other streams before this call's kernels have finished) race;
 * calls ordered on one stream are safe.  Synchronises `stream` once (after
 * copying the host-built operator data into the array); the fractional-term
 * kernels are then queued on `stream`. */
#define LBM_NOALLOC_SCRATCH_BYTES (16u << 20)
LBM_API int lbm_fade_apply_phi_noalloc(const lbm_grid* grid, const lbm_params* params, const float* C, float* Phi,
                                       void* stream);

/* Gradients reported by lbm_fade_adjoint (FP64). */
typedef struct {
    double dD[9]; /* d x d, symmetrised: dL = sum_ab dD_ab deltaD_ab for every symmetric
                     perturbation deltaD (so dL/dD_01 with D_01 = D_10 tied is 2 dD_01);
                     BGK: (dL/dD0 / d) Id for D = D0 Id */
    double du[3];
    double dp[3];
} lbm_grads;

/* Vector-Jacobian product of n steps (a hand-written adjoint; the paper has
 * none).  With C_n the concentration after n steps from the current state
 * (and the source given by set_source), returns the gradients of
 * L = <gC, C_n> with respect to D, u, p, the constant source (dS; nullable)
 * and, when the current state is the one set by set_C with no step since, the
 * initial concentration (dC0, wall entries zero; nullable; LBM_ESTATE
 * otherwise).  gC, dC0 and dS are host or device (same on_device), nodes
 * floats each.  The forward states are checkpointed every ckpt_every steps
 * and recomputed per segment; the GEMMs of the reverse sweep run in FP32
 * whatever the handle's precision.  Device memory held by the handle after
 * the first call: ceil(n / ckpt_every) checkpoints of the populations, and two
 * segment buffers of ckpt_every steps (populations, C and the fractional
 * terms) when both fit (one otherwise: the recompute then no longer overlaps
 * the reverse sweep on the handle's internal second stream), and the reverse
 * sweep's work fields (3Q + 4d + 4 floats per node).  The solver state
 * after the call is the state after n steps.  Synchronises `stream` (the
 * scalar gradients are written to host memory). */
LBM_API int lbm_fade_adjoint(lbm_fade_t h, int64_t n, int32_t ckpt_every, const float* gC, int32_t on_device,
                     lbm_grads* out, float* dC0, float* dS, void* stream);

/* ---------------------------------------------------------------------------
 * Levy-stable random walk (Sec. 3.1, equations (RW_STABLE), (distri); Sec. 3.2
 * compares the LB solutions with it).  Particles X in the open box ]lo, hi[
 * move by X_mu += u_mu dt + (D_mu g_mu)^(1/alpha_mu) (-cos(pi alpha_mu / 2) dt)^(1/alpha_mu)
 * S(alpha_mu, 2 p_mu - 1) per step and axis, S a stable variable with
 * characteristic function exp(-|k|^alpha (1 - j beta sign(k) tan(pi alpha / 2)))
 * (equations (stb), (stbb)) drawn with Weron's formula from two uniforms of
 * the counter-based generator Philox-4x32-10 at the counter
 * (particle, step, purpose) under `seed`; a particle not strictly inside the
 * box after a step is killed (first exit time, observed at the step times)
 * and stays dead.  The density of the surviving particles approximates the
 * FADE solution with homogeneous Dirichlet walls.  FP64 throughout; paths do
 * not depend on how the particles are split across calls (`first`).
 * Positions are device arrays of dim * n doubles, field-major (x[mu*n + k]);
 * alive flags one byte per particle (1 = alive).  All pointers are device
 * pointers ordered on `stream`; calls are asynchronous.  Errors: LBM_EINVAL
 * for dim outside 1..3, alpha outside (1, 2], p outside [0, 1], D < 0, g <= 0,
 * lo >= hi, dt <= 0, negative counts. */
typedef struct {
    int32_t dim;            /* 1, 2 or 3 */
    int32_t reserved;
    double lo[3], hi[3];    /* the box ]lo, hi[ */
    double alpha[3];        /* stability exponents, (1, 2] */
    double p[3];            /* skewness weights of the FADE; beta = 2 p - 1 */
    double D[3];            /* diagonal of the diffusion tensor (>= 0) */
    double g[3];            /* > 0 */
    double u[3];            /* velocity */
    double dt;              /* time step of the walk (the paper uses <= 1e-3) */
    uint64_t seed;          /* key of the generator */
} lbm_rw_params;

/* Initial positions of particles first .. first + n - 1: Gaussian hill of
 * standard deviation sigma0 around center (dim doubles, host) per axis, by
 * the Box-Muller transform (equation (Gaussian_IC_3D)); alive[k] = 1 if the
 * position lies in the box. */
LBM_API int lbm_rw_init_gaussian(const lbm_rw_params* P, const double* center, double sigma0, int64_t n, int64_t first,
                                 double* x, uint8_t* alive, void* stream);

/* Steps step0 + 1 .. step0 + nsteps (step0 + nsteps < 2^32) of particles
 * first .. first + n - 1, in place. */
LBM_API int lbm_rw_walk(const lbm_rw_params* P, double* x, uint8_t* alive, int64_t n, int64_t first, int64_t step0,
                        int64_t nsteps, void* stream);

/* Counts of the living particles per node of a grid with nodes[mu] nodes per
 * axis starting at lo with spacing dx (node j collects [lo + (j - 1/2) dx,
 * lo + (j + 1/2) dx); x fastest), into counts (device, prod(nodes) words,
 * cleared first; nodes is a host array of dim ints).  A density is
 * counts / (n dx^dim) times the initial mass. */
LBM_API int lbm_rw_histogram(const lbm_rw_params* P, const double* x, const uint8_t* alive, int64_t n,
                             const int32_t* nodes, double dx, uint32_t* counts, void* stream);

/* Message describing the calling thread's most recent failure ("" if none). */
LBM_API const char* lbm_fade_last_error(void);

/* Library version string. */
LBM_API const char* lbm_fade_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_FADE_H */
