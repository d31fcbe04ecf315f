/*
 * pibm.h -- C ABI of the MI355X (gfx950) library for the coupled thermal
 * lattice-Boltzmann / particulate-immersed-boundary / DEM time step of
 * Zhang, Yuan, Trias, Yu, Tan & Oliva, "Particulate immersed boundary method
 * for complex fluid-particle interaction problems with heat transfer"
 * (arXiv 1502.01159).
 *
 * One context = one simulation on one GPU.  The caller owns the device
 * workspace and the HIP stream; the library carves every buffer out of the
 * workspace and allocates no device memory of its own (its one fixed device
 * array belongs to pibm_mlp_grads_noalloc, below).  Host arrays passed in
 * are copied; the library keeps no host pointer after a call returns.
 * Contexts are not thread-safe: one host thread per context at a time.
 *
 * Units are lattice units throughout (h = dt = c = 1, reference fluid
 * density 1).  Lattice nodes are (i, j, k) with 0 <= i < nx, x fastest in
 * memory; non-periodic faces are no-slip walls half-way between the last node
 * and its missing neighbour (at -1/2 and n - 1/2).  Gravity acts along -y in
 * 2D and -z in 3D.
 *
 * Every call returns a pibm_status.  No C++ exception crosses this boundary.
 * After an error the context stays usable except after PIBM_EDEVICE.
 */
#ifndef PIBM_H
#define PIBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pibm_ctx pibm_ctx;

typedef enum {
    PIBM_OK = 0,
    PIBM_EINVAL = -1,    /* bad parameter, size, pointer or workspace too small */
    PIBM_ENOMEM = -2,    /* a device-side capacity (contacts, neighbours, tile lists) was exceeded */
    PIBM_EDEVICE = -3,   /* a HIP runtime call failed; the context must be destroyed */
    PIBM_EUNSTABLE = -4, /* the device watchdog saw a NaN, |u| > 0.4, a stale neighbour list
                            or a particle outside the domain */
    PIBM_EOVERLAP = -5,  /* initial particles overlap */
    PIBM_ESTATE = -6     /* call not valid in the current state (e.g. wrong checkpoint) */
} pibm_status;

/* Storage of the distributions.  Every variant stores deviations from the
 * rest state (f - w rho0, g - w T_s) and collides in a compute type:
 * F32 stores float and collides in double, rounding the stored deviations
 * stochastically (a counter hash of node, population and step decides the
 * rounding direction, so runs are reproducible); F64 stores and collides in
 * double; F16DEV / BF16DEV store 16-bit deviations scaled by 1/w, collide in
 * float and round stochastically the same way.  T_s = T_ref, except for the
 * 16-bit variants: there T_s is the middle of the temperatures the case sets
 * at pibm_init (T_init, the walls of non-periodic axes, the particles), so the
 * stored values keep the finest spacing.  Populations exchanged through
 * pibm_get_populations / pibm_set_populations are absolute either way. */
typedef enum {
    PIBM_STORE_F32 = 0,
    PIBM_STORE_F64 = 1,
    PIBM_STORE_F16DEV = 2,
    PIBM_STORE_BF16DEV = 3
} pibm_storage;

/* Lagrangian-point (marker) weights:
 *   SURFACE: the body surface element, pi D / N (2D) or pi D^2 / N (3D);
 *   PAPER:   the cross-section of a Lagrangian particle of diameter equal to
 *            the marker spacing s, pi s^2 / 4 in 3D and s per unit depth in
 *            2D (Sec. 2.2, after Eq. lbm12.6) -- the default;
 *   POINT:   one point at the body centre carrying the body cross-section
 *            (pi D^2 / 4 in 3D, D in 2D): the paper's sub-grid particle. */
typedef enum { PIBM_MARKERS_SURFACE = 0, PIBM_MARKERS_PAPER = 1, PIBM_MARKERS_POINT = 2 } pibm_markers;

/* Problem statement (Sec. 2): lattice, walls, Ra/Pr or nu/Gr, particles'
 * material.  Fields are read once by pibm_init. */
typedef struct pibm_params {
    int dim;                 /* 2 (D2Q9 + D2Q5) or 3 (D3Q19 or D3Q15, see lattice, + D3Q7) */
    int nx, ny, nz;          /* nodes per axis; nz = 1 in 2D */
    int periodic[3];         /* non-zero: periodic axis; zero: two walls */
    int storage;             /* pibm_storage */
    double T_wall[6];        /* Dirichlet wall temperature per face: -x,+x,-y,+y,-z,+z */
    double T_init;           /* initial fluid temperature (fluid at rest, rho = 1) */
    double T_ref;            /* Boussinesq reference temperature */
    /* Relaxation times.  If Ra > 0: Eqs. (lbm2.6), (lbm2.7) with
     * nu = sqrt(Pr) Lc uc / sqrt(Ra), alpha = Lc uc / sqrt(Pr Ra) and
     * g beta = uc^2 / (Lc dT_ref).  Otherwise nu is given, alpha = nu / Pr
     * and g beta = Gr nu^2 / Lc^3 (Gr on the length Lc).  Then
     * tau_f = 3 nu + 1/2 and tau_g = alpha / c_sg^2 + 1/2 (c_sg^2 = 1/3 for
     * D2Q5, 1/4 for D3Q7).  tau_f / tau_g > 0 override the derived values;
     * gbeta is used instead of the derived value when gbeta_set != 0. */
    double Ra, Pr, Lc, uc, dT_ref;
    double nu, Gr;
    double tau_f, tau_g;
    double gbeta;
    int gbeta_set;
    int marker_mode;         /* pibm_markers */
    double marker_spacing;   /* lattice units; <= 0 means 1 */
    double gravity;          /* particle gravity magnitude (lu / step^2) */
    double kappa_T;          /* thermal exchange prefactor of Q_l = 2 kappa_T (T_p - T_l) */
    double E_star;           /* Hertz effective modulus E* (same material for walls) */
    double poisson;          /* Poisson ratio (enters G*) */
    double mu_fric;          /* Coulomb friction coefficient */
    int n_sub;               /* DEM sub-steps per lattice step (>= 1) */
    double beta_p;           /* thermosensitive particles: rho_p(T) = rho_r (1 - beta_p (T - T_ref)) */
    double c_r;              /* particle / fluid volumetric heat-capacity ratio */
    double skin;             /* DEM neighbour-list skin (lu); <= 0 means 1 */
    int interp_order;        /* Lagrange nodes per axis of the interpolation, Eq. (lbm6): 2 (the
                                cell's corners, multilinear; 0 means 2) or 4 (nodes floor(X) - 1 ..
                                floor(X) + 2, cubic); other values are PIBM_EINVAL */
    int lattice;             /* 3D flow velocity set: 19 (D3Q19; 0 means 19) or 15 (the D3Q15 of
                                Sec. 2.1: rest, faces, corners, w = 2/9, 1/9, 1/72; FP32 and FP64
                                storage only); populations are ordered rest, +-x, +-y, +-z, then
                                the corners (+,+,+) (-,-,-) (+,+,-) (-,-,+) (+,-,+) (-,+,-)
                                (-,+,+) (+,-,-) */
    int thermal_model;       /* 0: D2Q5 / D3Q7 with the linear equilibrium (default); 1: temperature
                                on the flow lattice with the flow's quadratic equilibrium form and
                                c_sg^2 = 1/3 (Sec. 2.1 as printed; FP32 and FP64 storage only; the
                                wall of the last blocked axis sets a diagonal's Dirichlet value) */
    int streams;             /* 0: automatic (two streams on lattices of at least 2^22 nodes, one
                                below, where the cross-stream waits cost more than they hide);
                                1: every launch on the caller's stream; 2: the DEM and the next
                                step's cell and tile lists beside the lattice kernel on a second
                                stream.  Results are identical for every choice. */
} pibm_params;

enum { PIBM_FIXED = 1, PIBM_THERMO = 2 };

/* One particle: centre x, velocity u, angular velocity omega (2D: omega[2]),
 * accumulated rotation theta (diagnostic), radius R, density ratio rho_r =
 * rho_p / rho_f, temperature T, flags (PIBM_FIXED: not integrated;
 * PIBM_THERMO: temperature follows the lumped heat balance). */
typedef struct pibm_particle {
    double x[3], u[3], omega[3], theta[3];
    double R, rho_r, T;
    int flags;
    int reserved;
} pibm_particle;

/* Bytes of device workspace pibm_init needs for these parameters and
 * particles (radii decide the marker counts).  Returns 0 on invalid input. */
size_t pibm_workspace_bytes(const pibm_params *p, const pibm_particle *particles, int n_particles);

/* Create a context.  dev_workspace: device pointer (>= pibm_workspace_bytes,
 * 256-byte aligned) owned by the caller and borrowed until pibm_destroy;
 * hip_stream: the caller's hipStream_t (NULL = default stream) on which all
 * work is queued.  With two streams (pibm_params.streams) the context also
 * owns one non-blocking stream on that stream's device: within a step, the
 * DEM sub-steps and the next step's cell and tile lists run there beside the
 * lattice kernel (the first step's binning beside the exchange), forked from
 * and joined back into hip_stream by events, so every call's work is
 * complete once hip_stream is.  Validates tau > 1/2, sizes, particle overlap and containment; fills
 * f = w rho0, g = w T_init; uploads particles.  Returns after the uploads
 * completed; PIBM_EDEVICE if the stream or events cannot be created. */
int pibm_init(pibm_ctx **out, const pibm_params *p, const pibm_particle *particles, int n_particles,
              void *dev_workspace, size_t workspace_bytes, void *hip_stream);

/* Advance n_steps coupled time steps (Sec. 2): stream + PIBM exchange +
 * spreading + forced BGK collision for f and g, then the DEM sub-steps and
 * the thermosensitive update.  Asynchronous on the context's stream (no host
 * synchronisation); returns the first device error seen by an earlier
 * pibm_sync / pibm_particles / pibm_fields call, if any. */
int pibm_step(pibm_ctx *ctx, int n_steps);

/* Wait for the stream and return the device watchdog status. */
int pibm_sync(pibm_ctx *ctx);

/* Copy the particle state to out[cap] (cap >= n_particles); if fth is not
 * NULL, also the last step's reactions, 8 doubles per particle:
 * F[3] tau[3] H sum_l (T_p - T_l) A_l (Eq. lbm13; H = heat given to the
 * fluid).  Synchronises. */
int pibm_particles(pibm_ctx *ctx, pibm_particle *out, double *fth, int cap);

/* Replace the particle state (same count and radii as at init). */
int pibm_set_particles(pibm_ctx *ctx, const pibm_particle *p, int n);

/* Host copies of the macroscopic fields that the next collision would use:
 * rho[N], u[3 N] (node-major, 3 components), T[N]; any may be NULL.  The
 * state is not advanced.  Synchronises. */
int pibm_fields(pibm_ctx *ctx, double *rho, double *u, double *T);

/* Distributions of the current state as absolute values, q-major:
 * f[Q][N], g[Qg][N] (Q = 9/19, Qg = 5/7).  Synchronises. */
int pibm_get_populations(pibm_ctx *ctx, double *f, double *g);
int pibm_set_populations(pibm_ctx *ctx, const double *f, const double *g);

/* Number of lattice nodes, markers, and the step counter. */
long long pibm_num_nodes(const pibm_ctx *ctx);
long long pibm_num_markers(const pibm_ctx *ctx);
long long pibm_step_count(const pibm_ctx *ctx);

/* Derived parameters: out[0..4] = tau_f, tau_g, g beta, nu, alpha. */
int pibm_derived(const pibm_ctx *ctx, double *out);

/* Checkpoint: a versioned blob of parameters, step counter, distributions,
 * particles and contact history.  pibm_save with host_buf == NULL reports
 * the size in *used.  pibm_load requires identical parameters. */
int pibm_save(pibm_ctx *ctx, void *host_buf, size_t cap, size_t *used);
int pibm_load(pibm_ctx *ctx, const void *host_buf, size_t n);

/* Phase profiling.  While enabled, pibm_step records a pair of HIP events
 * around each timed phase of every step, on the stream that runs the phase:
 *   PIBM_PHASE_MARKERS  Lagrangian points: interpolation, exchange, reactions;
 *   PIBM_PHASE_BIN      particle -> lattice-tile binning;
 *   PIBM_PHASE_LATTICE  the fused stream / spreading / collision kernel;
 *   PIBM_PHASE_DEM      neighbour lists and the DEM sub-steps.
 * pibm_profile_read synchronises, returns per phase the summed elapsed
 * milliseconds ms[PIBM_NPHASE] and the number of timed phase executions
 * count[PIBM_NPHASE] since the previous read, and resets them.  Each event
 * pair costs the stream a few microseconds, so pibm_profile_phases times only
 * the phases whose bit (1 << PIBM_PHASE_*) is set in phase_mask (0: none;
 * bits beyond the phases: PIBM_EINVAL); pibm_profile(ctx, enable) times all
 * phases or none. */
enum { PIBM_PHASE_MARKERS = 0, PIBM_PHASE_BIN = 1, PIBM_PHASE_LATTICE = 2, PIBM_PHASE_DEM = 3, PIBM_NPHASE = 4 };
int pibm_profile(pibm_ctx *ctx, int enable);
int pibm_profile_phases(pibm_ctx *ctx, unsigned phase_mask);
int pibm_profile_read(pibm_ctx *ctx, double *ms, long long *count);

/* Release the context (not the caller's workspace or stream). */
int pibm_destroy(pibm_ctx *ctx);

/* ------------------------------------------------------------------------
 * Learned per-particle closure (not in the paper; it replaces the resolved
 * PIBM exchange of Sec. 2.2 in the coarse, one-point-per-particle mode):
 * a multilayer perceptron 16 -> 128 -> 128 -> 128 -> 4 with GELU (erf form)
 * hidden units.  Inputs are 16 normalised features per particle, outputs 4
 * normalised targets (drag, two lift components, Nusselt number); the
 * normalisation is the caller's.  Arithmetic: BF16 operands on the matrix
 * cores with FP32 accumulation, FP32 master weights and Adam state.
 *
 * Parameters, canonical order (FP32): W1[16][128], b1[128], W2[128][128],
 * b2[128], W3[128][128], b3[128], W4[128][4], b4[4]; layer l computes
 * z = h W_l + b_l.  The loss of a batch of n samples is
 * L = sum_s sum_c (y_sc - t_sc)^2 / (4 n).
 * ------------------------------------------------------------------------ */
enum { PIBM_MLP_IN = 16, PIBM_MLP_HIDDEN = 128, PIBM_MLP_OUT = 4, PIBM_MLP_NPARAM = 35716 };
typedef struct pibm_mlp pibm_mlp;

/* Device workspace for a network trained on batches of up to max_batch
 * samples (master weights, Adam moments, BF16 copies, per-workgroup gradient
 * slots).  Returns 0 if max_batch < 1. */
size_t pibm_mlp_workspace_bytes(int max_batch);

/* Create a network with weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)) drawn by
 * splitmix64 from `seed` and zero biases.  dev_workspace: 256-byte aligned,
 * >= pibm_mlp_workspace_bytes(max_batch), owned by the caller; hip_stream: the
 * caller's stream (NULL = default). */
int pibm_mlp_create(pibm_mlp **out, unsigned long long seed, int max_batch, void *dev_workspace,
                    size_t workspace_bytes, void *hip_stream);

/* Host copies of the FP32 parameters (PIBM_MLP_NPARAM floats, canonical
 * order).  set_params rejects non-finite values and restarts Adam. */
int pibm_mlp_set_params(pibm_mlp *m, const float *host_params);
int pibm_mlp_get_params(pibm_mlp *m, float *host_params);

/* Inference: dev_y[n][4] (FP32, 16-byte aligned) from dev_x[n][16] (BF16 bit
 * patterns, 8-byte aligned), both device pointers.  Asynchronous. */
int pibm_mlp_forward(pibm_mlp *m, const void *dev_x, float *dev_y, int n);

/* Gradient dL/dparam of one batch (1 <= n <= max_batch), copied to
 * host_grads[PIBM_MLP_NPARAM]; the loss to *loss if not NULL.  dev_t[n][4]
 * FP32 targets.  Parameters are not changed.  Synchronises. */
int pibm_mlp_grads(pibm_mlp *m, const void *dev_x, const float *dev_t, int n, float *host_grads, double *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with
 * learning rate lr on one batch; the batch loss before the step to *loss if
 * not NULL (then synchronises). */
int pibm_mlp_train_step(pibm_mlp *m, const void *dev_x, const float *dev_t, int n, float lr, double *loss);

/* Allocation-free variant of pibm_mlp_grads, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid hipMalloc).  Same kernels and the
 * same result bit for bit; the per-workgroup partial gradients, their sum and
 * the loss partials live in a fixed device array inside the library instead
 * of the network's workspace, so n may exceed the network's max_batch, up to
 * PIBM_MLP_NOALLOC_MAX_BATCH samples (larger n: PIBM_EINVAL).  The array is
 * about 9.3 MB per GPU, held from the first call on that GPU until the
 * process ends; every call on one GPU shares it and keeps the last call's
 * contents, so calls that overlap in time on one GPU (several host threads
 * or streams) race and must be serialised by the caller.  Calls no
 * allocating routine; synchronises the network's stream. */
enum { PIBM_MLP_NOALLOC_MAX_BATCH = 4096 };
int pibm_mlp_grads_noalloc(pibm_mlp *m, const void *dev_x, const float *dev_t, int n, float *host_grads,
                           double *loss);

int pibm_mlp_destroy(pibm_mlp *m);

/* Closure features and targets of the current state (not advanced), one row
 * per particle, host arrays x[n_particles][16] and t[n_particles][4] (either
 * may be NULL).  The fluid seen by a particle is the raw moments (rho, j, S)
 * summed over the nodes of the shell 0.75 D <= |x - X_p| <= 1.5 D around it,
 * U_f = sum j / sum rho, T_f = mean S (a region in units of D: the same on a
 * resolved and on a coarsened lattice); with the slip
 * s = U_f - U_p and its frame e1 = s/|s|, e2 = the up axis made normal to e1,
 * e3 = e1 x e2 (2D: e2 = e1 turned by +90 degrees):
 *   x = Re_p = |s| D/nu, Gr_p = g beta (T_p - T_f) D^3/nu^2, phi (solid
 *       volume of the particles with centres within 2 D over that ball),
 *       T_p - T_f, then the offsets of the 4 nearest centres in (e1, e2, e3)
 *       over D (2D: 6 nearest, 2 components), missing ones at 4;
 *   t = (F.e1, F.e2, F.e3) / (3 pi nu D |s|) (drag and lift over the
 *       Stokes drag of the slip; 2D: third entry 0) and the Nusselt number
 *       H / (pi D alpha (T_p - T_f)) (2D: H / (pi alpha (T_p - T_f))), 0 where
 *       |s| or T_p - T_f vanishes, from the Lagrangian-point exchange of
 *       Sec. 2.2 evaluated on this state (Eqs. lbm7-lbm8, lbm13); that
 *       exchange's reactions replace the last step's in pibm_particles.
 * Synchronises. */
int pibm_features(pibm_ctx *ctx, float *x, float *t);

/* Coarse one-point mode (PIBM_MARKERS_POINT only): replace the point
 * exchange by the network m (borrowed, on the same device).  Each step the
 * particle's features are normalised with norm[0..15] (mean) and
 * norm[16..31] (std > 0), the network's outputs denormalised with
 * norm[32..35] (mean) and norm[36..39] (std > 0) into the targets above,
 * and the force F = (t0 e1 + t1 e2 + t2 e3) 3 pi nu D |s| and heat
 * H = t3 pi D alpha (T_p - T_f) act on the particle (no fluid torque) while
 * -F and H are spread to the fluid from its centre with the kernel of
 * Eq. (lbm12).  m = NULL restores the point exchange. */
int pibm_set_closure(pibm_ctx *ctx, pibm_mlp *m, const float *norm);

/* Fallback of the learned closure to the method without it: lo[16], hi[16]
 * (host, raw feature units as pibm_features returns them; +-infinity allowed,
 * NaN refused) bound the inputs the network is trusted on.  Each step the
 * point exchange of Sec. 2.2 (Eqs. lbm7-lbm8, lbm13) is evaluated for every
 * particle, and the network's force and heat replace it only for particles
 * whose 16 features all lie within [lo, hi] (a non-finite feature is outside).
 * lo = hi = NULL removes the range (every particle takes the network);
 * pibm_set_closure clears it.  PIBM_EINVAL without a closure set, or with
 * only one of lo, hi.  Synchronises. */
int pibm_set_closure_range(pibm_ctx *ctx, const float *lo, const float *hi);

/* Static description of a status code. */
const char *pibm_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* PIBM_H */
