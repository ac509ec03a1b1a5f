/*
 * lks.h - C ABI of the MI355X (gfx950) library for the moving-body lattice kinetic scheme (LKS),
 * its rigid-body design-to-analysis transfer and its exact discrete adjoint.
 *
 * Method: Tanabe, Yaji, Ushijima, "Topology optimization of actively moving rigid bodies in
 * unsteady flows" (arXiv 2506.23895).
 *   - problem statement: Eq. (1), min_gamma J(gamma, p, u), 0 <= gamma <= 1 (Sec. 2.1);
 *   - velocity sets D2Q9 / D3Q15 (Sec. 2.2, Fig. of the velocity sets) and D3Q19;
 *   - LKS update with tau = 1: pull of the equilibrium (Eqs. rho and u), equilibrium with the
 *     viscous A-term, nu = (1/6 - 2A/9) dx (Sec. 2.2);
 *   - Brinkman interpolation kappa_ref(gamma) (Sec. 2.3, first equation);
 *   - rigid motion of the design grid (Eqs. rigid_body_position, rigid_body_velocity);
 *   - transfer of kappa and the solid velocity with W = prod w (Eqs. brinkman_ref,
 *     velocity_ref and the weight functions); implicit VPM update (Eq. u_ex_2);
 *   - macroscopic boundary conditions (Eqs. bc_rho, bc_u);
 *   - Algorithm 1 (forward) and Algorithm 2 (reverse), design sensitivity pulled back to the
 *     design grid (Sec. 2.4); objectives J1, J2 over a window I (Sec. 2.5).
 * The reverse sweep is the exact derivative of the discrete forward map (the transposes of the
 * pull, equilibrium, force update, boundary conditions and transfer), which has the structure
 * of the paper's ALKS: a pull from x + c_i, w-weighted moments rho~, u~, s~ and the adjoint
 * equilibrium.
 *
 * Units: lattice units (dx = dt = 1).  The design grid has unit spacing; design node (i,j,k)
 * sits at xi = (i,j,k) in the design frame.  Analysis node (i,j,k) sits at x = (i,j,k).
 *
 * Conventions for every entry point:
 *   - return int: LKS_OK (0) or a negative LKS_E* code; no C++ exception crosses the ABI;
 *   - the caller owns every input and output buffer; the library copies what it keeps and never
 *     holds a caller pointer after a call returns;
 *   - a context owns all the device memory it allocates; contexts are independent; one context
 *     must not be used from two threads at once;
 *   - all GPU work of a context is enqueued on its stream; entry points that return results to
 *     the host synchronise that stream before returning;
 *   - lks_last_error(ctx) describes the last failure on that context.
 */
#ifndef LKS_H
#define LKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes --------------------------------------------------------------------- */
#define LKS_OK 0
#define LKS_EINVAL (-1)        /* malformed descriptor or argument                        */
#define LKS_ENOMEM (-2)        /* over the HBM budget, or a device allocation failed       */
#define LKS_ESTATE (-3)        /* call out of order (adjoint before forward, ...)         */
#define LKS_ENONFINITE (-4)    /* a NaN/Inf appeared in the state                         */
#define LKS_EDEVICE (-5)       /* a HIP runtime call failed                               */
#define LKS_EUNSUPPORTED (-6)  /* valid but not supported by this library                 */

/* ---- enumerations ----------------------------------------------------------------------- */
enum { LKS_D2Q9 = 0, LKS_D3Q15 = 1, LKS_D3Q19 = 2 };
/* Brinkman interpolation.  PAPER: gamma = 1 solid, kappa_ref = kmax q g / ((1 - g) + q).
 * FLUID_ONE: gamma = 1 fluid, kappa_ref = kmax q (1 - g) / (q + g) (the mirror form). */
enum { LKS_INTERP_PAPER = 0, LKS_INTERP_FLUID_ONE = 1 };
/* transfer kernel w: COS4 = (1 + cos(pi r/2))/4 on |r| <= 2 (Peskin); LIN = max(0, 1 - |r|) */
enum { LKS_W_COS4 = 0, LKS_W_LIN = 1 };
/* boundary kinds, applied face by face in the order x-, x+, y-, y+, z-, z+ (a later face wins
 * at shared edges).  With s the next node inward from a face node:
 *   VELOCITY / NOSLIP : u = u_bar, rho = rho(s)
 *   ZERO_GRADIENT     : rho = rho_bar, u = u(s)  (outflow: du/dn = 0 with the pressure level
 *                       held at rho_bar, the paper's Eq. bc_rho; rho_bar > 0 is required)
 *   PRESSURE          : rho = rho_bar, normal u = normal u(s), tangential u = u_bar
 *   PERIODIC          : both faces of the axis must be PERIODIC */
enum { LKS_BC_PERIODIC = 0, LKS_BC_VELOCITY = 1, LKS_BC_PRESSURE = 2, LKS_BC_ZERO_GRADIENT = 3,
       LKS_BC_NOSLIP = 4 };
/* objective densities summed over the mask and over steps n0..n1 (Sec. 2.5 for J1, J2; the
 * body-force kinds use F_b = kappa (u - u_S), the reaction of the VPM force on the fluid):
 *   POWER  : F_b . u_S          DRAG : F_b . dir          TORQUE : dir . ((x - centre) x F_b)
 *   J1     : -rho / 3           J2   : -dir . u           MASS   : rho          NONE : no J */
enum { LKS_OBJ_NONE = -1, LKS_OBJ_POWER = 0, LKS_OBJ_DRAG = 1, LKS_OBJ_TORQUE = 2,
       LKS_OBJ_J1 = 3, LKS_OBJ_J2 = 4, LKS_OBJ_MASS = 5 };
#define LKS_NORM_TIME 1 /* divide J by (n1 - n0 + 1)  */
#define LKS_NORM_MASK 2 /* divide J by the mask count */
enum { LKS_F32 = 0, LKS_F64 = 1 };
/* Reverse sweep.  EXACT: the exact derivative of the discrete objective (the transposes of every
 * forward step).  PAPER: the paper's own adjoint form (Sec. 2.4, Eqs. arho_ex, au_ex, as_ex and
 * the sensitivity on D): the Brinkman source divides only the pulled moment 3 u~ by (1 + kappa),
 * and the kappa seed is -(3 u~ / (1 + kappa)) . (u - u_S); an approximation of the gradient that
 * approaches it as dx -> 0 (2D only; three plain launches per step, for verification). */
enum { LKS_ADJ_EXACT = 0, LKS_ADJ_PAPER = 1 };
#define LKS_STATE_FINAL (-1)

/* ---- descriptor ------------------------------------------------------------------------- */
typedef struct {
    int kind;       /* LKS_BC_* */
    double rho;     /* rho_bar (PRESSURE, ZERO_GRADIENT) */
    double u[3];    /* u_bar (VELOCITY, NOSLIP; tangential part for PRESSURE) */
} lks_bc;

/* rigid motion at step n (record n is used at t_n = n):
 *   x_ref(xi) = R (xi - xi_G) + xG,   u_ref(xi) = omega x (R (xi - xi_G)) + uG
 * R row-major and orthogonal; in 2D R must be a rotation about z and omega = (0, 0, w). */
typedef struct {
    double R[9];
    double omega[3];
    double xG[3];
    double uG[3];
} lks_motion;

typedef struct {
    int kind;            /* LKS_OBJ_* */
    int n0, n1;          /* window, 1 <= n0 <= n1 <= nsteps */
    int normalize;       /* LKS_NORM_* bits */
    double centre[3];    /* TORQUE reference point */
    double dir[3];       /* DRAG / J2 direction, TORQUE axis */
    const uint8_t *mask; /* host [ncell] (x fastest) or NULL = every node; copied */
} lks_objective;

typedef struct {
    int dim;                     /* 2 or 3 */
    int lattice;                 /* LKS_D2Q9 (dim 2), LKS_D3Q15 / LKS_D3Q19 (dim 3) */
    int n[3];                    /* analysis grid; n[2] = 1 in 2D; >= 4 on non-periodic axes,
                                    >= 3 on periodic ones */
    int nd[3];                   /* design grid; nd[2] = 1 in 2D */
    double xi_G[3];              /* design-frame point mapped to xG */
    double nu;                   /* kinematic viscosity (> 0); A = 4.5 (1/6 - nu) */
    int interp;                  /* LKS_INTERP_* */
    double kappa_max, q;         /* Brinkman interpolation parameters */
    int weight;                  /* LKS_W_* */
    lks_bc bc[6];                /* faces x-, x+, y-, y+, z-, z+ (z ignored in 2D) */
    double rho0, u0[3];          /* uniform initial state ... */
    const double *rho_init;      /* ... or host [ncell] (optional, copied) */
    const double *u_init;        /* ... host [3*ncell] component-major (optional, copied) */
    const double *kappa_static;  /* host [ncell] static Brinkman field, zero velocity (optional) */
    double body_force[3];        /* uniform force added to u* (test use; usually 0) */
    int nsteps;                  /* N >= 1 */
    const lks_motion *motion;    /* host, nsteps + 1 records (copied) */
    lks_objective objective;
    int precision;               /* LKS_F32 or LKS_F64 */
    int checkpoint_every;        /* K: state checkpoints every K steps and recomputation of each
                                    segment in reverse; 0 keeps the whole trajectory */
    int io_on_device;            /* gamma, dJdgamma and read_state buffers are device pointers */
    void *stream;                /* hipStream_t, or NULL for the null stream */
    size_t hbm_budget_bytes;     /* 0 = no budget; else lks_create fails with LKS_ENOMEM above it */
    int adjoint_form;            /* LKS_ADJ_EXACT (0) or LKS_ADJ_PAPER; PAPER needs dim 2 and is
                                    not served by lks_begin (LKS_EUNSUPPORTED) */
    int zchunk;                  /* 3D: z planes each block of the z-marching kernels takes.  0
                                    chooses from the grid for a job alone on the GPU (enough blocks
                                    to fill it, at least 8 planes); a value in [8, 32] is taken as
                                    is (evened out over the chunks of n[2]), for jobs that share
                                    the GPU in batched rounds, where longer chunks re-evaluate
                                    fewer halo planes.  It changes only the grouping of the
                                    per-block objective partials (J to FP64 rounding); the state
                                    and dJ/dgamma are the same.  Outside [8, 32]: LKS_EINVAL. */
} lks_desc;

typedef struct lks_ctx lks_ctx;

/* Device bytes a context for *d would allocate (the HBM ledger).  Validates *d; no GPU call. */
int lks_query_bytes(const lks_desc *d, size_t *bytes);

/* Validate *d, copy what it points to and allocate every device buffer.  The rigid-body
 * footprint (mapped design grid plus the kernel support) must stay inside the domain at every
 * step, at least one node away from every non-periodic face, and must not wrap a periodic axis
 * (LKS_EINVAL otherwise).  *out is NULL on failure. */
int lks_create(const lks_desc *d, lks_ctx **out);

/* Free the context (NULL is a no-op).  Synchronises its stream. */
void lks_destroy(lks_ctx *c);

/* Algorithm 1: kappa_ref = I(gamma) on the design grid, then for n = 1..N the transfer of kappa
 * and u_S at t_n, the LKS pull, the VPM force update and the boundary conditions, with the
 * objective accumulated in FP64 over the window.  gamma: [nd] in the context precision (float or
 * double), host or device memory per io_on_device, read before return.  *J receives the
 * objective (host).  Replaces any previous trajectory.  The state is scanned for NaN/Inf after
 * every 64th step and after the last: LKS_ENONFINITE if a scan finds one, and lks_last_error then
 * names the first scanned step at which it was seen. */
int lks_forward(lks_ctx *c, const void *gamma, double *J);

/* Algorithm 2: the exact reverse sweep against the last forward, restoring each checkpointed
 * segment and recomputing it before its reverse steps, accumulating G(xi) = sum_n sum_x
 * W_n(x, xi) kappa_bar^n(x) in FP64.  LKS_ESTATE if no forward has run.  The adjoint state is
 * scanned for NaN/Inf after the reverse step of every n = 1 (mod 64), and G at the end:
 * LKS_ENONFINITE if either holds one (lks_last_error names the latest reverse step seen). */
int lks_adjoint(lks_ctx *c);

/* dJ/dgamma = I'(gamma) * G on the design grid, [nd] in the context precision, host or device
 * per io_on_device.  LKS_ESTATE if no adjoint has run since the last forward. */
int lks_sensitivity(lks_ctx *c, void *dJdgamma);

/* Copy a state of the last forward: which = LKS_STATE_FINAL for X^N, or k >= 0 for the state
 * at step k * checkpoint_every (k = 0 is the initial state).  drho = rho - 1 as [ncell] and
 * u as [dim][ncell] (component-major), context precision, host or device per io_on_device;
 * either pointer may be NULL.  LKS_ESTATE before a forward, LKS_EINVAL for an unknown k. */
int lks_read_state(lks_ctx *c, int which, void *drho, void *u);

/* Per-step objective values j^n (n = 0..nsteps, already scaled), host double[nsteps + 1]. */
int lks_read_objective_steps(lks_ctx *c, double *jn);

/* Kernel timing: sample every k-th launch of each kernel kind with HIP events on the context
 * stream (k = 0 switches sampling off).  lks_kernel_timing returns, for kind 0 = forward step,
 * 1 = adjoint step, 2 = sensitivity gather, the number of sampled launches and their mean
 * duration in milliseconds. */
int lks_set_timing(lks_ctx *c, int every);
int lks_kernel_timing(lks_ctx *c, int kind, long *count, double *mean_ms);

/* ---- continuous batching (the served path) ------------------------------------------------
 * Many contexts advance together: each round moves every listed context by one micro-step of
 * its evaluation (a forward step, a recomputed step, or an adjoint step with its sensitivity
 * gather), and the kernels of all of them share one launch per kernel kind.  Every context of a
 * round must use the batch's stream and one precision.  Results are bitwise identical to the
 * single-context path: each job keeps its own buffers, tiles and fixed-order reductions. */
typedef struct lks_batch lks_batch;

/* Staging buffers for per-job kernel arguments (a ring of pinned slots) on stream. */
int lks_batch_create(void *stream, lks_batch **out);
void lks_batch_destroy(lks_batch *b);  /* NULL is a no-op; synchronises the stream */

/* Start an evaluation of c (forward, reverse sweep, sensitivity) on device buffers: gamma is
 * read and dJdgamma [nd] written in the context precision; both must stay valid until
 * lks_finish returns.  Needs an io_on_device context with an objective.  Enqueues only. */
int lks_begin(lks_ctx *c, const void *gamma, void *dJdgamma);

/* One round over cs[0..n-1]; done[i] (optional) becomes 1 once the last kernel of context i's
 * evaluation is enqueued.  Enqueues only (blocks only when the staging ring is full). */
int lks_batch_round(lks_batch *b, lks_ctx *const *cs, int n, int *done);
const char *lks_batch_error(const lks_batch *b);

/* 1 if context c's evaluation has completed on the device, 0 if not yet (never blocks). */
int lks_poll(lks_ctx *c);

/* Wait for context c's evaluation and return J (host); dJdgamma is then complete.
 * LKS_ENONFINITE if a scan of the forward state, the adjoint state or G found a NaN/Inf (the same
 * scans as lks_forward and lks_adjoint). */
int lks_finish(lks_ctx *c, double *J);

/* ---- forward sweep without device allocation ------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the forward sweep of lks_forward for descriptor d, with
 * every buffer the kernels need beyond the caller's (state ping-pong, X^0, X^N, footprint ring,
 * design arrays, objective partials and per-step values, argument blocks) carved out of one static
 * device array of LKS_NOALLOC_SCRATCH_BYTES bytes, which each device the library runs on holds
 * until the process ends.  No hipMalloc, hipFree or other allocating routine is called.
 *   gamma   [nd] design field in the descriptor's precision (host or device memory);
 *   J       host, receives the objective (may be NULL);
 *   drho, u X^N as rho - 1 [ncell] and u [dim][ncell], component-major, descriptor precision,
 *           host or device memory (either may be NULL).
 * The results are those of lks_create + lks_forward + lks_read_state(FINAL) on the same inputs.
 * d->checkpoint_every and d->io_on_device are ignored; the work runs on d->stream, which is
 * synchronised before return.  LKS_EINVAL if the workload needs more scratch than the array holds
 * (lks_last_error(NULL) says how much); LKS_ENONFINITE as for lks_forward.  Every call on one
 * device shares that device's array and leaves its contents behind: calls that overlap on one
 * device (two host threads, or two streams) race, so serialise them. */
#define LKS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int lks_forward_noalloc(const lks_desc *d, const void *gamma, double *J, void *drho, void *u);

/* Static description of the last failure of c (or, when c is NULL, of the last failed
 * lks_create or lks_forward_noalloc of the calling thread), and of a return code. */
const char *lks_last_error(const lks_ctx *c);
const char *lks_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* LKS_H */
