/*
 * FP64 CPU oracle for the moving-body lattice kinetic scheme and its exact discrete adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library.  It shares no code, header, table or helper with the
 * HIP library; the two agree only because both follow the paper:
 *
 *   Tanabe, Yaji, Ushijima, "Topology optimization of actively moving rigid bodies in unsteady
 *   flows" (arXiv 2506.23895),
 *     Sec. 2.2  LKS pull of the equilibrium (Eqs. rho, u), the equilibrium with the viscous
 *               A-term, nu = 1/6 - 2A/9, force update (Eqs. rho_ex, u_ex), direct macroscopic
 *               boundary conditions (Eqs. bc_rho, bc_u);
 *     Sec. 2.3  Brinkman interpolation kappa_ref(gamma), rigid-body position and velocity
 *               (Eqs. rigid_body_position, rigid_body_velocity), transfer with the product
 *               weight W (Eqs. brinkman_ref, velocity_ref), implicit VPM update (Eq. u_ex_2),
 *               Algorithm 1;
 *     Sec. 2.4  adjoint structure (Eqs. arho, au, as and the adjoint equilibrium), design
 *               sensitivity pulled back to the design grid, Algorithm 2;
 *     Sec. 2.5  objectives J1, J2 over a window I.
 *
 * Lattice units throughout (dx = dt = 1, tau = 1).  The reverse sweep computes the exact
 * derivative of the discrete objective defined by the forward steps (not the paper's
 * continuous-then-discretised adjoint); the readings of silent or garbled passages are listed
 * in the design notes of the repository.
 *
 * Pins: every function here is checked in the CPU test suite against closed forms (shear-wave
 * decay, Poiseuille, Couette, the pressure-driven channel, objective densities on constructed
 * fields), invariants (mass conservation, uniform flow, rigid isometry, the steady velocity-inlet
 * channel), special cases (integer-shift transfer, quarter-turn permutation), transpose
 * identities and central finite differences of J.  The Taylor-Couette comparison of the paper's
 * Appendix is a physics check within the penalisation error.  or_step_T_paper (the paper's own
 * adjoint form) is the derivative of no discrete map, so FD cannot pin it: it is pinned where it
 * must equal the exact step, by the closed-form per-step gain of an adjoint shear wave under a
 * uniform kappa (which separates the divided 3 u~ from the strain part that passes), and against
 * central differences within a few per cent.
 *
 * Layout: node (i,j,k) has index i + n0*(j + n1*k).  Vector fields are component-major:
 * u[a*ncell + idx].  2D problems use n[2] = nd[2] = 1 and only the x,y components.
 */
#ifndef LKS_ORACLE_H
#define LKS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_D2Q9 = 0, OR_D3Q15 = 1, OR_D3Q19 = 2 };
enum { OR_INTERP_PAPER = 0, OR_INTERP_FLUID_ONE = 1 };
enum { OR_W_COS4 = 0, OR_W_LIN = 1 };
enum { OR_BC_PERIODIC = 0, OR_BC_VELOCITY = 1, OR_BC_PRESSURE = 2, OR_BC_ZERO_GRADIENT = 3,
       OR_BC_NOSLIP = 4 };
enum { OR_OBJ_NONE = -1, OR_OBJ_POWER = 0, OR_OBJ_DRAG = 1, OR_OBJ_TORQUE = 2, OR_OBJ_J1 = 3,
       OR_OBJ_J2 = 4, OR_OBJ_MASS = 5 };
enum { OR_ADJ_EXACT = 0, OR_ADJ_PAPER = 1 };
#define OR_NORM_TIME 1
#define OR_NORM_MASK 2

typedef struct {
    int dim;                 /* 2 or 3 */
    int lattice;             /* OR_D2Q9 / OR_D3Q15 / OR_D3Q19 */
    int n[3];                /* analysis grid */
    int nd[3];               /* design grid (unit spacing) */
    double xi_G[3];          /* design-frame point mapped to x_G */
    double nu;               /* kinematic viscosity, lattice units */
    int interp;              /* Brinkman interpolation form */
    double kappa_max, q;
    int weight;              /* transfer kernel w */
    int bc_kind[6];          /* faces x-, x+, y-, y+, z-, z+ */
    double bc_rho[6];        /* rho_bar of PRESSURE and ZERO_GRADIENT faces */
    double bc_u[6][3];
    double rho0, u0[3];      /* uniform initial state unless the fields below are given */
    const double *rho_init;  /* [ncell] or NULL */
    const double *u_init;    /* [3*ncell] or NULL */
    const double *kappa_static; /* [ncell] or NULL: static Brinkman field, zero solid velocity */
    double g[3];             /* uniform body force (test use) */
    int nsteps;
    const double *motion;    /* (nsteps+1) x 18: R[9] row-major, Omega[3], xG[3], uG[3] */
    int obj_kind, obj_n0, obj_n1, obj_norm;
    double obj_centre[3], obj_dir[3];
    const unsigned char *obj_mask; /* [ncell] or NULL (= every node) */
    int adj_form;            /* OR_ADJ_EXACT or OR_ADJ_PAPER (see or_step_T_paper) */
} or_desc;

/* 0 on success, negative on a malformed description. */
int or_validate(const or_desc *d);

/* Brinkman coefficient on the design grid and its derivative. */
int or_interp(const or_desc *d, const double *gamma, double *kref, double *kprime);

/* Transfer at step n: kappa[ncell], uS[3*ncell] are overwritten. */
int or_transfer(const or_desc *d, int n, const double *kref, double *kappa, double *uS);

/* Transpose of the transfer's kappa part: G[nd] += sum_x W_n(x,xi) kbar(x). */
int or_transfer_T(const or_desc *d, int n, const double *kbar, double *G);

/* One forward step (gradient, equilibrium, pull, force, boundary conditions). */
int or_step(const or_desc *d, const double *kappa, const double *uS, const double *rho,
            const double *u, double *rho_out, double *u_out);

/* Boundary conditions alone (used for the initial state). */
int or_apply_bc(const or_desc *d, double *rho, double *u);

/* Exact transpose of or_step for given (kappa, uS, u_prev = input velocity, u_cur = output
 * velocity).  (P, V) is the adjoint of the step's output; (P_out, V_out) that of its input.
 * kbar_out[ncell] receives d<lambda, out>/d kappa (overwritten). */
int or_step_T(const or_desc *d, const double *kappa, const double *uS, const double *u_prev,
              const double *u_cur, const double *P, const double *V, double *P_out,
              double *V_out, double *kbar_out);

/* The paper's own (continuous-then-discretised) adjoint step, Sec. 2.4 Eqs. arho_ex, au_ex,
 * as_ex: the same as or_step_T except that (i) the Brinkman source divides only the pulled
 * velocity moment 3 u~ (carried in U3, with the objective's u-seed) by (1 + kappa), not the whole
 * adjoint velocity, and (ii) the kappa seed is -(3 u~ / (1 + kappa)) . (u - u_S), from the pulled
 * moment alone.  U3 [3*ncell] in, U3_out [3*ncell] = 3 u~ of the new level.  Not the derivative
 * of any discrete map; pinned by its reduction to the exact step where (i) and (ii) vanish, the
 * closed-form gain of an adjoint shear wave under a uniform kappa, and central differences. */
int or_step_T_paper(const or_desc *d, const double *kappa, const double *uS, const double *u_prev,
                    const double *u_cur, const double *P, const double *V, const double *U3,
                    double *P_out, double *V_out, double *U3_out, double *kbar_out);

/* Objective density summed over the mask at one step (un-normalised), and its partials
 * (overwritten; any pointer may be NULL). */
double or_objective_step(const or_desc *d, const double *kappa, const double *uS,
                         const double *rho, const double *u);
int or_objective_partials(const or_desc *d, const double *kappa, const double *uS,
                          const double *rho, const double *u, double *dP, double *dV,
                          double *dK);

/* Full solve: forward (Algorithm 1) storing the whole trajectory, J, and when grad != NULL the
 * reverse sweep and dJ/dgamma.  jn[nsteps+1], rho_traj[(nsteps+1)*ncell] and
 * u_traj[(nsteps+1)*3*ncell] are optional outputs. */
int or_solve(const or_desc *d, const double *gamma, double *J, double *jn, double *grad,
             double *rho_final, double *u_final, double *rho_traj, double *u_traj);

/* threads used by the OpenMP loops */
int or_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
