/*
 * ipmg.h - C ABI of the MI355X (gfx950) library for the multigrid-preconditioned
 * conjugate-gradient solves of the primal-dual interior-point method for
 * minimum-compliance topology optimisation (Kocvara & Mohammed, "Primal-dual
 * interior-point multigrid method for topology optimization").
 *
 * Problem (Sec. 1, problem (1)): minimise (1/2) f'u subject to K(x) u = f,
 * sum x = V, 0 <= x <= xbar, with K(x) = sum_e x_e K_e on a structured grid of
 * unit square (2D, bilinear Q1, plane stress) or cube (3D, trilinear Q1)
 * elements, one density x_e per element (Sec. 7).
 *
 * Conventions shared by every call
 *   - Grid: nel[0] x nel[1] (x nel[2]) elements.  Element (i,j,k) has index
 *     e = (k*ny + j)*nx + i; node (i,j,k) has index q = (k*(ny+1) + j)*(nx+1) + i;
 *     DOF slot = dim*q + c (c = 0: x, 1: y, 2: z).  Vectors over DOFs are full
 *     slot vectors ("n_slots" doubles) in this node-major interleaved layout.
 *   - Every DOF of a node with i == 0 is clamped.  Outputs hold 0 there; the
 *     entries of inputs at clamped slots are ignored (treated as 0).
 *   - Vectors of the augmented Newton system Z (eq. (nwtr2Z), Sec. 2) have
 *     n_slots + 1 entries, the volume multiplier lambda last.
 *   - Pointers marked [device] are caller-owned device memory on the context's
 *     GPU, contiguous, 8-byte aligned; the library never frees them and keeps
 *     no reference after the call returns.  Pointers marked [host] are host
 *     memory.  Inputs and outputs must not alias unless stated.
 *   - All GPU work is enqueued on the stream given to ipmg_create; calls that
 *     return host results (status, info structs, host outputs) synchronise it.
 *   - Return value: IPMG_OK (0) or a negative IPMG_E* code.  No C++ exception
 *     crosses this interface.  ipmg_last_error() gives a message.  A context
 *     must not be used from two threads at once.
 */
#ifndef IPMG_H
#define IPMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  IPMG_OK = 0,
  IPMG_E_INVALID = -1,      /* null pointer, bad size or descriptor            */
  IPMG_E_DOMAIN = -2,       /* x outside (0, xbar], non-finite data, bad V      */
  IPMG_E_HIP = -3,          /* HIP runtime error                               */
  IPMG_E_NOMEM = -4,        /* device or host allocation failed                */
  IPMG_E_BREAKDOWN = -5,    /* p'Ap <= 0 or r'y <= 0 in PCG; coarse matrix not PD */
  IPMG_E_NOT_CONVERGED = -6,/* PCG hit maxit (outputs valid, info filled)      */
  IPMG_E_STALLED = -7,      /* interior-point step length below 1e-14          */
  IPMG_E_STATE = -8         /* call out of order (e.g. solve before setup)     */
};

enum { IPMG_OP_K = 0, IPMG_OP_Z = 1 };

typedef struct ipmg_ctx ipmg_ctx;

/* Discretisation and multigrid description (Sec. 5.1, Sec. 7). */
typedef struct {
  int dim;          /* 2 or 3                                                     */
  int nel[3];       /* elements per axis; nel[2] ignored in 2D; each divisible by
                       2^(levels-1)                                               */
  int levels;       /* number of multigrid levels, >= 1 (1 = direct solve only)   */
  double E, nu;     /* Young's modulus and Poisson ratio (1, 0.3)                 */
  int vcycle_fp32;  /* 1: V-cycle (smoothing, transfers, coarse operators) in FP32,
                       coarsest solve and PCG in FP64; 0: everything FP64          */
  int nu_pre, nu_post; /* damped-Jacobi sweeps before / after the coarse correction */
  double omega;     /* Jacobi damping (0.6)                                       */
  int pcg_flexible; /* 0: PCG ratio beta = r~'y~ / r'y (Algorithm PCG, Sec. 6);
                       1: Polak-Ribiere form r~'(y~ - y) / r'y, the same in exact
                       arithmetic with a fixed preconditioner and more robust when
                       the preconditioner varies between steps (FP32 V-cycle)      */
} ipmg_desc;

typedef struct {
  int iters;           /* PCG iterations (alpha updates)                          */
  int restarts;        /* true-residual restarts                                  */
  int status;          /* IPMG_OK / IPMG_E_BREAKDOWN / IPMG_E_NOT_CONVERGED       */
  double relres;       /* recurrence residual ||r|| / ||b|| at exit               */
  double true_relres;  /* ||A u - b|| / ||b|| recomputed at exit                  */
  double setup_ms;     /* hierarchy setup time for this system (0 if reused)      */
  double solve_ms;     /* PCG wall time                                           */
  double bu;           /* b'u of the returned u (the compliance f'u when b = f)   */
} ipmg_pcg_info;

typedef struct {
  double lambda;       /* multiplier of the last bisection trial                  */
  double volume;       /* sum of the new densities                                */
  int trials;          /* bisection trials                                        */
} ipmg_oc_info;

/* Interior-point state (Sec. 3.1): caller-owned device arrays plus host scalars. */
typedef struct {
  double* u;       /* [device] n_slots displacements                             */
  double* x;       /* [device] m densities                                       */
  double* phi;     /* [device] m multipliers of x >= 0                           */
  double* psi;     /* [device] m multipliers of x <= xbar                        */
  double lam;      /* volume multiplier                                          */
  double s, r;     /* barrier parameters                                         */
} ipmg_ip_state;

typedef struct {
  double V, xbar;     /* volume and upper bound of problem (1)                    */
  double sigma;       /* barrier reduction factor (0.2, Sec. 3.2)                  */
  double tau_nwt;     /* Newton test tolerance (0.1, Sec. 3.4)                     */
  double pcg_rtol;    /* relative residual tolerance of every PCG solve            */
  int pcg_maxit;      /* maximum PCG iterations per system (1000)                  */
  double frac;        /* fraction to the boundary (0.9, Sec. 3.3)                  */
  int step_all_blocks;/* 1: the 0.9 rule also keeps phi, psi > 0                   */
  int stop_rule;      /* 0: relative duality gap <= kkt_tol at a point passing the
                         Newton test; 1: max(s, r) <= tau_ip (eq. (crit:ip))       */
  double kkt_tol, tau_ip;
  int max_newton;     /* safety cap on Newton steps                               */
  double accept_rtol; /* a Newton solve stopped by pcg_maxit is taken as an inexact
                         direction only if its true relative residual is at most
                         this (1e-2: the paper's own inexact stopping rule, eq.
                         (cgstop)); otherwise, and after any breakdown, the step
                         fails and leaves the state unchanged                      */
} ipmg_ip_params;

typedef struct {
  double alpha;       /* step length taken                                         */
  double nwt;         /* ||F1||/||f|| + ||G3||/(||phi|| + ||psi||) after the step  */
  double gap;         /* (phi'x + psi'(xbar - x)) / f'u after the step             */
  double volume_res;  /* sum x - V after the step                                  */
  double compliance;  /* f'u after the step                                        */
  int pcg_iters;      /* PCG iterations of the Newton system                       */
  int pcg_status;     /* IPMG_OK, or IPMG_E_NOT_CONVERGED when the solve stopped at
                         pcg_maxit within accept_rtol (the step then used the last
                         iterate as an inexact Newton direction), or the status of
                         a failed solve (the step then returns it)                  */
  int barrier_updated;/* 1 if s, r were multiplied by sigma after this step        */
  int converged;      /* 1 if the stop rule holds                                  */
  double setup_ms, solve_ms;
  double pcg_true_relres; /* true relative residual of the Newton solve          */
  int pcg_retries;    /* 1 if the solve broke down and was continued from its last
                         iterate after the damping of every level was estimated
                         again (four times the power steps, product 1.2)           */
} ipmg_ip_info;

/* Create a context: grid, element matrix, level hierarchy storage and scratch.
 * hip_stream: a hipStream_t (NULL = default stream).  out: [host] receives the
 * context.  Errors: IPMG_E_INVALID (bad desc), IPMG_E_NOMEM, IPMG_E_HIP. */
int ipmg_create(const ipmg_desc* desc, void* hip_stream, ipmg_ctx** out);
void ipmg_destroy(ipmg_ctx* ctx);
const char* ipmg_last_error(const ipmg_ctx* ctx);
const char* ipmg_status_string(int status);

/* Sizes on a level (level = levels-1 is the finest, 0 the coarsest). [host] outputs. */
int ipmg_sizes(const ipmg_ctx* ctx, int level, int64_t* n_slots, int64_t* n_free, int64_t* m_elems);

/* Integer maps, computed by the library on the host (Sec. 7 grid; indexing above).
 * free_to_slot: [host] n_free entries, the slot of every free DOF in slot order.
 * slot_of_node: returns the slot of component c of node (i,j,k) on a level, or -1. */
int ipmg_dof_map(const ipmg_ctx* ctx, int level, int64_t* free_to_slot);
int64_t ipmg_slot_of(const ipmg_ctx* ctx, int level, int i, int j, int k, int c);

/* Element stiffness K0 of the unit element (Sec. 7: Q1, E, nu; 2x2(x2) Gauss rule),
 * computed on the GPU.  K0: [host] (dim*2^dim)^2 doubles, row-major, local DOF order
 * node-major (nodes counter-clockwise on face k, then face k+1). */
int ipmg_element_matrix(ipmg_ctx* ctx, double* K0);

/* Set the densities x (K(x) = sum_e x_e K_e, Sec. 1).  x: [device] m doubles, each in
 * (0, inf) and finite, else IPMG_E_DOMAIN.  The library copies x. */
int ipmg_set_density(ipmg_ctx* ctx, const double* x);

/* y = K(x) v on the finest grid in FP64 (matrix-free, element by element).
 * v, y: [device] n_slots.  Requires ipmg_set_density. */
int ipmg_apply_K(ipmg_ctx* ctx, const double* v, double* y);

/* Build the multigrid hierarchy for op (Sec. 5.1 Galerkin coarse operators, dense
 * Cholesky of the coarsest operator).  IPMG_OP_K uses the current densities;
 * IPMG_OP_Z uses the Newton-system data of the last ipmg_ip_prepare. */
int ipmg_mg_setup(ipmg_ctx* ctx, int op);

/* Damping weight and spectral-radius estimate of the Jacobi smoother on a level after
 * the last ipmg_mg_setup: omega_k = min(omega, 1.6 / rho_k), rho_k the Rayleigh
 * quotient of D_k^-1 A_k after 12 power iterations (30 for the augmented system Z)
 * from the vector (-1)^(i+j+k)(1+c)
 * (damped Jacobi diverges once omega * rho >= 2; Sec. 5.1 leaves the smoother open).
 * omega, rho: [host] outputs (rho = 0 on the coarsest level, which is solved directly). */
int ipmg_level_damping(ipmg_ctx* ctx, int level, double* omega, double* rho);

/* One V-cycle z = M r from the zero initial guess (Algorithm MG, Sec. 5.1).
 * r, z: [device] n_slots (+1 for IPMG_OP_Z) doubles.  In FP32 mode r is rounded
 * to FP32 on entry and z is widened on exit. */
int ipmg_vcycle(ipmg_ctx* ctx, int op, const double* r, double* z);

/* y = Z v for the augmented Newton matrix of the last ipmg_ip_prepare (FP64).
 * v, y: [device] n_slots + 1. */
int ipmg_apply_Z(ipmg_ctx* ctx, const double* v, double* y);

/* Algorithm PCG (Sec. 5.2) with one V-cycle per step, to ||r|| <= rtol ||b||,
 * confirmed by the true residual.  b: [device] right-hand side; u: [device]
 * initial guess on entry (zero it for a cold start), solution on exit.  Sizes as
 * in ipmg_vcycle.  info: [host] may be NULL.  Returns IPMG_OK, IPMG_E_BREAKDOWN or
 * IPMG_E_NOT_CONVERGED (u holds the last iterate). */
int ipmg_pcg(ipmg_ctx* ctx, int op, const double* b, double* u, double rtol, int maxit,
             ipmg_pcg_info* info);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): ipmg_pcg with its work
 * vectors (seven of n_slots + 1 doubles) and its reduction scratch in a static
 * device array of IPMG_NOALLOC_SCRATCH_BYTES that the library holds on each GPU
 * it runs on until the process ends, instead of the context's buffers.  The call
 * allocates nothing: it needs the hierarchy of op already built (ipmg_mg_setup,
 * or an earlier solve of the same operator at the current data), else
 * IPMG_E_STATE; a grid whose scratch (ipmg_pcg_noalloc_bytes) exceeds the array
 * gives IPMG_E_INVALID (in 2D up to about 1.1M DOF slots, e.g. 1024 x 512
 * elements).  Results equal those of ipmg_pcg bit for bit.  Every call on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU (two contexts on
 * different streams or threads) race and must be serialised by the caller.
 * Arguments, return values and the stream synchronisation as for ipmg_pcg. */
#define IPMG_NOALLOC_SCRATCH_BYTES (64u << 20)
int ipmg_pcg_noalloc(ipmg_ctx* ctx, int op, const double* b, double* u, double rtol, int maxit,
                     ipmg_pcg_info* info);
/* Bytes of the static scratch ipmg_pcg_noalloc needs for this context's grid (-1 for a
 * null context). */
int64_t ipmg_pcg_noalloc_bytes(const ipmg_ctx* ctx);

/* Element sensitivities g_e = scale * w_e' K0 u_e (B(u)' w of Sec. 2 scaled; with
 * w = lambda, scale = -1 this is the adjoint gradient -lambda_e' K_e u_e).
 * w, u: [device] n_slots; g: [device] m. */
int ipmg_element_sens(ipmg_ctx* ctx, const double* w, const double* u, double scale, double* g);

/* Interior-point method (Sec. 3).  ipmg_ip_init sets x = V/m, u = K(x)^-1 f (MG-PCG),
 * lambda = 1, phi = psi = 1, s = r = 1 (Sec. 3.1).  f: [device] n_slots load vector.
 * st: [host] struct whose device arrays the caller allocated (n_slots, m, m, m). */
int ipmg_ip_init(ipmg_ctx* ctx, const double* f, const ipmg_ip_params* prm, ipmg_ip_state* st,
                 ipmg_pcg_info* info);

/* Form the Newton system at st (residuals F1..F5, D, G3, augmented matrix data and
 * its right-hand side; Sec. 2, eqs. (nwtr2Z), (nwtr2rhs)).  rhs: [device] n_slots+1
 * output, may be NULL. */
int ipmg_ip_prepare(ipmg_ctx* ctx, const double* f, const ipmg_ip_params* prm,
                    const ipmg_ip_state* st, double* rhs);

/* One Newton step (Sec. 3.1 steps 1-4): prepare, MG-PCG on Z, recovery of d_x,
 * d_phi, d_psi, step length (Sec. 3.3), update, Newton test and barrier update
 * (Sec. 3.2, 3.4), stop rule.  Updates st in place.  info: [host] may be NULL.
 * A Newton solve that breaks down is continued once from its last iterate with
 * the damping estimated again (pcg_retries).  A Newton solve stopped by pcg_maxit
 * with a true relative residual within
 * accept_rtol gives an inexact direction (pcg_status IPMG_E_NOT_CONVERGED, the
 * step proceeds).  Returns IPMG_OK; IPMG_E_BREAKDOWN or IPMG_E_NOT_CONVERGED when
 * the Newton solve broke down or stopped above accept_rtol; IPMG_E_STALLED when
 * the step length is below 1e-14 or the direction is not finite; IPMG_E_DOMAIN
 * (non-finite iterate) or another error.  On every status but IPMG_OK and
 * IPMG_E_DOMAIN the state is left unchanged. */
int ipmg_ip_step(ipmg_ctx* ctx, const double* f, const ipmg_ip_params* prm, ipmg_ip_state* st,
                 ipmg_ip_info* info);

/* One density update of the Optimality Conditions methods (Sec. 4, Algorithms OC,
 * DOC, AOC): with the element energies E_e = u_e'K0u_e of the displacements u
 * (solved at the densities x),
 *   x_new_e = min(x_e E_e^q / lambda, xbar),
 * lambda from the bisection of Algorithm OC: bracket [0, lam_hi] (1e4 in the paper),
 * while it is wider than tau (1e-11) its midpoint is tried and the lower end is
 * raised when sum x_new > V, the upper end lowered otherwise; x_new is formed from
 * the fixed x at every trial and the last trial gives the result.  q = 1: OC;
 * q < 1: DOC (damping exponent, 1/2 in the paper).  blend (nullable): the AOC mean,
 * x_new = (blend + update) / 2.  The bisection runs on the device, OC_LEVELS
 * (5) levels of trials per pass, in the order of sequential bisection.
 * u: [device] n_slots; x, x_new, blend: [device] m (x_new may alias blend, not x);
 * info: [host] nullable.  Errors: IPMG_E_INVALID (V, xbar, q, lam_hi, tau not
 * positive and finite, or tau >= lam_hi). */
int ipmg_oc_update(ipmg_ctx* ctx, const double* u, const double* x, double V, double xbar, double q,
                   double lam_hi, double tau, const double* blend, double* x_new, ipmg_oc_info* info);

/* SIMP model with a density filter (Sec. 9).  Filtered densities x~ = W x, with
 * W^_ij = max(0, rmin - dist(i, j)) for the Manhattan distance of element centres
 * and every column of W scaled to sum one, W_:i = W^_:i / sum_j W^_ij (so
 * sum x~ = sum x).  transpose = 0: out = W in; 1: out = W' in.  in, out: [device] m
 * doubles, not aliased.  rmin in (0, 5].  Errors: IPMG_E_INVALID. */
int ipmg_filter(ipmg_ctx* ctx, double rmin, const double* in, double* out, int transpose);

/* Compliance and gradient of the SIMP model at the densities x (Sec. 9): x~ = W x,
 * K^ = sum_e x~_e^p K_e (the context's densities are set to x~^p), u = K^-1 f by
 * MG-PCG to rtol (zero start), c = f'u (info->bu), and
 *   grad_i = dc/dx_i = -sum_j W_ji p x~_j^(p-1) u_j'K0u_j,
 * the bracket of the paper's modified condition (KKT3).  x: [device] m, each in
 * (0, inf); f: [device] n_slots; u: [device] n_slots output; grad: [device] m output;
 * info: [host] nullable.  p >= 1, rmin in (0, 5].  Returns the status of the solve
 * (u and info valid, grad only on IPMG_OK), IPMG_E_DOMAIN for x~^p not positive and
 * finite, IPMG_E_INVALID for bad arguments.  The Newton system of the SIMP
 * interior-point method (B^(u) of Sec. 9) is not provided. */
int ipmg_simp_compliance(ipmg_ctx* ctx, const double* x, const double* f, double rmin, double p, double rtol,
                         int maxit, double* u, double* grad, ipmg_pcg_info* info);

/* Interior-point method on the SIMP model with the density filter (Sec. 9): the
 * method of Sec. 2-3 for min f'u with K^(x~) u = f, K^ = sum_e x~_e^p K_e, x~ = W x (the
 * filter of ipmg_filter, radius rmin, Manhattan distance), and B(u) of the Newton
 * system replaced by B^(u) = B(u) diag(p x~^(p-1)) W.  The Newton matrix
 * Z^ = [[K^ + B^ D^-1 B^', B^ D^-1 e], [e'D^-1 B^', e'D^-1 e]] is applied element by
 * element (its rank-one terms span the elements of a filter patch) inside PCG, which
 * a V-cycle of the element-local matrix with the couplings between the elements of
 * a patch dropped preconditions (border exact, corner chosen so that the matrix is
 * SPD).  init: the starting point of ip_init with K^ (x = V/m, phi = psi = 1,
 * lambda = s = r = 1, u = K^(x)^-1 f by MG-PCG).  step: one Newton step as
 * ipmg_ip_step (same parameters, state, acceptance rule, measures and return
 * codes).  rmin in (0, 5], pexp >= 1 (p, 3 in the paper), else IPMG_E_INVALID. */
int ipmg_simp_ip_init(ipmg_ctx* ctx, const double* f, const ipmg_ip_params* prm, double rmin, double pexp,
                      ipmg_ip_state* st, ipmg_pcg_info* info);
int ipmg_simp_ip_step(ipmg_ctx* ctx, const double* f, const ipmg_ip_params* prm, double rmin, double pexp,
                      ipmg_ip_state* st, ipmg_ip_info* info);

/* Kernel timing for roofline measurements.  Between begin and end, the launch of
 * the main kernel of every selected class (bit k of class_mask selects class k) is
 * bracketed by a pair of HIP events on the context's stream; the one-block
 * finalize kernels that follow some of them are not inside the bracket:
 *   0: damped-Jacobi sweep on the finest level from a nonzero iterate (V-cycle precision)
 *   1: FP64 finest-level apply of the PCG direction (p = -y + beta p, q = A p, p'q)
 *   2: residual pass on the finest level (V-cycle precision)
 *   3: fused PCG update (z += alpha p, r += alpha q, ||r||^2)
 *   4: damped-Jacobi sweep on the first coarse level from a nonzero iterate
 *   5: first damped-Jacobi sweep on the finest level (zero iterate)
 *   6: last post-smoothing sweep on the finest level with the fused PCG ratio
 *   7: fused pre-smoothing, residual and restriction on the first coarse level
 *   8: fused prolongation and post-smoothing on the first coarse level
 *   9, 10: reserved (no kernel records them)
 *  11: prolongation folded into the first post-smoothing sweep on the finest level
 *  12: the first two pre-smoothing sweeps on the finest level in one pass
 *  13: 3D finest level, element products of a V-cycle pass (before its node pass)
 *  14: 3D finest level, element products of the FP64 PCG direction
 * Launches skipped on device after convergence are recorded too (with near-zero
 * duration).  max_launches: event pairs to keep (further launches are not timed).
 * durations_ms: [host] capacity entries, each launch's duration; classes: [host,
 * nullable] capacity entries, each launch's class; launches: [host] number
 * recorded.  Both calls synchronise the stream.  IPMG_E_INVALID for an empty or
 * unknown mask or max_launches outside [1, 65536]. */
int ipmg_profile_begin(ipmg_ctx* ctx, unsigned class_mask, int max_launches);
int ipmg_profile_end(ipmg_ctx* ctx, double* durations_ms, int* classes, int capacity, int* launches);

#ifdef __cplusplus
}
#endif
#endif /* IPMG_H */
