/*
 * polardisk.h -- C ABI of the MI355X θ-scheme solver for the singular
 * parabolic equation and the drift-diffusion continuity equation on the unit
 * disk in polar coordinates (Zhang, Zhang, Song, Fang, "A Multidimensional
 * Self-Adaptive Numerical Simulation Framework for Semiconductor Boltzmann
 * Transport Equation", arXiv:2509.15879).
 *
 * What one time step computes.  With the implicit weight θ = 1 - a (a is the
 * weight of the old level in scheme (2.5) of §2.1 and in the Ch. 3 scheme of
 * §3.2.1) every step solves
 *
 *     (I/Δt + θ L_h) n^{k+1} = (I/Δt - (1-θ) L_h) n^k
 *                              + (1-θ) S(t_k) + θ S(t_{k+1}) + boundary terms,
 *
 * i.e. the linear system (2.11)/(2.12) of §2.2 and its Ch. 3 form (§3.2.3).
 * L_h is the conservative five-point polar operator: the diffusion part of
 * ϖ_h (§3.2.1, which reduces to ℘_h of §2.1 for D = 1), a face-flux drift
 * term for the vector field E = (E_r, E_θ), a reaction term b, and the
 * control-volume origin closure of §3.2.2 (the Swarztrauber-Sweet row of
 * §2.1 for D = 1, E = 0).  Meshes: the radial stretch (2.4), the angular and
 * time stretches of §3.1, the comparison stretch (2.13), or explicit nodes.
 *
 * Conventions.
 *  - Every function returns an int status: PD_OK (0) or a negative PD_E*
 *    code (PD_PENDING = 1 only from pd_batch_poll).  Nothing throws or
 *    aborts.  pd_last_error() returns a message for the calling thread's
 *    last failure (valid until that thread's next call).
 *  - Handles are opaque and owned by the library until pd_destroy /
 *    pd_batch_destroy.  Inputs are copied at create/submit time, so the
 *    caller may free them on return.  Output buffers belong to the caller.
 *  - Node vectors have N = m*n + 1 entries (the origin plus m rings of n
 *    angular nodes).  Layout PD_LAYOUT_RING: index 0 is the origin and node
 *    (i, j), i = 1..m, j = 0..n-1, sits at 1 + (i-1)*n + j.  Layout
 *    PD_LAYOUT_PAPER is the ordering of (2.12): index 0 is the origin and
 *    (i, j) sits at 1 + j*m + (i-1).
 *  - Face arrays are row-major.  Radial faces "i+1/2" (i = 0..m, face 0 joins
 *    the origin to ring 1, face m joins ring m to the boundary r = 1) are
 *    sampled at (r_{i+1/2}, θ_j) and stored at [i*n + j].  Angular faces
 *    "j+1/2" of ring i (i = 1..m, joining (i, j) and (i, j+1 mod n)) are
 *    sampled at (r_i, θ_{j+1/2}) and stored at [(i-1)*n + j].  The sample
 *    points come from pd_mesh_coords.
 *  - Pointers are host pointers unless a `device_ptrs`/`device_ptr` flag
 *    says they are device pointers (for instance torch tensor data_ptr()).
 *  - Errors: PD_EINVAL for bad arguments (m < 2, n < 4, θ outside (0, 1],
 *    Δt <= 0, non-monotone explicit meshes, NULL where data is required),
 *    PD_ENOMEM when device memory or the batch pool is exhausted, PD_EHIP
 *    for a HIP runtime failure, PD_EBREAKDOWN / PD_ENOCONV when the Krylov
 *    solve of some step broke down or hit its iteration cap, PD_EBUSY when an
 *    instance is owned by a running batch.
 */
#ifndef POLARDISK_H
#define POLARDISK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pd_instance pd_instance;
typedef struct pd_batch pd_batch;

enum {
  PD_OK = 0,
  PD_PENDING = 1,
  PD_EINVAL = -1,
  PD_ENOMEM = -2,
  PD_EBREAKDOWN = -3,
  PD_ENOCONV = -4,
  PD_EHIP = -5,
  PD_EBUSY = -6
};

typedef enum { PD_PARABOLIC = 0, PD_CONTINUITY = 1 } pd_pde;

/* PD_FP64: every vector, coefficient and Krylov scalar in FP64.
 * PD_MIXED: FP64 right-hand side, outer residual and origin-row sum; the
 * inner BiCGSTAB (stencil, sweeps, vectors) runs in FP32 and is refined
 * until the FP64 residual meets the tolerance.
 * In both precisions the preconditioner's tridiagonal factors (pivots,
 * multipliers, the Sherman-Morrison vector) are computed in FP64 and stored
 * in FP32: they define a fixed preconditioner, which moves the iterates but
 * not the converged solution.                                             */
typedef enum { PD_FP64 = 0, PD_MIXED = 1 } pd_precision;

enum { PD_MESH_UNIFORM = 0, PD_MESH_SINE = 1, PD_MESH_EXPLICIT = 2, PD_MESH_POLY = 3 };
enum { PD_LAYOUT_RING = 0, PD_LAYOUT_PAPER = 1 };
enum { PD_FLUX_CENTRAL = 0, PD_FLUX_UPWIND = 1, PD_FLUX_LITERAL = 2 };
enum { PD_TIME_UNIFORM = 0, PD_TIME_SINE = 1, PD_TIME_TABLE = 2, PD_TIME_ADAPTIVE = 3 };

/* Mesh (§2.1 "region divided", §3.1 stretching equations).
 *   r_kind: PD_MESH_UNIFORM r_i = i h; PD_MESH_SINE r_i = sin((i h)^p π/2)
 *           (eq. (2.4)); PD_MESH_POLY r_i = 1 - (1 - i h)^{p+1} (eq. (2.13));
 *           PD_MESH_EXPLICIT: r_explicit holds r_0..r_{m+1} (host, strictly
 *           increasing, r_0 = 0, r_{m+1} = 1).  h = 1/(m+1).
 *   th_kind: PD_MESH_UNIFORM θ_j = 2πj/n; PD_MESH_SINE θ_j = 2π sin((j/n)^q π/2)
 *           (§3.1 angular stretch); PD_MESH_EXPLICIT: th_explicit holds
 *           θ_0..θ_n (host, strictly increasing, θ_0 = 0, θ_n = 2π).
 *   nr = m >= 2 unknown rings, ntheta = n >= 4 angular nodes.             */
typedef struct {
  int32_t nr, ntheta;
  int32_t r_kind;
  double p;
  int32_t th_kind;
  double q;
  const double *r_explicit;
  const double *th_explicit;
} pd_mesh_desc;

/* PDE data (eqs. (2.1)-(2.3), (3.1)-(3.4)): n_t + L n = S(t) with
 * L n = -∇·(D∇n) + ∇·(nE) + b n and Dirichlet data N(t, θ) on r = 1.
 *   pde:  PD_PARABOLIC or PD_CONTINUITY (informational; both use the arrays).
 *   flux: 0 central drift average (n_P + n_Q)/2 (the origin choice of
 *         §3.2.2), 1 upwind drift, 2 PD_FLUX_LITERAL: the operator ϖ_h of
 *         §3.2.1 and the origin row of §3.2.2 as printed (scalar E at the
 *         nodes, one-sided drift differences; not conservative).  It needs
 *         E_node and D_origin and Dirichlet data; Er/Et faces are ignored.
 *         Kept to reproduce the paper's Ch. 3 tables.
 *   bc:   0 Dirichlet on r = 1, 1 zero flux through r = 1.
 *   D_rface, Er_rface: (m+1)*n radial-face samples, NULL means D = 1 / E_r = 0.
 *   D_tface, Et_tface: m*n angular-face samples, NULL means D = 1 / E_θ = 0.
 *   b_node: N node values in `layout` (NULL means b = 0).
 *   Time modes q = 0..nsrc-1 (nsrc <= 4): τ_q(t) = t^{tpow_q} exp(λ_q t),
 *   S(t) = Σ_q τ_q(t) g_q with g: nsrc*N node values in `layout` (the origin
 *   entry is the source's limit at r = 0, §3.2.2 source integral), and
 *   N(t, θ_j) = Σ_q τ_q(t) nb_q[j] with nb: nsrc*n values (NULL means 0).
 *   tpow may be NULL (all 0).
 *   u0: N initial values in `layout` (eq. (2.10) / (3.3)).
 *   device_ptrs: 1 if every array above (lambda and tpow included) is a
 *   device pointer; they are copied to the host at creation.
 *   E_node, D_origin (PD_FLUX_LITERAL only): the scalar field E at the N
 *   nodes in `layout` (E_node follows device_ptrs), and D at the origin.   */
typedef struct {
  int32_t pde;
  int32_t flux;
  int32_t bc;
  int32_t layout;
  int32_t device_ptrs;
  const double *b_node;
  const double *D_rface, *Er_rface;
  const double *D_tface, *Et_tface;
  int32_t nsrc;
  const double *lambda;
  const int32_t *tpow;
  const double *g;
  const double *nb;
  const double *u0;
  const double *E_node;          /* PD_FLUX_LITERAL only */
  double D_origin;               /* PD_FLUX_LITERAL only */
} pd_problem_desc;

/* Time levels (§2.1 Δt = T/K; §3.1 t_k = V(k T/K), V(t) = T sin((t/T)^l π/2);
 * or an explicit table t_0..t_K, host, strictly increasing).  The solve
 * starts from the instance's current state and time, which must equal t_0.
 *   theta: implicit weight θ = 1 - a in (0, 1]; 0.5 is Crank-Nicolson,
 *          1 is backward Euler.
 *   tol:   per-step stopping tolerance on the diagonally scaled residual
 *          ||D^{-1}(b - A x)||_2 / ||D^{-1} b||_2 (FP64), D = diag(A); every
 *          row weighs alike, whatever the local mesh spacing.
 *   max_iters: cap on BiCGSTAB iterations per step (0: library default).
 * PD_TIME_ADAPTIVE (the paper fixes its levels in advance; this is an
 * a-posteriori step control of the same scheme): advances from the current
 * time t_s to t_s + T choosing each Δt on the GPU from a local error
 * estimate of the step just taken, with f(t, x) = -L x + S(t) + c N(t) the
 * semi-discrete right-hand side: (θ - 1/2) Δt (f_{k+1} - f_k) for θ ≠ 1/2,
 * the trapezoidal rule against the variable-step Adams-Bashforth-2
 * predictor for θ = 1/2.  e = ||d||_2 / ||x_{k+1}||_2 (relative); a step with
 * e > 2 tol_time (and Δt > dt_min) is retaken smaller, an accepted one sets
 * the next Δt = Δt clamp(0.9 (tol_time/e)^{1/(q+1)}, 1/2, 2) within
 * [dt_min, dt_max] (q = 1, or 2 for θ = 1/2); the first step is dt0 and the
 * second tries dt0 again; steps land exactly on t_s + T.  K caps the number
 * of accepted steps (PD_ENOCONV if T is not reached); per-step statistics
 * past the steps taken are zero.  Not accepted by pd_batch_submit.
 * Bounds of a solve call: the library stops launching work and returns
 * PD_ENOCONV ("wall-clock limit") once max_seconds have passed on the host
 * (the smallest limit of a batch applies), and once the batch has used the
 * Krylov cycles its levels can need: levels x attempts per level x
 * (max_iters + refinements + 8), where an adaptive solve can take at most
 * ceil(T/dt_min) + 2 accepted steps and ceil(ln(dt_max/dt_min)/ln 1.4) + 1
 * rejected attempts per step (each rejection shrinks Δt by at least 1/1.4).
 * After either stop the instances keep the last completed level (their
 * time says which) and may be solved again.                              */
typedef struct {
  int32_t t_kind;
  int32_t K;
  double T, l;
  const double *t_table;
  double theta;
  double tol;
  int32_t max_iters;
  double dt0, dt_min, dt_max;   /* PD_TIME_ADAPTIVE only                  */
  double tol_time;              /* PD_TIME_ADAPTIVE: local error tolerance */
  double max_seconds;           /* host wall-clock limit of the solve call
                                   (0: 600 s); see below                   */
} pd_time_desc;

typedef struct {
  int32_t iters;        /* Krylov iterations (inner, for PD_MIXED)         */
  int32_t refinements;  /* FP64 outer refinements (PD_MIXED), else 0       */
  int32_t status;       /* PD_OK, PD_EBREAKDOWN or PD_ENOCONV              */
  int32_t reserved;     /* Krylov restarts                                 */
  double rel_resid;     /* final scaled relative residual (see tol)        */
  double dt, t;         /* step size and the time reached (0: no step)     */
  double err_time;      /* adaptive stepping: the step's local error estimate e */
  int32_t rejected;     /* adaptive stepping: attempts rejected before it  */
  int32_t pad;
} pd_step_stats;

/* Mesh nodes and face sample points of a mesh description: r_nodes r_0..r_{m+1}
 * (m+2), r_faces r_{1/2}..r_{m+1/2} (m+1), th_nodes θ_0..θ_n (n+1), th_faces
 * θ_{1/2}..θ_{n-1/2} (n), all host buffers owned by the caller (any may be
 * NULL).  Pure host computation (§2.1, §3.1 mesh formulas).              */
int pd_mesh_coords(const pd_mesh_desc *mesh, double *r_nodes, double *r_faces,
                   double *th_nodes, double *th_faces);

/* The time levels t_0..t_K (K+1 values, host buffer owned by the caller)
 * that a solve with this descriptor advances through from t_start: the
 * sine-stretched schedule t_k = t_start + T sin((k/K)^l π/2) (§3.1), the
 * uniform one, or the explicit table (then t_0 must equal t_start).
 * PD_EINVAL for K < 1, T <= 0, l <= 0 or levels that do not increase.
 * Pure host computation.                                                  */
int pd_time_levels(const pd_time_desc *time, double t_start, double *out);

/* Creates an instance: builds the mesh, turns the sampled coefficients into
 * face conductances and drift coefficients, uploads everything to the
 * current HIP device, and sets the state to u0 at t = 0.  hip_stream may be
 * NULL: the instance then uses a default-priority stream the library owns,
 * one per device and shared by every such instance (so they can be
 * batched together).                                                     */
int pd_mesh_create(const pd_mesh_desc *mesh, const pd_problem_desc *problem,
                   int32_t precision, void *hip_stream, pd_instance **out);

/* One θ-scheme step from the current state at t_k to t_k + dt. */
int pd_scheme_step(pd_instance *inst, double t_k, double dt, double theta, double tol,
                   pd_step_stats *stats);

/* All K steps of a time description; per_step (K entries) may be NULL. */
int pd_solve_to_T(pd_instance *inst, const pd_time_desc *time, pd_step_stats *per_step);

/* Advances several instances together: every kernel launch covers all of
 * them (uneven sizes and PDE types allowed).  times[q] belongs to insts[q];
 * per_step (count pointers, may be NULL; each per_step[q] NULL or an array
 * of times[q].K entries) receives every step's statistics.  All instances
 * must share one stream.  Results equal those of solving each instance
 * alone (the reductions of an instance depend only on its own tiling).   */
int pd_solve_batch(pd_instance *const *insts, int32_t count, const pd_time_desc *times,
                   pd_step_stats *const *per_step);

/* Current state n^k (N values) in the requested layout. */
int pd_get_solution(const pd_instance *inst, double *out, int32_t layout, int32_t device_ptr);

/* The time of the instance's current state (0 after create, else the last
 * level reached or the time given to pd_set_solution).                   */
int pd_get_time(const pd_instance *inst, double *t);

/* Replaces the state by `in` (N values) at time t (checkpoint resume). */
int pd_set_solution(pd_instance *inst, const double *in, int32_t layout, int32_t device_ptr,
                    double t);

/* Diagnostics on the same kernels the solver uses:
 *   pd_apply_operator: y = (I/dt + θ L_h) x with the homogeneous boundary
 *   (N = 0), in FP64 (precision 0) or through the FP32 inner stencil (1).
 *   pd_assemble_rhs: the right-hand side of the step t_k -> t_k + dt from the
 *   current state (§2.2 eq. (2.11), §3.2.3 e_ij).                         */
int pd_apply_operator(pd_instance *inst, double dt, double theta, const double *x, double *y,
                      int32_t layout, int32_t device_ptrs, int32_t precision);
int pd_assemble_rhs(pd_instance *inst, double t_k, double dt, double theta, double *rhs,
                    int32_t layout, int32_t device_ptr);

/* pd_apply_preconditioner (diagnostic): z = M^{-1} y for the preconditioner
 * the solver builds for the step system A = I/dt + θ L_h of (2.11)/(2.12)
 * (the paper solves that system directly; the preconditioner is the
 * library's).  The Krylov iteration works on the diagonally scaled system
 * D^{-1} A (D = diag A), and M = (I + D^{-1} R)(I + D^{-1} Θ): R holds the
 * radial (same θ-line) couplings of the ring nodes -- the tridiagonal blocks
 * A_j of (2.12) -- and Θ the angular (same-ring, periodic) couplings plus
 * the couplings between the origin and ring 1 (an arrow system).
 * z = (I + D^{-1}Θ)^{-1} (I + D^{-1}R)^{-1} y.  The factors are computed in
 * FP64 and stored in FP32, and a mixed-precision instance applies M in FP32,
 * so z agrees with the exact M^{-1} y to about FP32 rounding.  y, z: N
 * values in `layout`, host or device (device_ptrs).  The instance's state
 * and time are not changed.  With the multigrid preconditioner
 * (pd_set_preconditioner) z is its V-cycle instead, whose first step is
 * this M^{-1} y.                                                          */
int pd_apply_preconditioner(pd_instance *inst, double dt, double theta, const double *y, double *z,
                            int32_t layout, int32_t device_ptrs);

/* Two carriers coupled through their field.  §3.1 states the continuity
 * equations of electrons n and holes p, each with the drift of a field,
 * and then solves one of them, (3.1), with the field given.  These calls
 * couple two carrier instances through a polar Poisson problem
 * -∇·(ε∇ψ) = p - n + C, 𝓔 = -∇ψ, in scaled units, by Gummel's iteration.
 * Each carrier is (3.1) with the drift velocity E = s μ 𝓔 (3.4), s = -1 for
 * electrons and +1 for holes, on the conservative face-flux operator; the
 * drift of a face comes from the potential's difference across it:
 *   radial face (i+1/2, j):  E_r = s μ (ψ_{i,j} - ψ_{i+1,j}) / h_{i+1},
 *   angular face (i, j+1/2): E_θ = s μ (ψ_{i,j} - ψ_{i,j+1}) / (r_i μ_{j+1}),
 * ψ_{0,j} the origin value and ψ_{m+1,j} the potential's Dirichlet value.
 *
 * pd_set_mobility: makes `carrier` a carrier of charge sign `sign` (+1 or
 * -1) with face mobilities mu_rface ((m+1) n values at (r_{i+1/2}, θ_j)) and
 * mu_tface (m n values at (r_i, θ_{j+1/2})), the layout of D_rface and
 * D_tface, host or device (device_ptrs).  The carrier must be an FP64
 * instance with the central or upwind flux created without drift
 * (Er_rface = Et_tface = 0 or NULL); its faces then hold the conductances,
 * which it keeps.  Allocates a small device array (2 words per face), freed
 * by pd_destroy.  PD_EINVAL otherwise.
 *
 * pd_gummel_step: one time level t_k -> t_k + dt of the coupled system.
 * `psi` is the potential: an FP64 continuity instance on the same mesh with
 * D = ε, no drift, Dirichlet data ψ_b, source mode 0 its charge slot (its g
 * is overwritten with p - n) and any further modes the doping C; every mode
 * steady (lambda = tpow = 0).  From the carriers' states (n^k, p^k), repeat:
 * ψ <- the steady solve of the potential (a θ = 1 level of length 1e30
 * from its last state) with the charge p - n; the carriers' faces from ψ;
 * (n, p) <- one θ-level t_k -> t_k + dt from (n^k, p^k); until the relative
 * max-norm change of ψ between iterations is at most gummel_tol (checked
 * from the second iteration on) or max_gummel iterations.  tol is the
 * per-solve scaled-residual tolerance.  On return the carriers hold
 * n^{k+1}, p^{k+1} at t_k + dt and psi the last potential; stats (or NULL)
 * gets the Gummel and Krylov iteration counts and the last change.  The
 * carriers must share one stream; no other call may use the three
 * instances during the call.  PD_EINVAL for mismatched meshes or settings,
 * the solve's codes otherwise.                                            */
typedef struct {
  int32_t gummel_iters;   /* Gummel iterations taken */
  int32_t krylov_iters;   /* Krylov iterations over all solves of the step */
  double change;          /* last relative max-norm change of ψ */
} pd_gummel_stats;
int pd_set_mobility(pd_instance *carrier, const double *mu_rface, const double *mu_tface, double sign,
                    int32_t device_ptrs);
int pd_gummel_step(pd_instance *psi, pd_instance *n_carrier, pd_instance *p_carrier, double t_k, double dt,
                   double theta, double tol, double gummel_tol, int32_t max_gummel, pd_gummel_stats *stats);

/* Device bytes an instance of this mesh and precision occupies. */
int pd_footprint(const pd_mesh_desc *mesh, int32_t nsrc, int32_t precision, size_t *bytes);

int pd_destroy(pd_instance *inst);

/* Adaptivity.  The paper's adaptivity is the choice of the exponent p of
 * the radial stretch (2.4) (α = pσ in Theorem 2.1); how a run picks or
 * changes p is left open (§4.2).  These calls supply the indicator and the
 * transfer; the caller samples its problem on the new mesh and creates the
 * new instance itself (coefficients are caller data).
 *
 * pd_error_indicator: at every ring node of the current state (time of the
 * last solve), from the second divided differences on the mesh,
 *   δ_r² n = 2[(n_{i+1,j}-n_{i,j})/h_{i+1} - (n_{i,j}-n_{i-1,j})/h_i]/(h_i+h_{i+1}),
 *   δ_θ² n = 2[(n_{i,j+1}-n_{i,j})/μ_{j+1} - (n_{i,j}-n_{i,j-1})/μ_j]/(μ_j+μ_{j+1}),
 * (ring 0 the origin, ring m+1 the Dirichlet value, or ring m again for
 * zero flux; j periodic):  η_ij = max(ĥ_i² |δ_r² n|, Δθ_j² |δ_θ² n|),
 * ĥ_i = (h_i+h_{i+1})/2, Δθ_j = (μ_j+μ_{j+1})/2.  kappa (m values, may be
 * NULL) receives κ_i = max_j |δ_r² n|; eta (m*n values, ring-major
 * (i-1)*n + j, may be NULL) the indicator.  Among the stretches (2.4) with
 * the same m and the exponents p_candidates, out->p_best minimises the
 * predicted largest radial indicator P(p) = max_k ĥ'_k² κ(r'_k) (κ linear
 * in r between nodes; the first of equal ones); out->recommend is 1 when
 * P(p_best) <= 0.8 P(p_current).  Host buffers owned by the caller.        */
typedef struct {
  double eta_max, eta_sum;
  int32_t i_max, j_max;      /* ring 1..m and angle index of eta_max (first) */
  double p_best;
  double pred_best, pred_current;
  int32_t recommend;
  int32_t reserved;
} pd_indicator;
int pd_error_indicator(pd_instance *inst, double p_current, const double *p_candidates,
                       int32_t n_candidates, double *kappa, double *eta, pd_indicator *out);

/* pd_error_indicator_noalloc: for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Computes what pd_error_indicator computes, with the
 * same kernel and the same host arithmetic (identical results), and calls
 * no hipMalloc, hipFree or other allocating routine.  The per-ring values
 * go through a fixed device array of 4*2048 doubles (64 KiB) that each GPU
 * the library runs on holds until the process ends.
 *   eta_device: NULL, or a DEVICE pointer to m*n doubles (ring-major
 *   (i-1)*n + j) owned by the caller, which receives the indicator field;
 *   kappa and out are host buffers as for pd_error_indicator.
 * Limits and errors: PD_EINVAL for m > 2048 (larger than any instance the
 * library creates) and for the arguments pd_error_indicator refuses.  The
 * call waits for its kernel on the instance's stream.  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (from several
 * host threads, or on several streams) race and may return each other's
 * values; serialise them.                                                  */
int pd_error_indicator_noalloc(pd_instance *inst, double p_current, const double *p_candidates,
                               int32_t n_candidates, double *kappa, double *eta_device,
                               pd_indicator *out);

/* pd_remesh_transfer: sets the state of `to` (another mesh of the same
 * problem and boundary condition) from the current state of `from` by
 * tensor cubic Lagrange interpolation: radially along each θ-line of
 * `from` on the nodes r = 0 (the origin value), r_1..r_m and, for
 * Dirichlet data, r = 1 (the boundary value at the current time), each
 * target radius taking the four consecutive nodes around it (shifted
 * inwards at the ends); then periodically in θ.  The origin value is kept;
 * `to` takes the time of `from` and restarts its extrapolated guesses.
 * PD_EINVAL for zero flux with m < 3 or instances on different devices.   */
int pd_remesh_transfer(pd_instance *from, pd_instance *to);

/* Serving: a request loop with continuous batching.  pd_batch_create starts
 * a host worker thread that owns a HIP stream (the caller's, or its own when
 * hip_stream is NULL) and a device-memory budget of hbm_pool_bytes.
 *   pd_batch_submit copies the request's inputs (host or device arrays, as
 *   the problem says) and returns at once with a ticket; it never waits on
 *   the GPU.  PD_ENOMEM if the request alone exceeds the pool, PD_EINVAL for
 *   inputs pd_mesh_create or pd_solve_to_T would reject.  The request starts
 *   from its u0 at t = 0 and advances through the time levels of `time`.
 *   The worker admits pending requests in arrival order at time-level
 *   boundaries while fewer than max_slots are active and their footprints
 *   (pd_footprint plus the time table) fit the pool; every admitted request
 *   then takes its levels in the same batched launches as the others
 *   (requests of any mesh size, PDE and precision mix), and leaves the batch
 *   when its last level ends.  A request's result does not depend on which
 *   others share its launches (every reduction and sweep of an instance
 *   depends only on the instance).
 *   pd_batch_poll returns PD_PENDING while the request is queued or running;
 *   then its outcome (PD_OK, or the first error of its solve), copies the
 *   final state (N values in the problem's layout, host buffer owned by the
 *   caller, may be NULL) to out and its summary to summary (may be NULL);
 *   the poll that reports an outcome releases the ticket (later polls of it
 *   return PD_EINVAL).
 *   pd_batch_stats fills the loop's counters.
 *   pd_batch_destroy stops the worker at the next level boundary, drops
 *   unfinished requests and frees everything.  The calls are thread safe.  */
typedef struct {
  int32_t status;        /* outcome, as returned by the poll                */
  int32_t levels;        /* time levels taken                               */
  int32_t iters;         /* Krylov iterations summed over the levels        */
  int32_t refinements;   /* FP64 refinements summed over the levels (mixed) */
  double max_rel_resid;  /* largest final scaled residual of a level        */
  double t;              /* time reached                                    */
  double queue_s;        /* submit -> admission, seconds (host clock)       */
  double latency_s;      /* submit -> result ready, seconds                 */
} pd_request_summary;

typedef struct {
  int32_t pending;       /* submitted, not yet admitted                     */
  int32_t active;        /* admitted, stepping                              */
  int32_t peak_active;   /* most requests active at once                    */
  int32_t reserved;
  uint64_t submitted, completed, slices_run, plans_built;
  size_t used_bytes, peak_bytes;   /* admitted footprint, now and at most   */
  double build_s;        /* worker time building launch plans and graphs    */
  double admit_s;        /* worker time uploading admitted requests         */
  double retire_s;       /* worker time reading back and freeing results    */
  double run_s;          /* worker time launching slices and waiting on them */
} pd_batch_info;

int pd_batch_create(size_t hbm_pool_bytes, int32_t max_slots, void *hip_stream, pd_batch **out);
int pd_batch_submit(pd_batch *batch, const pd_mesh_desc *mesh, const pd_problem_desc *problem,
                    const pd_time_desc *time, int32_t precision, uint64_t *ticket);
int pd_batch_poll(pd_batch *batch, uint64_t ticket, double *out, pd_request_summary *summary);
int pd_batch_stats(pd_batch *batch, pd_batch_info *info);
int pd_batch_destroy(pd_batch *batch);

/* Preconditioner of an instance's later solves.  The paper solves every
 * level's system (2.11)/(2.12) directly and names multigrid-type
 * preconditioners as the way to large grids (§4.2, outlook); the library's
 * Krylov solver offers two:
 *   PD_PRECOND_LINE (default): M above, the alternating line sweeps;
 *   PD_PRECOND_MG: a θ-semi-coarsening multigrid V-cycle built on them.
 *     Level l+1 merges the θ-lines of level l in pairs (the last three when
 *     n_l is odd) while n_l >= 16, by the Galerkin product of the
 *     volume-weighted system (radial faces add, the angular face inside a
 *     merged cell drops out, volumes add); the ring means (one value per
 *     ring and the origin) lie below the last level and are solved directly.
 *     Every level smooths with one step of its own line sweeps before and
 *     after its coarse correction.  It costs about three line-preconditioned
 *     iterations per iteration and pays where iterations are many: cold
 *     starts, large steps, steady problems (the potential of
 *     pd_gummel_step is solved with it when its instance has it).
 * The multigrid preconditioner takes FP64 instances.  They batch with other
 * FP64 instances (each V-cycle runs after the batch's own sweeps in every
 * Krylov iteration); a batch that also holds a mixed-precision instance
 * fails with PD_EINVAL.  Its levels (about 150 bytes per unknown) are
 * allocated by the instance's next solve that needs them and kept until
 * PD_PRECOND_LINE is set again or the instance is destroyed.
 * Solutions agree with either preconditioner to the solve's tolerance.
 * PD_EINVAL: unknown kind, or PD_PRECOND_MG on a mixed-precision instance;
 * PD_EBUSY while the instance is in use.                                  */
enum { PD_PRECOND_LINE = 0, PD_PRECOND_MG = 1 };
int pd_set_preconditioner(pd_instance *inst, int32_t kind);

/* Launch schedule (process-wide default for later solves and serving
 * plans).  groups: a batch is split into this many parts (by cells, largest
 * first, each to the part with the fewest), each stepping on its own stream
 * (the instances' stream and library-owned streams of default priority), so
 * that the parts' launches overlap; results do not depend on it.
 * cycles_per_graph: Krylov cycles per captured HIP graph, a round (a part's
 * active-instance count is read back after each round).  An instance can
 * only start a level at a round head, so rounds about as long as a level's
 * iterations suit batch solves; the serving loop caps them at 4 cycles.
 * stencil_rings: rings per wave of the stencil tiles, 4 or 8 (0 = 4), for
 * every instance; deeper tiles halve the stencil blocks, their edge reads
 * and the partial sums that later kernels read.  It changes the summation
 * order of an instance's partial sums, so results are the same alone and
 * batched under one schedule, not across schedules.
 * NULL restores groups = 1, cycles_per_graph = 2, stencil_rings = 4.
 * PD_EINVAL outside [1, 8] / [1, 16] / {0, 4, 8}.                          */
typedef struct {
  int32_t groups;
  int32_t cycles_per_graph;
  int32_t stencil_rings;
} pd_schedule;
int pd_set_schedule(const pd_schedule *schedule);
int pd_get_schedule(pd_schedule *schedule);

/* Kernel timing (diagnostics).  While enabled, every kernel launch of the
 * solver goes through hipExtLaunchKernel with a start and a stop event that
 * the dispatch itself stamps, so each launch's execution time (no launch
 * gaps) is added to its family's total (families PD_KF_*: one per kernel of
 * the Krylov cycle, PD_KF_MG for every launch of a multigrid V-cycle beyond
 * the instance's own sweeps; a level is synchronised after it ends so the events can
 * be read, and captured graphs are not used meanwhile).  total_ms /
 * launches (PD_KF_N entries each, may be NULL) receive the totals since the
 * last reset.                                                             */
enum { PD_KF_BEGIN = 0, PD_KF_FACTOR = 1, PD_KF_RAD_P = 2, PD_KF_ANG_P = 3, PD_KF_STEN_V = 4,
       PD_KF_RAD_S = 5, PD_KF_ANG_S = 6, PD_KF_STEN_T = 7, PD_KF_UPDATE = 8, PD_KF_REFINE = 9,
       PD_KF_CONTROL = 10, PD_KF_LEVEL_END = 11, PD_KF_MG = 12, PD_KF_N = 13 };
int pd_kernel_timing(int32_t enable, int32_t reset, double *total_ms, int64_t *launches);

const char *pd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* POLARDISK_H */
