// Device-side data structures shared by the HIP kernels and the host runtime
// of the polar-disk θ-scheme solver.
//
// Internal vector layout (per instance): ring-major, node (i, j) of ring
// i = 1..m at (i-1)*n + j, the origin at m*n, padded with zeros to npad.
// Face arrays hold, per face, the two coefficients of the numerical flux
// from its inner/lower node P to its outer/upper node Q:
//     F = gp * x_P - gm * x_Q,
// with gp = G + K/2, gm = G - K/2 for the central drift average and
// gp = G + max(K,0), gm = G - min(K,0) for upwinding (G the diffusive
// conductance, K the drift coefficient of the face).  Radial face i+1/2
// (i = 0..m) is stored at i*n + j, angular face j+1/2 of ring i at
// (i-1)*n + j.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PD_MAXSRC 4
#define PD_RB 4           // rings per stencil wave (one wave = 64 columns x rb rings; a schedule may ask for 2 PD_RB)
#define PD_STEN_WAVES 4   // waves per stencil block, stacked over consecutive rings
#ifndef PD_ELEM_PER_BLOCK
#define PD_ELEM_PER_BLOCK 2048
#endif
#define PD_RAD_THREADS 1024
#define PD_RAD_BMAX 32    // max rows per radial segment held in registers
#define PD_ANG_BMAX 32    // max angular nodes per lane held in registers
#define PD_NSLOT 4
#define PD_REFACTOR_DT 0.25   // relative change of Δt that triggers a new factorisation
#define PD_LSTAT 10           // statistics per level (see end_level)
#define PD_NHIST 4        // earlier levels kept for the initial guess: n^k .. n^{k-3}
#define PD_NSOL 5         // rotating solution slots: the PD_NHIST levels and the iterate
#define PD_RANNACHER 2    // backward-Euler steps that start an adaptive Crank-Nicolson solve
#define PD_STALL 20       // steps at dt_min above the error tolerance that end an adaptive solve
#define PD_NBEGIN 2        // partials of the level-begin pass: ||D^-1 b||², ||D^-1 r||²
// partials of the Gram pass: Z Z^T (upper triangle), Z r_c for both
// candidates, ||r_c||² for both, S0 of n^k (the earlier levels' S0 are kept
// in PdScalars::s0h from their own Gram passes)
#define PD_GRAM_S0 (10 + 2 * PD_NHIST + 2)
#define PD_NGRAM (PD_GRAM_S0 + 1)

// Slot holding n^{k-back} (back = 0..3) or, for back = -1, the iterate of
// the level under way, under rotation `rot`.
__host__ __device__ inline int sol_slot(int rot, int back) { return (rot + 3 - back) % PD_NSOL; }

enum { ST_IDLE = 0, ST_ACTIVE = 1, ST_DONE = 2, ST_BREAKDOWN = 3, ST_NOCONV = 4 };
enum { PH_INNER = 0, PH_OUTER = 1 };
// What the next radial p-sweep closes: an update step, a level's begin, a refinement.
enum { PEND_UPDATE = 0, PEND_BEGIN = 1, PEND_REFINE = 2 };
// Stage of an instance's level: its factorisation and right-hand side are
// due (START), or it is iterating (ITER).
enum { STAGE_ITER = 0, STAGE_START = 1 };


struct PdScalars {
  // time level
  double t0, t1, dt, inv_dt, theta;
  double ex_w[2][PD_NHIST]; // two polynomial candidate guesses: Σ_a w[c][a] n^{k-a}
  int ex_n;                 // earlier levels beyond n^k the guesses use (0..3)
  int guess_kind;           // the guess taken: candidate 0 or 1, plus 2 with the least-squares correction
  double guess_w[PD_NHIST]; // its weights (set by the level-begin stencil)
  double cq[PD_MAXSRC];
  double tol, tol_inner;
  double fact_dt, fact_theta;
  int maxit, level, K, refactor;
  int status, phase, iters, outer;
  int inner_iters, restarts, first, reset_rh;
  int inner_first, have_prev, rot, nfail;
  int max_outer, maxit_inner, total_iters, pad1;
  int pend, restarted;      // what the next radial p-sweep closes; restart flag
  int stage, in_level;      // STAGE_* of the level under way; a level has been started
  // Krylov scalars
  double rho_next, rho_cur; // ρ of this iteration (set by the p-sweep), of the last (by the s-sweep)
  double alpha, omega;
  double bnorm2, rnorm2, r0norm2;
  double rel_resid;
  double t_now;
  double rout0[2];          // FP64 outer residual at the origin (mixed), by refinement parity
  // adaptive time stepping: the next level's Δt is chosen from the local
  // error estimate of the step just taken (time levels written on the fly)
  int adaptive, need_f0;    // adaptive mode; f(t_0, x_0) not formed yet
  int nrej, pad5;           // rejected attempts of the level under way
  double t_end, dt_min, dt_max, tol_time;
  double err_last;          // relative local error estimate of the last step
  double theta_run;         // θ of the solve (theta is the level's: an adaptive
                            // Crank-Nicolson solve starts with PD_RANNACHER
                            // backward-Euler steps)
  int stall, pad6;          // consecutive steps forced through at dt_min with e > 2 tol_time
  // the level-begin passes reuse L n^{k-a} and S0(n^{k-a}) of the earlier
  // levels (PdInst::lsol): S0 per solution slot, set by each level's Gram
  // totals; the diagonal of L is stored once per solve call
  double s0h[PD_NSOL];
  int ld_ready, pad7;
};

template <typename T>
struct KSet {
  T *r, *rh, *p, *v, *ph, *s, *sh, *t, *w;
  T *d;                              // inner iterate (mixed precision only)
  const T *gp_r, *gm_r, *gp_t, *gm_t;  // faces
  const T *inv_d;                    // 1/diag(A): the Krylov iteration runs on D^{-1}A
};

// One level of the θ-semi-coarsening multigrid preconditioner (device
// descriptor).  Level 0 is the instance's own system; level l+1 merges the
// θ-lines of level l in pairs (J <- 2J, 2J+1; the last coarse line takes
// three when n_l is odd).  A level's operator is I/dt + θ L_l in the face
// form of PdInst, with its own faces and angular cell widths: radial faces
// of merged lines add up, the angular face between them drops out, the
// volumes add (the Galerkin product of the volume-weighted system).  The
// level below the last holds the ring means and is solved directly.
struct PdMgLevel {
  int m, n, npad;                     // rings, θ-lines, padded length (origin at m*n)
  int has_b;
  const double *gp_r, *gm_r, *gp_t, *gm_t;   // faces (PdInst layout)
  const double *inv_rw;               // [m+2] the instance's (shared by every level)
  const double *inv_dth;              // [n] 1/(angular cell width)
  const double *b_node;               // [npad] volume-weighted reaction, or null
  const double *diag, *inv_diag;      // [npad] diagonal of I/dt + θL_l (its factorisation)
  double inv_V0;                      // 1/(origin volume), the same on every level
  double *g;                          // right-hand side per volume (levels >= 1)
  double *x;                          // iterate after the coarse correction (levels >= 1)
  double *r, *w, *sh;                 // sweep input, radial intermediate, output
};

struct PdInst {
  int m, n, npad, nsrc;
  int K, mixed, has_b, zero_flux;
  int rb, pad_rb;                    // rings per stencil wave (set by the launch plan)
  int ncg, nrg, nb_sten, nb_elem;    // stencil tiling and block counts
  int cw, nseg, brad, nb_rad;        // radial sweep: columns per block, segments, rows/segment
  int bang, nb_ang, nb_frad, nb_fang;
  int aw, pad_aw;                    // waves per ring of the ring sweep (1, 2 or 4)
  double inv_V0;
  double l0;                // diagonal of L at the origin: inv_V0 Σ_j gp_r(1/2, j) + b_0 (fixed order)
  const double *inv_rw;     // [m+2] 1/(r_i (h_i+h_{i+1})/2), index i
  const double *inv_dth;    // [n]   1/Δθ_j
  const double *r_nodes;    // [m+2] r_0..r_{m+1}
  const double *th_nodes;   // [n+1] θ_0..θ_n
  const double *b_node;     // [npad] or null
  const double *g;          // [nsrc*npad]
  const double *nb;         // [nsrc*n]
  const double *lam;        // [nsrc]
  const int *tpow;          // [nsrc]
  double *t_table;          // [K+1] (adaptive stepping writes its levels as it goes)
  double *sol[PD_NSOL];     // rotating (sol_slot): n^{k-3} .. n^k, iterate
  double *lsol[PD_NSOL];    // L of the slot's state, written by the Gram pass of the level
                            // where it is n^k (L: the operator without 1/dt, θ)
  double *ldiag;            // [npad] diagonal of L (faces only; l_diag)
  double *bvec;             // right-hand side (FP64)
  double *rout;             // FP64 outer residual (mixed)
  double *diag;             // [npad] diagonal of I/dt + θL at the last factorisation
  double *inv_diag;         // [npad] its reciprocal (k64.inv_d; the FP64 kernels form 1/diag themselves)
  float *inv_diag32;        // [npad] FP32 1/diag of the level under way (k32.inv_d, mixed precision)
  // Factors of the two sweeps of the preconditioner, computed in FP64 and
  // stored in FP32 in both precisions (the sweeps themselves run in FP64 in
  // the FP64 solve: the rounded factors define a fixed, slightly different
  // preconditioner, which moves the iterates but not the converged solution).
  float *rf_uinv, *rf_f, *rf_g;           // [m*n] radial pivots 1/u and multipliers
  float *af_uinv, *af_f, *af_g, *af_z;    // [m*64*bang] angular (sweep order), SM vector
  double *af_kappa, *af_alpha0;   // [m] Sherman-Morrison scalars per ring
  // The origin row and ring 1's couplings to the origin belong to the
  // angular factor (ring 1 and the origin form an arrow system): with
  // T1 = ring 1's block of (I + D^{-1}Θ), ã_j = ring 1's scaled coupling to
  // the origin, c̃_j = the origin row's scaled coupling to ring 1,
  // q = T1^{-1} ã and σ = 1 - c̃·q, the sweep takes u = T1^{-1} w_1,
  // z_0 = (w_0 - c̃·u)/σ, z_1 = u - q z_0.
  float *af_q, *af_c;       // [64*bang] q and c̃, sweep order
  double *af_sigma;         // [1] σ (1, with q = c̃ = 0, when the arrow is not used)
  KSet<double> k64;
  KSet<float> k32;
  // per-block partial sums, one region per producer
  double *part_b, *part_v, *part_t, *part_ur, *part_a;   // [slots * nb_sten]
  double *part_x;                                        // [2 * nb_elem]
  double *part_g;                                        // [PD_NGRAM * nb_sten]
  double *gram_tot;                                      // [PD_NGRAM] totals of part_g
  PdScalars *sc;
  int *n_active;            // shared counter of the batch (device)
  int *lvl_out;             // (levels done, status) written at each level end
  double *level_stats;      // [K * PD_LSTAT]: iters, outer, status, rel_resid, dt, t1, restarts,
                            // error estimate, rejected attempts, 0
  double *fdot[3];          // adaptive stepping: f(t_k, x_k) by level modulo 3 (FP64)
  double *part_e;           // [3 * nb_sten]: the level-end pass's ||d||², ||x||², S0
  // Ring-mean correction at the end of every level: the Galerkin projection
  // of the system onto ring-constant vectors (one unknown per ring plus the
  // origin) is a tridiagonal system of m+1 unknowns whose coefficients are
  // ring sums of the faces and volumes, fixed per instance:
  //   crs[k*(m+1) + i], k = 0..5: Σ_j V_ij, Σ_j V_ij b_ij, Σ_j gp_r(i+1/2, j),
  //   Σ_j gm_r(i-1/2, j), Σ_j gm_r(i+1/2, j), Σ_j gp_r(i-1/2, j)
  // (ring 0 is the origin, with V_0 and b_0; terms outside the mesh are 0).
  const double *crs;
  double *cr_c;             // [m+1] the correction of the level that just ended
  double *part_c;           // [m * ncg] per ring and column group: Σ_j V_ij (b - A x)_ij
  double *cr_f;             // [m+1] the ring totals of part_c (index i = ring, 0 unused)
  double *part_c0;          // [nb_sten] S0 partials of the same pass
};
