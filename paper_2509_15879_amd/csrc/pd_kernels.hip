// HIP kernels (gfx950 / CDNA4) of the polar-disk θ-scheme solver.
//
// Every kernel is batched: a block map turns blockIdx.x into (instance,
// local block), so one launch advances every instance of a batch, whatever
// its mesh size or PDE type.  Reductions never synchronise blocks inside a
// launch: a reducing kernel leaves one partial sum per block and slot, and
// the next kernel that needs the total (always a later launch on the same
// stream, so no fence is needed) sums the partials in a fixed order in every
// block.  Block 0 of that kernel records the instance's Krylov scalars and
// status, writing only fields that kernel does not read.  The order of every
// sum depends only on the instance's own tiling, so a result does not depend
// on which other instances share the launch.
//
// One time level (scheme (2.5) of §2.1, Ch. 3 scheme of §3.2.1, system
// (2.11)/(2.12)) is
//   k_level_begin   per-instance set-up: Δt, θ, source weights, extrapolation
//   k_fact_rad      radial-line LU of (I + D^{-1}R) per θ-column (when Δt/θ change)
//   k_fact_ang      ring-periodic LU of (I + D^{-1}Θ) per ring, Sherman-Morrison
//   k_sten<GRAM>    the least-squares problem of the initial guess (partial sums)
//   k_gram_total    their totals, one block per instance and sum
//   k_sten<BEGIN>   rhs, initial guess (extrapolation, corrected by least squares) and its residual
//   BiCGSTAB cycles k_rad -> k_ang -> k_sten<V> -> k_rad -> k_ang -> k_sten<T> -> k_elem_x
//   (mixed precision: k_sten<UR> refines in FP64 between FP32 inner solves)
//   k_level_end
// The Krylov iteration runs on the diagonally scaled system D^{-1}A x = D^{-1}b
// (D the diagonal of A = I/Δt + θ L_h), whose residual weighs every row
// alike: the unscaled residual is dominated by the few rows next to r = 1
// (and next to the origin) whose coefficients grow like 1/h² on graded
// meshes.  The preconditioner of the scaled system is the alternating-line
// product
//   M = (I + D^{-1}R)(I + D^{-1}Θ),  M^{-1} y = (I + D^{-1}Θ)^{-1} (I + D^{-1}R)^{-1} y,
// with R the radial (same-column) couplings and Θ the angular (same-ring,
// periodic) couplings of A.  Θ also holds the origin row and ring 1's
// couplings to the origin, so that ring 1 and the origin are solved as one
// arrow system (the radial sweep passes the origin through).  The radial
// blocks are the tridiagonal A_j of (2.12).
//
// Both tridiagonal families are solved by segmented scans: a thread owns a
// contiguous segment of a line, substitutes locally in registers, and the
// segments are joined by composing their affine maps w -> P w + e (forward
// and backward substitution) or their 2x2 continuant matrices (the pivot
// recurrence of the factorisation).  Radial lines join through LDS across
// the waves of a block; rings join across the lanes of one wave.
//
// Arithmetic is FP64, except that the inner solve of the mixed-precision
// mode keeps its vectors and faces in FP32 and its sweeps compute in FP32,
// and that the preconditioner's factors (pivots, multipliers, the
// Sherman-Morrison vector) are computed in FP64 but stored in FP32 in both
// precisions.  Pointers taken from the instance descriptor are handed to the
// bodies as restrict-qualified global-address-space pointers, so that loads
// of different arrays can be in flight together.

#include "pd_device.h"

#include <hip/hip_ext.h>

#include <math.h>

#define GAS __attribute__((address_space(1)))

namespace pd {

// ------------------------------------------------------------------ helpers

template <class T>
__device__ __forceinline__ GAS T *G(T *p) {
  return (GAS T *)p;
}
template <class T>
__device__ __forceinline__ const GAS T *G(const T *p) {
  return (const GAS T *)p;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double tau_q(double lam, int tp, double t) {
  double v = exp(lam * t);
  for (int k = 0; k < tp; ++k) v *= t;
  return v;
}

// Per-block partial sums of a reducing kernel: one value per slot and block,
// written by thread 0 with plain stores (the consumer is a later launch).
template <int NS>
__device__ __forceinline__ void produce(double (&v)[NS], double *part, int nblk, int blk) {
  __shared__ double red[NS][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double x = wave_sum(v[k]);
    if (lane == 0) red[k][wave] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      double sum = 0.0;
      for (int w = 0; w < nw; ++w) sum += red[k][w];
      part[k * nblk + blk] = sum;
    }
  }
}

// Total of a producer's partials: wave 0 sums them in a fixed order (lane
// strided, then a butterfly) and the block shares the result.  Every thread
// of the block must call it.  All slots advance together and the strided
// loop is unrolled, so that many loads are in flight at once (a large
// instance leaves thousands of partials per slot); each slot is still summed
// in ascending block order.
template <int NS>
__device__ __forceinline__ void consume(const double *part, int nblk, double (&tot)[NS]) {
  __shared__ double sh[NS];
  if (threadIdx.x < 64) {
    double sum[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) sum[k] = 0.0;
#pragma unroll 4
    for (int b = threadIdx.x; b < nblk; b += 64) {
#pragma unroll
      for (int k = 0; k < NS; ++k) sum[k] += part[k * nblk + b];
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const double v = wave_sum(sum[k]);
      if (threadIdx.x == 0) sh[k] = v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NS; ++k) tot[k] = sh[k];
}

// One snapshot of an instance's status per block: block 0 of a kernel may
// change the status while other blocks of the same launch start, and all
// threads of a block must take the same path through its barriers.
__device__ __forceinline__ int block_status(const PdScalars *sc) {
  __shared__ int st;
  if (threadIdx.x == 0) st = sc->status;
  __syncthreads();
  return st;
}

// A level of the instance has just met its tolerance and is not yet
// recorded: the round head closes it (ring-mean correction, then control).
__device__ __forceinline__ bool level_converged(const PdScalars *sc) {
  return sc->in_level && sc->status == ST_DONE;
}

__device__ __forceinline__ void finish_instance(const PdInst &, PdScalars *sc, int status) {
  sc->status = status;   // the level ends; the control kernel takes it from here
}

__device__ __forceinline__ bool inner_active(const PdScalars *sc) {
  return sc->status == ST_ACTIVE && sc->phase == PH_INNER;
}

// An inner kernel instantiated for storage type T only serves instances of
// the matching precision (FP32 storage <=> mixed precision).
template <typename T>
__device__ __forceinline__ bool prec_match(const PdInst &I) {
  return (sizeof(T) == 4) == (I.mixed != 0);
}

template <typename T>
__device__ __forceinline__ T *iterate_ptr(const PdInst &I, const PdScalars *sc);
template <>
__device__ __forceinline__ double *iterate_ptr<double>(const PdInst &I, const PdScalars *sc) {
  return I.sol[sol_slot(sc->rot, -1)];
}
template <>
__device__ __forceinline__ float *iterate_ptr<float>(const PdInst &I, const PdScalars *sc) {
  return I.k32.d;
}

template <typename T>
__device__ __forceinline__ const KSet<T> &kset(const PdInst &I);
template <>
__device__ __forceinline__ const KSet<double> &kset<double>(const PdInst &I) { return I.k64; }
template <>
__device__ __forceinline__ const KSet<float> &kset<float>(const PdInst &I) { return I.k32; }

// Composition of affine maps u -> P u + e:  (P2, e2) ∘ (P1, e1).
template <typename C>
struct AffT {
  C P, e;
};
using Aff = AffT<double>;
template <typename C>
__device__ __forceinline__ AffT<C> compose(AffT<C> later, AffT<C> earlier) {
  return {later.P * earlier.P, later.P * earlier.e + later.e};
}

// ------------------------------------------------------------ level control

// Weights of the initial guesses of level k -> k+1 (t = t_{k+1}) from the
// levels t_{k-a}, a = 0..ne, of this solve (ne = 0..3).
//  candidate 0: the Lagrange polynomial through all of them (cubic at ne = 3);
//  candidate 1: at ne = 3, a quadratic plus a component multiplied by
//    ρ = -(1-θ)/θ per level, the amplification of the θ-scheme on its
//    stiffest modes (ρ = -1 for Crank-Nicolson, whose stiff error components
//    alternate in sign instead of decaying); the quadratic through the last
//    three levels when ρ is near 0 (θ near 1); below ne = 3, candidate 0.
// Only where the iteration starts depends on them, not the solution.
__device__ void guess_weights(const double *tt, int k, int ne, double theta, double (&w)[2][PD_NHIST]) {
  const double t = tt[k + 1], h = t - tt[k];
  double s[PD_NHIST];   // (t_{k-a} - t)/Δt
#pragma unroll
  for (int a = 0; a < PD_NHIST; ++a) s[a] = a <= ne ? (tt[k - a] - t) / h : 0.0;
  // Lagrange weights through the ne + 1 known levels, at s = 0
#pragma unroll
  for (int a = 0; a < PD_NHIST; ++a) {
    double l = a <= ne ? 1.0 : 0.0;
#pragma unroll
    for (int c = 0; c < PD_NHIST; ++c)
      if (c != a && c <= ne && a <= ne) l *= (0.0 - s[c]) / (s[a] - s[c]);
    w[0][a] = w[1][a] = l;
  }
  if (ne < PD_NHIST - 1) return;
  const double rho = -(1.0 - theta) / theta;
  if (rho > -0.05) {
    // the quadratic through the last three levels
#pragma unroll
    for (int a = 0; a < PD_NHIST; ++a) {
      double l = a < 3 ? 1.0 : 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (c != a && a < 3) l *= (0.0 - s[c]) / (s[a] - s[c]);
      w[1][a] = l;
    }
    return;
  }
  // The cubic's weights reproduce quadratics; so do they plus any multiple
  // of v_a = 1/Π_{c≠a}(s_a - s_c), which annihilates quadratics.  The
  // multiple is fixed by Σ_a w_a ρ^{-a} = ρ (exactness on the stiff mode).
  double v[PD_NHIST], sw = 0.0, sv = 0.0, pa = 1.0;
#pragma unroll
  for (int a = 0; a < PD_NHIST; ++a) {
    double q = 1.0;
#pragma unroll
    for (int c = 0; c < PD_NHIST; ++c)
      if (c != a) q *= s[a] - s[c];
    v[a] = 1.0 / q;
    sw += w[0][a] * pa;
    sv += v[a] * pa;
    pa /= rho;
  }
  const double g = (rho - sw) / sv;
#pragma unroll
  for (int a = 0; a < PD_NHIST; ++a) w[1][a] = w[0][a] + g * v[a];
}

// Sets up level sc->level of an instance, t_k -> t_{k+1}: Δt, θ, the
// source weights, the weights of both polynomial candidate guesses (the
// level-begin passes choose between them and correct the choice); its
// factorisation (when θ changed or Δt moved enough) and right-hand side
// are then due.
__device__ __forceinline__ void begin_level(const PdInst &I, PdScalars *sc) {
  const int k = sc->level;
  const double t0 = I.t_table[k], t1 = I.t_table[k + 1];
  // an adaptive Crank-Nicolson solve takes its first steps with backward
  // Euler, which damps the stiff components of the initial state that
  // Crank-Nicolson would carry undamped (and the step control would chase)
  const double th = (sc->adaptive && sc->theta_run == 0.5 && k < PD_RANNACHER) ? 1.0 : sc->theta_run;
  sc->theta = th;
  const double dt = t1 - t0;
  sc->t0 = t0;
  sc->t1 = t1;
  sc->dt = dt;
  sc->inv_dt = 1.0 / dt;
  // the preconditioner is refactored when θ changed or Δt moved by more than
  // PD_REFACTOR_DT (relative) since its factorisation: it only has to stay
  // close to the system, not equal it (the operator, the diagonal scaling
  // and the right-hand side always follow the current Δt)
  sc->refactor = (th != sc->fact_theta || !(fabs(dt - sc->fact_dt) <= PD_REFACTOR_DT * sc->fact_dt)) ? 1 : 0;
  if (sc->refactor) {
    sc->fact_dt = dt;
    sc->fact_theta = th;
  }
  const int ne = min(sc->have_prev, PD_NHIST - 1);
  double w[2][PD_NHIST];
  guess_weights(I.t_table, k, ne, th, w);
  for (int c = 0; c < 2; ++c)
    for (int a = 0; a < PD_NHIST; ++a) sc->ex_w[c][a] = w[c][a];
  sc->ex_n = ne;
  sc->guess_kind = 0;
  for (int s = 0; s < PD_MAXSRC; ++s) sc->cq[s] = 0.0;
  for (int s = 0; s < I.nsrc; ++s)
    sc->cq[s] = (1.0 - th) * tau_q(I.lam[s], I.tpow[s], t0) + th * tau_q(I.lam[s], I.tpow[s], t1);
  sc->status = ST_ACTIVE;
  sc->stage = STAGE_START;
  sc->in_level = 1;
  sc->phase = PH_INNER;
  sc->pend = PEND_BEGIN;
  sc->restarted = 0;
  sc->iters = 0;
  sc->outer = 0;
  sc->inner_iters = 0;
  sc->restarts = 0;
  sc->first = 1;
  sc->reset_rh = 0;
  sc->inner_first = 1;
  sc->alpha = sc->omega = 1.0;
  sc->rho_next = sc->rho_cur = 1.0;
}

// Records the level that just ended and rotates the solution buffers
// (iterate -> n^{k+1}); returns whether it met its tolerance.
__device__ __forceinline__ bool end_level(const PdInst &I, PdScalars *sc) {
  const int k = sc->level;
  double *st = I.level_stats + PD_LSTAT * k;
  st[0] = sc->iters;
  st[1] = sc->outer;
  st[2] = sc->status;
  st[3] = sc->rel_resid;
  st[4] = sc->dt;
  st[5] = sc->t1;
  st[6] = sc->restarts;
  st[7] = sc->adaptive ? sc->err_last : 0.0;
  st[8] = sc->nrej;
  st[9] = 0.0;
  sc->total_iters += sc->iters;
  const bool ok = sc->status == ST_DONE;
  if (!ok) sc->nfail += 1;
  sc->rot = (sc->rot + 1) % PD_NSOL;   // the iterate's slot becomes n^k
  sc->have_prev = min(sc->have_prev + 1, PD_NHIST - 1);
  sc->t_now = sc->t1;
  sc->level = k + 1;
  sc->nrej = 0;
  sc->in_level = 0;
  if (I.lvl_out) I.lvl_out[0] = k + 1;
  return ok;
}

// One level's set-up alone (right-hand side assembly without a solve).
__global__ void k_level_begin(PdInst *insts, int ninst) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ninst) return;
  PdInst &I = insts[q];
  PdScalars *sc = I.sc;
  if (sc->status == ST_IDLE) return;
  begin_level(I, sc);
}

// ------------------------------------------------------------ adaptive steps
//
// A-posteriori control of Δt (the paper fixes its levels in advance; this is
// the library's adaptive mode).  With f(t, x) = -L x + S(t) + c N(t) the
// θ-scheme is (x_{k+1} - x_k)/Δt = (1-θ) f_k + θ f_{k+1}.  Local error
// estimate of the step t_k -> t_{k+1}, from Taylor expansion:
//   θ ≠ 1/2: d = (θ - 1/2) Δt (f_{k+1} - f_k)                      (order q = 1)
//   θ = 1/2: d = (x_{k+1} - x^P) / (3 (1 + Δt_prev/Δt)),            (order q = 2)
//            x^P = x_k + Δt ((1 + r/2) f_k - (r/2) f_{k-1}), r = Δt/Δt_prev
//            (trapezoidal rule against the variable-step Adams-Bashforth 2)
// e = ||d||/||x_{k+1}||.  The first step is accepted with Δt_0 and the second
// tried with Δt_0; later a step with e > 2 tol (and Δt > dt_min) is retaken
// with Δt max(1/4, 0.9 (tol/e)^{1/(q+1)}), and an accepted one sets the
// next Δt to Δt clamp(0.9 (tol/e)^{1/(q+1)}, 1/2, 2) within [dt_min, dt_max];
// a step that would pass T ends on it, one that would leave less than a
// step ends half-way.  f and the ring part of the norms come from a stencil
// pass at the end of every level; k_ctl closes the origin and decides.

__device__ __forceinline__ double est_d(double x1, double x0, double f1, double f0, double fm1,
                                        double dt, double dtp, double th) {
  if (th != 0.5) return (th - 0.5) * dt * (f1 - f0);
  const double r = dt / dtp;
  const double xp = x0 + dt * ((1.0 + 0.5 * r) * f0 - 0.5 * r * fm1);
  return (x1 - xp) / (3.0 * (1.0 + dtp / dt));
}

__device__ __forceinline__ double land_step(double t, double dt, double t_end) {
  const double rem = t_end - t;
  if (dt >= rem) return rem;
  if (dt > 0.5 * rem) return 0.5 * rem;
  return dt;
}

// The time level reached by a step dt from t (exactly t_end when it lands).
__device__ __forceinline__ double next_level(double t, double dt, double t_end) {
  return dt >= t_end - t ? t_end : t + dt;
}

// f at the origin: -(L x)_0 + S_0(t), from the ring-1 face sum S0.
__device__ __forceinline__ double origin_f(const PdInst &I, double x0, double S0, double t) {
  const int orig = I.m * I.n;
  const double bo = I.has_b ? I.b_node[orig] : 0.0;
  double f = -(I.inv_V0 * S0 + bo * x0);
  for (int q = 0; q < I.nsrc; ++q) f += tau_q(I.lam[q], I.tpow[q], t) * I.g[q * I.npad + orig];
  return f;
}

// Control of asynchronous levels (one thread per instance), first in every
// cycle: an instance whose level has ended (converged, or stopped) records
// it and starts its next level at once, whatever the others are doing; one
// that has taken all its levels, or failed one, leaves the batch and is
// counted out of the active-instance counter.
__global__ void k_ctl(PdInst *insts, int ninst) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ninst) return;
  PdInst &I = insts[q];
  PdScalars *sc = I.sc;
  const int orig = I.m * I.n;
  // each slot in ascending block order; the slots advance together and the
  // loop is unrolled, so that many loads are in flight
  auto level_end_sums = [&](double (&tot)[3]) {
    double sum[3] = {0.0, 0.0, 0.0};
#pragma unroll 8
    for (int b = 0; b < I.nb_sten; ++b) {
#pragma unroll
      for (int c = 0; c < 3; ++c) sum[c] += I.part_e[c * I.nb_sten + b];
    }
    for (int c = 0; c < 3; ++c) tot[c] = sum[c];
  };
  if (sc->adaptive && sc->need_f0) {
    // f(t_0, x_0): the ring part was formed by the level-end pass
    double tot[3];
    level_end_sums(tot);
    const double x0 = I.sol[sol_slot(sc->rot, 0)][orig];
    I.fdot[sc->level % 3][orig] = origin_f(I, x0, tot[2], sc->t_now);
    sc->need_f0 = 0;
  }
  const int st = sc->status;
  if (st == ST_IDLE || st == ST_ACTIVE) return;
  bool ok = true;
  double e = 0.0;
  const int qord = sc->theta == 0.5 ? 2 : 1;
  if (sc->in_level && sc->adaptive && st == ST_DONE) {
    // the step just taken: f at its end, its error estimate, accept or retake
    double tot[3];
    level_end_sums(tot);
    const int k = sc->level;
    const double x1 = I.sol[sol_slot(sc->rot, -1)][orig];
    const double f1 = origin_f(I, x1, tot[2], sc->t1);
    I.fdot[(k + 1) % 3][orig] = f1;
    if (k >= 1) {
      const double dtp = I.t_table[k] - I.t_table[k - 1];
      const double d0 = est_d(x1, I.sol[sol_slot(sc->rot, 0)][orig], f1, I.fdot[k % 3][orig],
                              I.fdot[(k + 2) % 3][orig], sc->dt, dtp, sc->theta);
      const double xx = tot[1] + x1 * x1;
      e = sqrt(tot[0] + d0 * d0) / fmax(sqrt(xx), 1e-300);
    }
    sc->err_last = e;
    // "longer than dt_min" compares levels: the step's level against the one a
    // dt_min step reaches (t1 - t0 itself may round above dt_min, which would
    // reject a step at dt_min again and again)
    if (k >= 1 && e > 2.0 * sc->tol_time && sc->t1 > next_level(sc->t0, sc->dt_min, sc->t_end)) {
      const double fr = fmax(0.25, 0.9 * pow(sc->tol_time / e, 1.0 / (qord + 1)));
      const double dtr = land_step(sc->t0, fmax(sc->dt_min, sc->dt * fr), sc->t_end);
      I.t_table[k + 1] = next_level(sc->t0, dtr, sc->t_end);
      sc->nrej += 1;
      begin_level(I, sc);                 // the same level again from n^k
      return;
    }
    // a step forced through at dt_min although its error is above 2 tol_time
    sc->stall = (k >= 1 && e > 2.0 * sc->tol_time) ? sc->stall + 1 : 0;
  }
  if (sc->in_level) ok = end_level(I, sc);
  // PD_STALL such steps in a row: tol_time is out of reach at dt_min, the
  // solve stops (PD_ENOCONV: T not reached)
  if (ok && sc->adaptive && sc->stall >= PD_STALL) ok = false;
  if (ok && sc->adaptive) {
    // the next level's time: grown or shrunk after the second step
    const int k1 = sc->level;
    const double t = sc->t_now;
    if (t >= sc->t_end) {
      sc->K = k1;                         // reached T: no more levels
    } else if (k1 >= 1) {
      double nxt = sc->dt;
      if (k1 >= 2) {
        const double g = e > 0.0 ? fmin(2.0, fmax(0.5, 0.9 * pow(sc->tol_time / e, 1.0 / (qord + 1)))) : 2.0;
        nxt = sc->dt * g;
      }
      nxt = fmin(fmax(nxt, sc->dt_min), sc->dt_max);
      if (k1 < sc->K) I.t_table[k1 + 1] = next_level(t, land_step(t, nxt, sc->t_end), sc->t_end);
      else ok = false;                    // the level cap came before T
    }
  }
  if (ok && sc->level < sc->K) {
    begin_level(I, sc);
  } else {
    sc->status = ST_IDLE;
    atomicSub(I.n_active, 1);
    if (I.lvl_out) I.lvl_out[1] = 1;
  }
}

// ------------------------------------------------------------ factorisations
//
// Radial lines of (I + D^{-1}R), column j, rows i = 1..m: diagonal 1,
// sub-diagonal a_i = -θ gp_r(i-1/2)/(V_i d_i) (i >= 2), super-diagonal
// c_i = -θ gm_r(i+1/2)/(V_i d_i) (i < m).  Pivots u_1 = 1,
// u_i = 1 - a_i c_{i-1}/u_{i-1}.  Stored: uinv_i = 1/u_i, f_i = a_i/u_i,
// g_i = c_i/u_i, so that forward  w_i = uinv_i y_i - f_i w_{i-1}  and
// backward  x_i = w_i - g_i x_{i+1}.  Also stores d and 1/d.
//
// The pivot recurrence is the ratio u_i = q_i/q_{i-1} of the continuants
// q_i = q_{i-1} - a_i c_{i-1} q_{i-2}, a linear recurrence: each segment
// multiplies its 2x2 matrices [[1, -a_i c_{i-1}], [1, 0]] (rescaled to stay
// in range), the segments' products are chained through LDS to give every
// segment its incoming u, and each segment then runs the pivot recurrence
// on its own rows.

struct RadRow {
  double d, a, c;   // diagonal of A, scaled sub and super entries
};

// Diagonal of L at a ring node from the coefficients of its four faces
// that multiply it (outer radial gp, inner radial gm, upper angular gp,
// lower angular gm), and the diagonal of A = I/dt + θL.  Written with
// explicit fused multiply-adds, so that the factorisation (which stores
// 1/diag) and the stencils (which form it again from the faces they hold)
// get the same bits.
__device__ __forceinline__ double l_diag(double ivV, double gpo, double gmi, double gpt, double gmtl,
                                         double bP) {
  return __builtin_fma(ivV, ((gpo + gmi) + gpt) + gmtl, bP);
}
__device__ __forceinline__ double diag_of(double inv_dt, double th, double ld) {
  return __builtin_fma(th, ld, inv_dt);
}
// 1/diag of the origin row for the level under way.
__device__ __forceinline__ double origin_invd(const PdInst &I, double inv_dt, double th) {
  return 1.0 / diag_of(inv_dt, th, I.l0);
}

struct Mat2 {
  double a, b, c, d;   // [[a, b], [c, d]]
};
__device__ __forceinline__ Mat2 mul2(Mat2 x, Mat2 y) {
  return {x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d, x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}
// Rescales by a power of two (exact) to keep the products in range.
__device__ __forceinline__ Mat2 norm2(Mat2 x) {
  const double s = fmax(fmax(fabs(x.a), fabs(x.b)), fmax(fabs(x.c), fabs(x.d)));
  if (!(s > 0.0) || !(s < INFINITY)) return x;
  const int e = -ilogb(s);
  return {ldexp(x.a, e), ldexp(x.b, e), ldexp(x.c, e), ldexp(x.d, e)};
}

// Row i of the radial system from its loaded face values: diagonal of A and
// the scaled sub/super entries (ring 1 has no sub entry, ring m no super).
__device__ __forceinline__ RadRow rad_row_of(int i, int m, double gpo, double gmo, double gpi,
                                             double gmi, double gpt, double gmtl, double ivV,
                                             double bP, double inv_dt, double th) {
  RadRow R;
  R.d = diag_of(inv_dt, th, l_diag(ivV, gpo, gmi, gpt, gmtl, bP));
  const double s = th * ivV / R.d;
  R.a = (i >= 2) ? -s * gpi : 0.0;
  R.c = (i < m) ? -s * gmo : 0.0;
  return R;
}

// A block: 16 columns x 64 segments of B <= BM rows.  Every thread loads the
// faces of its rows (up to 4 rows at once; longer segments load and form
// their rows again for the pivots) and of the row before its segment, forms
// its segment's continuant product, and the products are chained by a
// shuffle scan over the 4 segments of a wave and a fold over the earlier
// waves' totals (LDS).  Block 0 of an instance also sums the origin's faces.
template <int BM>
__global__ __launch_bounds__(PD_RAD_THREADS) void k_fact_rad(const PdInst *insts, const int2 *map) {
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  const PdScalars *sc = I.sc;
  if (sc->status != ST_ACTIVE || sc->stage != STAGE_START || !sc->refactor) return;
  constexpr int NW = PD_RAD_THREADS / 64;
  const int m = I.m, n = I.n, cw = I.cw, B = I.brad;
  const int c = threadIdx.x % cw, seg = threadIdx.x / cw;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, sub = lane >> 4;
  const int j = mp.y * cw + c;
  const bool act = j < n;
  const int jj = act ? j : 0, jl = (jj == 0) ? n - 1 : jj - 1;
  const int k0 = seg * B;                          // first 0-based row of the segment
  const int cnt = act ? max(0, min(B, m - k0)) : 0;
  const double th = sc->theta, inv_dt = sc->inv_dt;
  const GAS double *gpr = G(I.k64.gp_r), *gmr = G(I.k64.gm_r);
  const GAS double *gpt = G(I.k64.gp_t), *gmt = G(I.k64.gm_t);
  const GAS double *irw = G(I.inv_rw), *bnode = I.has_b ? G(I.b_node) : nullptr;
  const double idth = G(I.inv_dth)[jj];

  // the row of ring i (clamped to [1, m]); loads of CH rows are issued together
  auto load_row = [&](int i) -> RadRow {
    i = min(max(i, 1), m);
    return rad_row_of(i, m, gpr[i * n + jj], gmr[i * n + jj], gpr[(i - 1) * n + jj],
                      gmr[(i - 1) * n + jj], gpt[(i - 1) * n + jj], gmt[(i - 1) * n + jl],
                      irw[i] * idth, bnode ? bnode[(i - 1) * n + jj] : 0.0, inv_dt, th);
  };
  constexpr int CH = BM < 4 ? BM : 4;     // rows per chunk
  constexpr int NCH = BM / CH;            // chunks; with one, rows stay in registers
  double c_prev = 0.0;
  {
    const RadRow R0 = load_row(k0);       // the row before the segment
    if (cnt > 0 && k0 >= 1) c_prev = R0.c;
  }
  // segment product of continuant matrices (later rows on the left)
  Mat2 Mp{1.0, 0.0, 0.0, 1.0};
  double cp = c_prev;
  RadRow rw[CH];
#pragma unroll 1
  for (int h = 0; h < NCH; ++h) {
#pragma unroll
    for (int q = 0; q < CH; ++q) rw[q] = load_row(k0 + min(h * CH + q, max(cnt - 1, 0)) + 1);
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      if (h * CH + q < cnt) {
        const Mat2 Mi{1.0, -rw[q].a * cp, 1.0, 0.0};
        Mp = norm2(mul2(Mi, Mp));
        cp = rw[q].c;
      }
    }
  }
  // inclusive scan over the wave's 4 segments, then the earlier waves' totals
  Mat2 S = Mp;
#pragma unroll
  for (int d = 1; d < 4; d <<= 1) {
    const Mat2 o{__shfl_up(S.a, 16 * d, 64), __shfl_up(S.b, 16 * d, 64), __shfl_up(S.c, 16 * d, 64),
                 __shfl_up(S.d, 16 * d, 64)};
    if (sub >= d) S = norm2(mul2(S, o));
  }
  Mat2 ex{__shfl_up(S.a, 16, 64), __shfl_up(S.b, 16, 64), __shfl_up(S.c, 16, 64), __shfl_up(S.d, 16, 64)};
  if (sub == 0) ex = Mat2{1.0, 0.0, 0.0, 1.0};
  __shared__ double tw[NW][4][16];
  if (sub == 3) {
    tw[wave][0][c] = S.a;
    tw[wave][1][c] = S.b;
    tw[wave][2][c] = S.c;
    tw[wave][3][c] = S.d;
  }
  __syncthreads();
  Mat2 Pw{1.0, 0.0, 0.0, 1.0};
  for (int w = 0; w < wave; ++w) Pw = norm2(mul2(Mat2{tw[w][0][c], tw[w][1][c], tw[w][2][c], tw[w][3][c]}, Pw));
  const Mat2 E = mul2(ex, Pw);
  // incoming (q_{k0}, q_{k0-1}) = E (1, 0); then the pivots of the own rows
  const double q1 = E.a, q0 = E.c;
  double u_prev = (q0 != 0.0) ? q1 / q0 : 1.0;
  cp = c_prev;
  GAS double *dg = G(I.diag), *idg = G(I.inv_diag);
  GAS float *uinv = G(I.rf_uinv), *ff = G(I.rf_f), *gg = G(I.rf_g);
#pragma unroll 1
  for (int h = 0; h < NCH; ++h) {
    if (NCH > 1) {
#pragma unroll
      for (int q = 0; q < CH; ++q) rw[q] = load_row(k0 + min(h * CH + q, max(cnt - 1, 0)) + 1);
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int k = h * CH + q;
      if (k < cnt) {
        const int idx = (k0 + k) * n + jj;
        const double u = 1.0 - rw[q].a * cp / u_prev;
        const double ui = 1.0 / u;
        const double id = 1.0 / rw[q].d;
        dg[idx] = rw[q].d;
        idg[idx] = id;
        uinv[idx] = (float)ui;
        ff[idx] = (float)(rw[q].a * ui);
        gg[idx] = (float)(rw[q].c * ui);
        u_prev = u;
        cp = rw[q].c;
      }
    }
  }
  if (mp.y == 0 && threadIdx.x == 0) {
    const double d0 = diag_of(inv_dt, th, I.l0);
    dg[m * n] = d0;
    idg[m * n] = 1.0 / d0;
  }
}

// Where the ring sweeps keep the factor of node j of a ring (ring offset
// frow, lane span bang): with one wave per ring (aw = 1), lane L owns nodes
// [L*bang, (L+1)*bang) and node L*bang + k sits at 64k + L; with aw waves
// per ring each of the 64*aw threads owns 8 nodes, node 8t + k at k*64*aw + t.
// Either way the threads of a sweep read their factors with coalesced loads.
__device__ __forceinline__ int afac_index(int frow, int j, int bang, int aw) {
  return aw == 1 ? frow + 64 * (j % bang) + j / bang : frow + (j & 7) * 64 * aw + (j >> 3);
}

// Ring-periodic LU of (I + D^{-1}Θ) for ring i: row j has diagonal 1,
// sub α_j = -θ gp_t(j-1/2)/(V d_j), super γ_j = -θ gm_t(j+1/2)/(V d_j),
// periodic corners α_0 (row 0, column n-1) and γ_{n-1} (row n-1, column 0).
// Sherman-Morrison with u = (-1, 0.., γ_{n-1}), v = (1, 0.., -α_0): the
// non-periodic T0 has diagonal 2 at row 0 and 1 + γ_{n-1} α_0 at row n-1;
// z = T0^{-1} u and κ = 1/(1 + z_0 - α_0 z_{n-1}) are stored so that
// x = y - κ (y_0 - α_0 y_{n-1}) z with y = T0^{-1} d.
// One wave per ring; lane L owns the nodes [L*bang, (L+1)*bang).  The
// multipliers, pivots and z of a ring are stored in the sweep's own order:
// node L*bang + k at (i-1)*64*bang + 64*k + L (a ring stride of 64*bang),
// so that the sweep reads them with coalesced loads.

__device__ __forceinline__ void ang_coef(const PdInst &I, int i, int j, double th, double &al,
                                         double &ga) {
  const int n = I.n;
  const int row = (i - 1) * n;
  const int jl = (j == 0) ? n - 1 : j - 1;
  const double s = -th * G(I.inv_rw)[i] * G(I.inv_dth)[j] / G(I.diag)[row + j];
  al = s * G(I.k64.gp_t)[row + jl];
  ga = s * G(I.k64.gm_t)[row + j];
}

template <int BM>
__global__ __launch_bounds__(256) void k_fact_ang(const PdInst *insts, const int2 *map) {
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  const PdScalars *sc = I.sc;
  if (sc->status != ST_ACTIVE || sc->stage != STAGE_START || !sc->refactor) return;
  const int m = I.m, n = I.n, B = I.bang, aw = I.aw;
  const int lane = threadIdx.x & 63;
  const int i = mp.y * 4 + (threadIdx.x >> 6) + 1;
  if (i > m) return;                                  // whole wave exits together
  const double th = sc->theta;
  const int frow = (i - 1) * 64 * B;   // ring i in the sweep's layout
  const int j0 = lane * B;
  const int cnt = max(0, min(B, n - j0));
  double a0, gl, tmp;
  ang_coef(I, i, 0, th, a0, tmp);
  ang_coef(I, i, n - 1, th, tmp, gl);

  double al[BM] = {}, ga[BM] = {}, dd[BM] = {};
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    if (k < cnt) {
      const int j = j0 + k;
      ang_coef(I, i, j, th, al[k], ga[k]);
      dd[k] = (j == 0) ? 2.0 : ((j == n - 1) ? 1.0 + gl * a0 : 1.0);
      if (j == 0) al[k] = 0.0;          // T0 drops the corners
      if (j == n - 1) ga[k] = 0.0;
    }
  }
  // γ of the row before this lane's segment
  double gprev = 0.0;
  if (cnt > 0 && j0 >= 1) {
    double t0;
    ang_coef(I, i, j0 - 1, th, t0, gprev);
  }
  // segment continuant product, then an exclusive scan over the lanes
  Mat2 Mp{1.0, 0.0, 0.0, 1.0};
  double cp = gprev;
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    if (k < cnt) {
      const Mat2 Mi{dd[k], -al[k] * cp, 1.0, 0.0};
      Mp = norm2(mul2(Mi, Mp));
      cp = ga[k];
    }
  }
  Mat2 S = Mp;   // inclusive product over lanes 0..lane (later lanes on the left)
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    Mat2 o{__shfl_up(S.a, d, 64), __shfl_up(S.b, d, 64), __shfl_up(S.c, d, 64), __shfl_up(S.d, d, 64)};
    if (lane >= d) S = norm2(mul2(S, o));
  }
  Mat2 E{__shfl_up(S.a, 1, 64), __shfl_up(S.b, 1, 64), __shfl_up(S.c, 1, 64), __shfl_up(S.d, 1, 64)};
  // incoming (q_{j0-1}, q_{j0-2}) = E (1, 0)
  double q1 = E.a, q0 = E.c;
  if (lane == 0) {
    q1 = 1.0;
    q0 = 0.0;
  }
  double u_prev = (q0 != 0.0) ? q1 / q0 : 1.0;
  cp = gprev;
  double fl[BM] = {}, gf[BM] = {}, ul[BM] = {};
  GAS float *uinv = G(I.af_uinv), *ff = G(I.af_f), *gg = G(I.af_g), *zz = G(I.af_z);
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    if (k < cnt) {
      const double u = dd[k] - al[k] * cp / u_prev;
      const double ui = 1.0 / u;
      ul[k] = ui;
      fl[k] = al[k] * ui;
      gf[k] = ga[k] * ui;
      const int fi = afac_index(frow, j0 + k, B, aw);
      uinv[fi] = (float)ui;
      ff[fi] = (float)fl[k];
      gg[fi] = (float)gf[k];
      u_prev = u;
      cp = ga[k];
    }
  }
  // z = T0^{-1} u, u = (-1, 0, ..., 0, γ_{n-1}): forward then backward scans
  double wl[BM] = {};
  Aff A{1.0, 0.0};
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    if (k < cnt) {
      const int j = j0 + k;
      const double uj = (j == 0) ? -1.0 : ((j == n - 1) ? gl : 0.0);
      A.e = ul[k] * uj - fl[k] * A.e;
      A.P *= -fl[k];
      wl[k] = A.e;
    }
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const Aff o{__shfl_up(A.P, d, 64), __shfl_up(A.e, d, 64)};
    if (lane >= d) A = compose(A, o);
  }
  double Win = __shfl_up(A.e, 1, 64);
  if (lane == 0) Win = 0.0;
  double P = 1.0;
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    if (k < cnt) {
      P *= -fl[k];
      wl[k] += P * Win;
    }
  }
  Aff Bk{1.0, 0.0};
#pragma unroll
  for (int k = BM - 1; k >= 0; --k) {
    if (k < cnt) {
      Bk.e = wl[k] - gf[k] * Bk.e;
      Bk.P *= -gf[k];
      wl[k] = Bk.e;
    }
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const Aff o{__shfl_down(Bk.P, d, 64), __shfl_down(Bk.e, d, 64)};
    if (lane + d < 64) Bk = compose(Bk, o);
  }
  double Xin = __shfl_down(Bk.e, 1, 64);
  if (lane == 63) Xin = 0.0;
  double Q = 1.0, zlast = 0.0;
#pragma unroll
  for (int k = BM - 1; k >= 0; --k) {
    if (k < cnt) {
      Q *= -gf[k];
      wl[k] += Q * Xin;
      zz[afac_index(frow, j0 + k, B, aw)] = (float)wl[k];
      if (j0 + k == n - 1) zlast = wl[k];
    }
  }
  const double z0 = __shfl(wl[0], 0, 64);
  const double zl = __shfl(zlast, (n - 1) / B, 64);
  const double kap = 1.0 / (1.0 + z0 - a0 * zl);
  if (lane == 0) {
    G(I.af_kappa)[i - 1] = kap;
    G(I.af_alpha0)[i - 1] = a0;
  }
  if (i != 1) return;

  // Ring 1 and the origin: ã_j = -θ gp_r(1/2, j)/(V_1j d_1j) couples ring 1
  // to the origin, c̃_j = -θ gm_r(1/2, j)/(V_0 d_0) the origin to ring 1.
  // q = T1^{-1} ã by the same substitutions and Sherman-Morrison closure,
  // then σ = 1 - c̃·q (a fixed-order wave sum: every lane gets the same bits).
  const GAS double *dg = G(I.diag), *gpr = G(I.k64.gp_r), *gmr = G(I.k64.gm_r);
  const double d0 = dg[m * n], iv1 = G(I.inv_rw)[1];
  double qv[BM] = {};
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    if (k < cnt) {
      const int j = j0 + k;
      qv[k] = -th * iv1 * G(I.inv_dth)[j] * gpr[j] / dg[j];
    }
  }
  Aff F{1.0, 0.0};
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    if (k < cnt) {
      F.e = ul[k] * qv[k] - fl[k] * F.e;
      F.P *= -fl[k];
      qv[k] = F.e;
    }
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const Aff o{__shfl_up(F.P, d, 64), __shfl_up(F.e, d, 64)};
    if (lane >= d) F = compose(F, o);
  }
  double Fin = __shfl_up(F.e, 1, 64);
  if (lane == 0) Fin = 0.0;
  double PF = 1.0;
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    if (k < cnt) {
      PF *= -fl[k];
      qv[k] += PF * Fin;
    }
  }
  Aff Bq{1.0, 0.0};
#pragma unroll
  for (int k = BM - 1; k >= 0; --k) {
    if (k < cnt) {
      Bq.e = qv[k] - gf[k] * Bq.e;
      Bq.P *= -gf[k];
      qv[k] = Bq.e;
    }
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const Aff o{__shfl_down(Bq.P, d, 64), __shfl_down(Bq.e, d, 64)};
    if (lane + d < 64) Bq = compose(Bq, o);
  }
  double Qin = __shfl_down(Bq.e, 1, 64);
  if (lane == 63) Qin = 0.0;
  double QB = 1.0, qlast = 0.0;
#pragma unroll
  for (int k = BM - 1; k >= 0; --k) {
    if (k < cnt) {
      QB *= -gf[k];
      qv[k] += QB * Qin;
      if (j0 + k == n - 1) qlast = qv[k];
    }
  }
  const double sf = kap * (__shfl(qv[0], 0, 64) - a0 * __shfl(qlast, (n - 1) / B, 64));
  double dot = 0.0, cv[BM] = {};
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    if (k < cnt) {
      qv[k] -= sf * wl[k];
      cv[k] = -th * I.inv_V0 * gmr[j0 + k] / d0;
      dot += cv[k] * qv[k];
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) dot += __shfl_xor(dot, d, 64);
  const double sigma = 1.0 - dot;
  // an arrow whose Schur complement is not safely positive is not used:
  // the origin then passes through as in the radial sweep
  const bool use = sigma > 1e-6 && sigma < INFINITY;
  GAS float *qq = G(I.af_q), *cc = G(I.af_c);
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    if (k < cnt) {
      qq[afac_index(0, j0 + k, B, aw)] = use ? (float)qv[k] : 0.0f;
      cc[afac_index(0, j0 + k, B, aw)] = use ? (float)cv[k] : 0.0f;
    }
  }
  if (lane == 0) G(I.af_sigma)[0] = use ? sigma : 1.0;
}

// ------------------------------------------------------------ stencil march
//
// One wave owns 64 consecutive θ-columns and rb consecutive rings (PD_RB, or
// twice that when the launch schedule asks for it) and
// marches outward in r, keeping the radial neighbours and the shared radial
// faces in registers and fetching the next ring (stencil operands and the
// epilogue's own operands) while it computes the current one.  A block
// stacks PD_STEN_WAVES such waves on top of each other, so the rings one
// wave reads beyond its own are mostly read by its neighbour in the same CU.
// The θ-neighbours come from the adjacent lanes by cross-lane permutes; the
// columns just outside the wave (including the periodic seam j = n-1 <-> 0)
// are fetched for all of the tile's rings at once and handed out row by row.
// The origin row is a sum over ring 1, left as a per-block partial.

struct Nil {};
struct Pre2 {
  double a, b;
};
struct Pre3 {
  double a, b, c;
};
struct Hist3 {   // n^{k-1..k-3} and their L at a node
  double x1, x2, x3, l1, l2, l3;
};
__device__ __forceinline__ Nil no_pre(int) { return Nil{}; }

struct TileGeo {
  int m, n, lane, j, jc, i0, i1, jl0, jr0;
  bool act, need_l, need_r;
};

__device__ __forceinline__ TileGeo tile_geo(int m, int n, int cg, int rg, int rb) {
  TileGeo g;
  g.m = m;
  g.n = n;
  g.lane = threadIdx.x & 63;
  g.j = cg * 64 + g.lane;
  g.act = g.j < n;
  g.jc = g.act ? g.j : n - 1;
  const int jfirst = cg * 64, jlast = min(cg * 64 + 63, n - 1);
  g.jl0 = (jfirst == 0) ? n - 1 : jfirst - 1;
  g.jr0 = (jlast == n - 1) ? 0 : jlast + 1;
  g.need_l = g.lane == 0;
  g.need_r = g.j == jlast;
  g.i0 = rg * rb + 1;
  g.i1 = min(g.i0 + rb - 1, m);
  return g;
}

// pre(idx) loads what the epilogue needs at node idx (one ring ahead);
// epi(i, j, idx, x, Lx, ld, pre) finishes node idx (ld: the diagonal of L
// there, l_diag).
template <typename TF, typename TX, int NV, class Pre, class Epi>
__device__ __forceinline__ void sten_tile(const TileGeo &g, const GAS TF *__restrict__ gp_r,
                                          const GAS TF *__restrict__ gm_r,
                                          const GAS TF *__restrict__ gp_t,
                                          const GAS TF *__restrict__ gm_t,
                                          const GAS TX *__restrict__ X0,
                                          const GAS TX *__restrict__ X1,
                                          const GAS TX *__restrict__ X2,
                                          const GAS TX *__restrict__ X3,
                                          const GAS double *__restrict__ inv_rw,
                                          const GAS double *__restrict__ inv_dth,
                                          const GAS double *__restrict__ bnode, double (&S0)[NV],
                                          Pre &&pre, Epi &&epi) {
  const int m = g.m, n = g.n, jc = g.jc;
  const int i0 = g.i0, i1 = g.i1, nr = i1 - i0 + 1;
  const int orig = m * n;
  const GAS TX *X[4] = {X0, X1, X2, X3};
  const double idth = inv_dth[jc];
  // wave-edge columns for every row of the tile
  const int hr = (g.lane < nr) ? (i0 - 1 + g.lane) * n : (i0 - 1) * n;
  double hxl[NV], hxr[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    hxl[v] = (double)X[v][hr + g.jl0];
    hxr[v] = (double)X[v][hr + g.jr0];
  }
  const double hgpl = (double)gp_t[hr + g.jl0], hgml = (double)gm_t[hr + g.jl0];

  double xb[NV], xc[NV], xa[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    xb[v] = (i0 == 1) ? (double)X[v][orig] : (double)X[v][(i0 - 2) * n + jc];
    xc[v] = (double)X[v][(i0 - 1) * n + jc];
    xa[v] = (i0 < m) ? (double)X[v][i0 * n + jc] : 0.0;
  }
  double gpi = (double)gp_r[(i0 - 1) * n + jc], gmi = (double)gm_r[(i0 - 1) * n + jc];
  double gpo = (double)gp_r[i0 * n + jc], gmo = (double)gm_r[i0 * n + jc];
  double gpt = (double)gp_t[(i0 - 1) * n + jc], gmt = (double)gm_t[(i0 - 1) * n + jc];
  double bP = bnode ? bnode[(i0 - 1) * n + jc] : 0.0;
  double ivr = inv_rw[i0];
  auto pc = pre((i0 - 1) * n + jc);
  for (int i = i0; i <= i1; ++i) {
    // prefetch ring i+1
    double nxa[NV], ngpo = 0.0, ngmo = 0.0, ngpt = 0.0, ngmt = 0.0, nb = 0.0, nivr = 0.0;
    const bool more = i < i1;
    const auto pn = pre((more ? i : i - 1) * n + jc);
#pragma unroll
    for (int v = 0; v < NV; ++v) nxa[v] = (more && i + 1 < m) ? (double)X[v][(i + 1) * n + jc] : 0.0;
    if (more) {
      ngpo = (double)gp_r[(i + 1) * n + jc];
      ngmo = (double)gm_r[(i + 1) * n + jc];
      ngpt = (double)gp_t[i * n + jc];
      ngmt = (double)gm_t[i * n + jc];
      nb = bnode ? bnode[i * n + jc] : 0.0;
      nivr = inv_rw[i + 1];
    }
    const int row = (i - 1) * n;
    const int hi = i - i0;
    double gptl = __shfl_up(gpt, 1, 64), gmtl = __shfl_up(gmt, 1, 64);
    const double hgp = __shfl(hgpl, hi, 64), hgm = __shfl(hgml, hi, 64);
    if (g.need_l) {
      gptl = hgp;
      gmtl = hgm;
    }
    const double ivV = ivr * idth;
    double Lx[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double xl = __shfl_up(xc[v], 1, 64), xr = __shfl_down(xc[v], 1, 64);
      const double hl = __shfl(hxl[v], hi, 64), hrr = __shfl(hxr[v], hi, 64);
      if (g.need_l) xl = hl;
      if (g.need_r) xr = hrr;
      const double fs = gpo * xc[v] - gmo * xa[v] + gmi * xc[v] - gpi * xb[v] + gpt * xc[v] -
                        gmt * xr + gmtl * xc[v] - gptl * xl;
      Lx[v] = ivV * fs + bP * xc[v];
      if (i == 1 && g.act) S0[v] += gpi * xb[v] - gmi * xc[v];
    }
    if (g.act) epi(i, jc, row + jc, xc, Lx, l_diag(ivV, gpo, gmi, gpt, gmtl, bP), pc);
    pc = pn;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      xb[v] = xc[v];
      xc[v] = xa[v];
      xa[v] = nxa[v];
    }
    gpi = gpo;
    gmi = gmo;
    gpo = ngpo;
    gmo = ngmo;
    gpt = ngpt;
    gmt = ngmt;
    bP = nb;
    ivr = nivr;
  }
}

enum { SM_APPLY = 0, SM_BEGIN = 1, SM_V = 2, SM_T = 3, SM_UR = 4, SM_EST = 5, SM_GRAM = 6, SM_RES = 7 };

// Origin rows, closed by a later kernel from the producers' partial sums
// (the ring-1 face sums S0 and the ring parts of the norms).

// S0 (the origin row's ring-1 face sum) of n^{k-a}: the Gram pass's total
// s0k for n^k (and for the levels the guess does not use, which alias n^k),
// the value its own Gram pass kept for an earlier level.
__device__ __forceinline__ double s0_of(const PdScalars *sc, int a, double s0k) {
  return (a == 0 || a > sc->ex_n) ? s0k : sc->s0h[sol_slot(sc->rot, a)];
}

// Level begin at the origin: rhs b_0, the guess and its scaled residual.
struct OriginBegin {
  double b, xg, r, rs, bb, rr;
};
__device__ __forceinline__ OriginBegin origin_begin(const PdInst &I, const PdScalars *sc,
                                                    const double (&tot)[PD_NBEGIN]) {
  const int orig = I.m * I.n;
  const double inv_dt = sc->inv_dt, th = sc->theta;
  const int ne = sc->ex_n;
  const double bo = I.has_b ? I.b_node[orig] : 0.0;
  const double s0k = I.gram_tot[PD_GRAM_S0];
  double xa[PD_NHIST], La[PD_NHIST];
  for (int a = 0; a < PD_NHIST; ++a) {
    xa[a] = I.sol[sol_slot(sc->rot, a <= ne ? a : 0)][orig];
    La[a] = I.inv_V0 * s0_of(sc, a, s0k) + bo * xa[a];
  }
  double b = inv_dt * xa[0] - (1.0 - th) * La[0];
  for (int q = 0; q < I.nsrc; ++q) b += sc->cq[q] * I.g[q * I.npad + orig];
  const double id = origin_invd(I, inv_dt, th);
  double g = 0.0, Lg = 0.0;
  for (int a = 0; a < PD_NHIST; ++a) {
    g += sc->guess_w[a] * xa[a];
    Lg += sc->guess_w[a] * La[a];
  }
  OriginBegin O;
  O.b = b;
  O.xg = g;
  O.r = b - (inv_dt * g + th * Lg);
  O.rs = O.r * id;
  O.rr = tot[1] + O.rs * O.rs;
  const double bs = b * id;
  O.bb = tot[0] + bs * bs;
  return O;
}
__device__ __forceinline__ void origin_begin_store(const PdInst &I, const PdScalars *sc,
                                                   const OriginBegin &O) {
  const int orig = I.m * I.n;
  I.bvec[orig] = O.b;
  I.sol[sol_slot(sc->rot, -1)][orig] = O.xg;
  if (I.mixed) {
    I.k32.r[orig] = (float)O.rs;
    I.k32.rh[orig] = (float)O.rs;
    I.inv_diag32[orig] = (float)origin_invd(I, sc->inv_dt, sc->theta);
  } else {
    I.k64.r[orig] = O.rs;
    I.k64.rh[orig] = O.rs;
  }
}

// The initial guess of a level.  With y_a = D^{-1} A n^{k-a} (a = 0..ne),
// the Gram pass sums over the ring nodes both polynomial candidates' scaled
// residuals r_c = D^{-1}b - Σ_a w_{c,a} y_a, so that the better candidate
// is known at this very level.  It is then corrected by least squares over
// the span of n^k and its first ne differences, whose images are z_0 = y_0,
// z_1 = y_0 - y_1, z_2 = y_0 - 2y_1 + y_2, z_3 = y_0 - 3y_1 + 3y_2 - y_3:
// minimise ||r_c - Σ_i d_i z_i|| by the normal equations, scaled to a unit
// diagonal and factored by Cholesky while the pivots stay above rounding
// level.  Solving for the correction, whose right-hand side is the already
// small r_c, keeps the rounding of these badly conditioned equations at the
// scale of r_c rather than of b.  The correction is taken only when it
// predicts at most half the candidate's residual norm.  The origin row is
// added to the partial sums here.  Returns the candidate, plus 2 when
// corrected.
__device__ __forceinline__ void gram_dirs(const double (&y)[PD_NHIST], double (&z)[PD_NHIST]) {
  const double d1a = y[0] - y[1], d1b = y[1] - y[2], d1c = y[2] - y[3];
  const double d2a = d1a - d1b, d2b = d1b - d1c;
  z[0] = y[0];
  z[1] = d1a;
  z[2] = d2a;
  z[3] = d2a - d2b;
}
__device__ __forceinline__ int begin_guess(const PdInst &I, const PdScalars *sc,
                                           const double (&tot)[PD_NGRAM], double (&w)[PD_NHIST]) {
  const int orig = I.m * I.n;
  const double inv_dt = sc->inv_dt, th = sc->theta;
  const int ne = sc->ex_n;
  const double bo = I.has_b ? I.b_node[orig] : 0.0;
  const double id = origin_invd(I, inv_dt, th);
  double y[PD_NHIST], xa0 = 0.0, La0 = 0.0;
#pragma unroll
  for (int a = 0; a < PD_NHIST; ++a) {
    const double xa = I.sol[sol_slot(sc->rot, a <= ne ? a : 0)][orig];
    const double La = I.inv_V0 * s0_of(sc, a, tot[PD_GRAM_S0]) + bo * xa;
    y[a] = (inv_dt * xa + th * La) * id;
    if (a == 0) {
      xa0 = xa;
      La0 = La;
    }
  }
  double b = inv_dt * xa0 - (1.0 - th) * La0;
  for (int q = 0; q < I.nsrc; ++q) b += sc->cq[q] * I.g[q * I.npad + orig];
  const double bs = b * id;
  double z[PD_NHIST], rc[2];
  gram_dirs(y, z);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    rc[c] = bs;
#pragma unroll
    for (int a = 0; a < PD_NHIST; ++a) rc[c] -= sc->ex_w[c][a] * y[a];
  }
  const double rr0 = tot[18] + rc[0] * rc[0], rr1 = tot[19] + rc[1] * rc[1];
  // below three earlier levels both candidates are the same polynomial
  const int base = (ne == PD_NHIST - 1 && rr1 < rr0) ? 1 : 0;
  const double rrb = base ? rr1 : rr0, rb = rc[base];
  double G[PD_NHIST][PD_NHIST], h[PD_NHIST];
  int t = 0;
#pragma unroll
  for (int i = 0; i < PD_NHIST; ++i) {
#pragma unroll
    for (int j = i; j < PD_NHIST; ++j) {
      G[i][j] = G[j][i] = tot[t] + z[i] * z[j];
      ++t;
    }
    h[i] = tot[10 + PD_NHIST * base + i] + z[i] * rb;
  }
  // fixed loop bounds and masks throughout, so that everything stays in registers
  double sca[PD_NHIST], L[PD_NHIST][PD_NHIST], u[PD_NHIST];
  bool live = true;
  int used = 0;
#pragma unroll
  for (int j = 0; j < PD_NHIST; ++j) {
    sca[j] = 0.0;
    u[j] = 0.0;
#pragma unroll
    for (int k = 0; k < PD_NHIST; ++k) L[j][k] = 0.0;
    if (live && j <= ne && G[j][j] > 0.0 && G[j][j] < INFINITY) {
      sca[j] = 1.0 / sqrt(G[j][j]);
    } else {
      live = false;
    }
  }
  live = true;
#pragma unroll
  for (int j = 0; j < PD_NHIST; ++j) {
    if (live && sca[j] > 0.0) {
      double d = G[j][j] * sca[j] * sca[j];
#pragma unroll
      for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
      if (d > 1e-13) {
        L[j][j] = sqrt(d);
#pragma unroll
        for (int i = j + 1; i < PD_NHIST; ++i) {
          double v = G[i][j] * sca[i] * sca[j];
#pragma unroll
          for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
          L[i][j] = sca[i] > 0.0 ? v / L[j][j] : 0.0;
        }
        used = j + 1;
      } else {
        live = false;
      }
    } else {
      live = false;
    }
  }
#pragma unroll
  for (int j = 0; j < PD_NHIST; ++j) {
    if (j < used) {
      double v = h[j] * sca[j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[j][k] * u[k];
      u[j] = v / L[j][j];
    }
  }
#pragma unroll
  for (int j = PD_NHIST - 1; j >= 0; --j) {
    if (j < used) {
      double v = u[j];
#pragma unroll
      for (int k = j + 1; k < PD_NHIST; ++k)
        if (k < used) v -= L[k][j] * u[k];
      u[j] = v / L[j][j];
    }
  }
  // the correction's coefficients, its predicted residual ||r_c||² - h·d,
  // and the weights of the levels (z_i = Σ_a C[i][a] y_a)
  const double C[PD_NHIST][PD_NHIST] = {{1, 0, 0, 0}, {1, -1, 0, 0}, {1, -2, 1, 0}, {1, -3, 3, -1}};
  double dw[PD_NHIST] = {0.0, 0.0, 0.0, 0.0}, hd = 0.0;
  bool fin = true;
#pragma unroll
  for (int j = 0; j < PD_NHIST; ++j) {
    const double d = j < used ? u[j] * sca[j] : 0.0;
    hd += h[j] * d;
#pragma unroll
    for (int a = 0; a < PD_NHIST; ++a) dw[a] += d * C[j][a];
  }
#pragma unroll
  for (int a = 0; a < PD_NHIST; ++a) fin = fin && fabs(dw[a]) < INFINITY;
  const bool corr = used > 0 && fin && (rrb - hd) < 0.25 * rrb;
#pragma unroll
  for (int a = 0; a < PD_NHIST; ++a) w[a] = sc->ex_w[base][a] + (corr ? dw[a] : 0.0);
  return base + (corr ? 2 : 0);
}

// Refinement at the origin: r_0 <- r_0 - (A d)_0, with the previous r_0 kept
// in the scalars (slot by refinement parity, so the kernel that reads one
// slot writes the other).
struct OriginRefine {
  double d0, r, rs, rr;
};
__device__ __forceinline__ OriginRefine origin_refine(const PdInst &I, const PdScalars *sc,
                                                      const double (&tot)[2]) {
  const int orig = I.m * I.n;
  const double inv_dt = sc->inv_dt, th = sc->theta;
  const double bo = I.has_b ? I.b_node[orig] : 0.0;
  OriginRefine O;
  O.d0 = (double)I.k32.d[orig];
  const double rprev = sc->rout0[(sc->outer + 1) & 1];
  O.r = rprev - (inv_dt * O.d0 + th * (I.inv_V0 * tot[1] + bo * O.d0));
  O.rs = O.r * origin_invd(I, inv_dt, th);
  O.rr = tot[0] + O.rs * O.rs;
  return O;
}

// A row at the origin: (I/dt + θL)_0 x, scaled by 1/d_0.
template <typename TK>
__device__ __forceinline__ double origin_apply(const PdInst &I, double inv_dt, double th, double x0,
                                               double S0, double invd0) {
  const double bo = I.has_b ? I.b_node[I.m * I.n] : 0.0;
  return (inv_dt * x0 + th * (I.inv_V0 * S0 + bo * x0)) * invd0;
}

// Totals of the Gram pass's partial sums, one block per instance and slot,
// read by every block of the level-begin stencil (which would otherwise
// each sum PD_NGRAM x nb_sten partials).  Thread t sums blocks t, t + 256,
// ... in ascending order, then the block adds its threads in a fixed tree,
// so the order depends on the instance's own tiling alone.
__global__ __launch_bounds__(256) void k_gram_total(const PdInst *insts, int ninst) {
  const int q = blockIdx.x / PD_NGRAM, k = blockIdx.x % PD_NGRAM;
  if (q >= ninst) return;
  const PdInst &I = insts[q];
  PdScalars *sc = I.sc;
  if (sc->status != ST_ACTIVE || sc->stage != STAGE_START) return;
  const int nb = I.nb_sten;
  const double *part = I.part_g + (size_t)k * nb;
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) v += part[b];
  __shared__ double red[4];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double tot = ((red[0] + red[1]) + red[2]) + red[3];
    I.gram_tot[k] = tot;
    if (k == PD_GRAM_S0) {
      sc->s0h[sol_slot(sc->rot, 0)] = tot;   // S0 of n^k, for the levels to come
      sc->ld_ready = 1;                      // the Gram pass has stored L's diagonal
    }
  }
}

// Stencil kernels.  TK: storage type of the Krylov set the mode works on.
// Ring rows only; the origin row is closed by the consumer of the partials.
//  SM_APPLY: y = x/dt + θ L x (diagnostic; partial S0)
//  SM_GRAM:  (level begin, first pass) L n^k (stored), b as below and
//            y_a = D^{-1}A n^{k-a} from the stored L n^{k-a}; partials: the
//            Gram matrix of the difference directions of the y_a, their
//            products with D^{-1}b, S0 of n^k
//  SM_BEGIN: (no stencil) b = x^k/dt - (1-θ) L x^k + Σ_q c_q g_q + boundary;
//            x0 = Σ_a w_a n^{k-a};  r = D^{-1}(b - A x0);  r̂ = r
//            partials ||D^{-1}b||², ||r||²
//  SM_V:     v = D^{-1} A p̂,  partials r̂·v, S0(p̂)
//  SM_T:     t = D^{-1} A ŝ,  partials t·s, t·t, S0(ŝ)
//  SM_UR:    (mixed, when the inner solve has converged) r <- r - A d in
//            FP64, x <- x + d, r32 = r̂32 = D^{-1} r; partials ||r32||², S0(d)
//  SM_RES:   (a level has just converged) the FP64 residual b - A x of its
//            system, summed per ring with the cell volumes as weights
//            (Σ_j V_ij (b - A x)_ij per ring and column group), and S0(x)
template <typename TK, int MODE>
__global__ __launch_bounds__(256) void k_sten(const PdInst *insts, const int2 *map, double a_dt,
                                              double a_th, const TK *ax, TK *ay) {
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  PdScalars *sc = I.sc;
  if (MODE == SM_EST) {
    // adaptive stepping: f(t_0, x_0) once, then f at the end of every level
    if (!sc->adaptive) return;
    const bool ended = sc->in_level && sc->status == ST_DONE;
    if (!sc->need_f0 && !ended) return;
  } else if (MODE == SM_RES) {
    if (!level_converged(sc)) return;
  } else if (MODE != SM_APPLY) {
    if (sc->status != ST_ACTIVE) return;     // no block of this kernel changes the status
    if ((MODE == SM_BEGIN || MODE == SM_GRAM) && sc->stage != STAGE_START) return;
    if ((MODE == SM_V || MODE == SM_T) && !prec_match<TK>(I)) return;
    if (MODE == SM_UR && !I.mixed) return;
  }
  if (MODE == SM_UR) {
    // refine once the inner solve has iterated and met its tolerance: a
    // reduction by tol_inner, or a residual of half the outer tolerance,
    // whichever is reached first (no inner solve goes beyond what the
    // outer test needs)
    if (sc->inner_iters == 0) return;
    double tot[2];
    consume<2>(I.part_x, I.nb_elem, tot);
    const double goal = fmax(sc->tol_inner * sc->tol_inner * sc->r0norm2,
                             0.25 * sc->tol * sc->tol * sc->bnorm2);
    const bool due = tot[1] <= goal ||
                     sc->inner_iters >= sc->maxit_inner || sc->iters >= sc->maxit || !(tot[1] == tot[1]);
    if (!due) return;
    if (mp.y == 0 && threadIdx.x == 0) {
      sc->pend = PEND_REFINE;
      sc->outer = sc->outer + 1;
    }
  }
  // block mp.y: column group mp.y % ncg, waves stacked over row groups
  const int wave = threadIdx.x >> 6;
  const int rg0 = (mp.y / I.ncg) * PD_STEN_WAVES + wave;
  const bool wave_on = rg0 < I.nrg;
  const int cg = mp.y % I.ncg, rg = wave_on ? rg0 : 0;
  const int m = I.m, n = I.n;
  const KSet<TK> &KS = kset<TK>(I);
  const TileGeo geo = tile_geo(m, n, cg, rg, I.rb);
  const GAS double *inv_rw = G(I.inv_rw), *inv_dth = G(I.inv_dth);
  const GAS double *bnode = I.has_b ? G(I.b_node) : nullptr;

  if (MODE == SM_APPLY) {
    const double inv_dt = 1.0 / a_dt, th = a_th;
    double S0[1] = {0.0};
    GAS TK *y = G(ay);
    if (wave_on)
      sten_tile<TK, TK, 1>(geo, G(KS.gp_r), G(KS.gm_r), G(KS.gp_t), G(KS.gm_t), G(ax), G(ax), G(ax), G(ax), inv_rw,
                           inv_dth, bnode, S0, no_pre,
                           [&](int, int, int idx, const double *xc, const double *Lx, double, Nil) {
                             y[idx] = (TK)(inv_dt * xc[0] + th * Lx[0]);
                           });
    produce<1>(S0, I.part_a, I.nb_sten, mp.y);
  } else if (MODE == SM_GRAM) {
    // the rows of the least-squares problem of the guess, summed per block.
    // The stencil runs on n^k alone: L n^k is stored (lsol) for this level's
    // begin pass and the next levels, whose L n^{k-a} are read back (the same
    // values a stencil on those states would give).  The first Gram pass of
    // a solve call also stores L's diagonal.
    const double inv_dt = sc->inv_dt, th = sc->theta;
    const int ne = sc->ex_n, rot = sc->rot;
    const bool put_ld = sc->ld_ready == 0;
    const int s0 = sol_slot(rot, 0);
    const double *xk0 = I.sol[s0];
    // levels the guess does not use read n^k (their values are not used)
    const GAS double *xh1 = G((const double *)(ne >= 1 ? I.sol[sol_slot(rot, 1)] : xk0));
    const GAS double *xh2 = G((const double *)(ne >= 2 ? I.sol[sol_slot(rot, 2)] : xk0));
    const GAS double *xh3 = G((const double *)(ne >= 3 ? I.sol[sol_slot(rot, 3)] : xk0));
    const GAS double *lh1 = G((const double *)(ne >= 1 ? I.lsol[sol_slot(rot, 1)] : xk0));
    const GAS double *lh2 = G((const double *)(ne >= 2 ? I.lsol[sol_slot(rot, 2)] : xk0));
    const GAS double *lh3 = G((const double *)(ne >= 3 ? I.lsol[sol_slot(rot, 3)] : xk0));
    GAS double *lo = G(I.lsol[s0]), *ldo = G(I.ldiag);
    double cq[PD_MAXSRC], w0[PD_NHIST], w1[PD_NHIST];
    for (int q = 0; q < PD_MAXSRC; ++q) cq[q] = sc->cq[q];
    for (int a = 0; a < PD_NHIST; ++a) {
      w0[a] = sc->ex_w[0][a];
      w1[a] = sc->ex_w[1][a];
    }
    const int nsrc = I.nsrc, npad = I.npad;
    double acc[PD_NGRAM] = {};
    double S0[1] = {0.0};
    const GAS double *gmr = G(I.k64.gm_r), *gsrc = G(I.g), *nbv = G(I.nb);
    if (wave_on)
      sten_tile<double, double, 1>(
          geo, G(I.k64.gp_r), G(I.k64.gm_r), G(I.k64.gp_t), G(I.k64.gm_t), G(xk0), G(xk0), G(xk0),
          G(xk0), inv_rw, inv_dth, bnode, S0,
          [&](int idx) { return Hist3{xh1[idx], xh2[idx], xh3[idx], lh1[idx], lh2[idx], lh3[idx]}; },
          [&](int i, int j, int idx, const double *xk, const double *Lk, double ld, Hist3 hq) {
            lo[idx] = Lk[0];
            if (put_ld) ldo[idx] = ld;
            const double xc[PD_NHIST] = {xk[0], ne >= 1 ? hq.x1 : xk[0], ne >= 2 ? hq.x2 : xk[0],
                                         ne >= 3 ? hq.x3 : xk[0]};
            const double Lx[PD_NHIST] = {Lk[0], ne >= 1 ? hq.l1 : Lk[0], ne >= 2 ? hq.l2 : Lk[0],
                                         ne >= 3 ? hq.l3 : Lk[0]};
            double b = inv_dt * xc[0] - (1.0 - th) * Lx[0];
            for (int q = 0; q < nsrc; ++q) b += cq[q] * gsrc[q * npad + idx];
            if (i == m) {
              double Nm = 0.0;
              for (int q = 0; q < nsrc; ++q) Nm += cq[q] * nbv[q * n + j];
              b += inv_rw[i] * inv_dth[j] * gmr[m * n + j] * Nm;
            }
            const double id = 1.0 / diag_of(inv_dt, th, ld);
            double y[PD_NHIST], z[PD_NHIST];
#pragma unroll
            for (int a = 0; a < PD_NHIST; ++a) y[a] = (inv_dt * xc[a] + th * Lx[a]) * id;
            gram_dirs(y, z);
            double r0 = b * id, r1 = r0;
#pragma unroll
            for (int a = 0; a < PD_NHIST; ++a) {
              r0 -= w0[a] * y[a];
              r1 -= w1[a] * y[a];
            }
            int t = 0;
#pragma unroll
            for (int a = 0; a < PD_NHIST; ++a) {
#pragma unroll
              for (int c = a; c < PD_NHIST; ++c) acc[t++] += z[a] * z[c];
              acc[10 + a] += z[a] * r0;
              acc[10 + PD_NHIST + a] += z[a] * r1;
            }
            acc[18] += r0 * r0;
            acc[19] += r1 * r1;
          });
    acc[PD_GRAM_S0] = S0[0];
    produce<PD_NGRAM>(acc, I.part_g, I.nb_sten, mp.y);
  } else if (MODE == SM_BEGIN) {
    // b, the guess x0 = Σ_a w_a n^{k-a} and its residual D^{-1}(b - A x0),
    // node by node from the states, their L (lsol: A x0 = Σ_a w_a
    // (n^{k-a}/dt + θ L n^{k-a})) and L's diagonal; no stencil.  Every
    // block solves the same small problem of the guess from the Gram
    // totals; block 0 records the weights for the origin row.  The nodes
    // and the order of the partial sums are the stencil tile's.
    const double inv_dt = sc->inv_dt, th = sc->theta;
    const int ne = sc->ex_n, rot = sc->rot;
    double w0[PD_NHIST];
    int kind;
    {
      double tg[PD_NGRAM];
#pragma unroll
      for (int k = 0; k < PD_NGRAM; ++k) tg[k] = I.gram_tot[k];
      kind = begin_guess(I, sc, tg, w0);
    }
    const GAS double *xs[PD_NHIST], *ls[PD_NHIST];
#pragma unroll
    for (int a = 0; a < PD_NHIST; ++a) {
      const int sl = sol_slot(rot, a <= ne ? a : 0);
      xs[a] = G((const double *)I.sol[sl]);
      ls[a] = G((const double *)I.lsol[sl]);
    }
    double *x0 = I.sol[sol_slot(rot, -1)];
    double cq[PD_MAXSRC];
    for (int q = 0; q < PD_MAXSRC; ++q) cq[q] = sc->cq[q];
    const int nsrc = I.nsrc, npad = I.npad;
    const GAS double *gmr = G(I.k64.gm_r), *gsrc = G(I.g), *nbv = G(I.nb), *ldv = G(I.ldiag);
    GAS double *bv = G(I.bvec), *xo = G(x0);
    GAS double *rout = G(I.rout);
    GAS double *r64 = G(I.k64.r), *rh64 = G(I.k64.rh);
    GAS float *r32 = G(I.k32.r), *rh32 = G(I.k32.rh), *id32 = G(I.inv_diag32);
    const bool mixed = I.mixed;
    if (mp.y == 0 && threadIdx.x == 0) {
      sc->guess_kind = kind;
      for (int a = 0; a < PD_NHIST; ++a) sc->guess_w[a] = w0[a];
    }
    double acc[PD_NBEGIN] = {};   // ||D^-1 b||², ||D^-1 r||²
    if (wave_on && geo.act) {
      const int jc = geo.jc, nr = geo.i1 - geo.i0 + 1;
      // rings of the tile in groups of four, every load of a group issued
      // first (rows past the tile reread its last row and are not stored)
      for (int h0 = 0; h0 < nr; h0 += 4) {
        double xv[4][PD_NHIST], lv[4][PD_NHIST], ldn[4], gq[4][PD_MAXSRC];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int idx = (min(geo.i0 + h0 + u, geo.i1) - 1) * n + jc;
#pragma unroll
          for (int a = 0; a < PD_NHIST; ++a) {
            xv[u][a] = xs[a][idx];
            lv[u][a] = ls[a][idx];
          }
          ldn[u] = ldv[idx];
#pragma unroll
          for (int q = 0; q < PD_MAXSRC; ++q) gq[u][q] = gsrc[max(0, min(q, nsrc - 1)) * npad + idx];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = geo.i0 + h0 + u;
          if (i > geo.i1) break;
          const int idx = (i - 1) * n + jc;
          double b = inv_dt * xv[u][0] - (1.0 - th) * lv[u][0];
          for (int q = 0; q < nsrc; ++q) b += cq[q] * gq[u][q];
          if (i == m) {
            double Nm = 0.0;
            for (int q = 0; q < nsrc; ++q) Nm += cq[q] * nbv[q * n + jc];
            b += inv_rw[i] * inv_dth[jc] * gmr[m * n + jc] * Nm;
          }
          double xg = 0.0, Lg = 0.0;
#pragma unroll
          for (int a = 0; a < PD_NHIST; ++a) {
            xg += w0[a] * xv[u][a];
            Lg += w0[a] * lv[u][a];
          }
          const double r = b - (inv_dt * xg + th * Lg);
          const double id = 1.0 / diag_of(inv_dt, th, ldn[u]);
          const double rs = r * id, bs = b * id;
          bv[idx] = b;
          xo[idx] = xg;
          if (mixed) {
            rout[idx] = r;
            r32[idx] = (float)rs;
            rh32[idx] = (float)rs;
            id32[idx] = (float)id;
          } else {
            r64[idx] = rs;
            rh64[idx] = rs;
          }
          acc[0] += bs * bs;
          acc[1] += rs * rs;
        }
      }
    }
    produce<PD_NBEGIN>(acc, I.part_b, I.nb_sten, mp.y);
  } else if (MODE == SM_V || MODE == SM_T) {
    const double inv_dt = sc->inv_dt, th = sc->theta;
    const TK *xin = (MODE == SM_V) ? KS.ph : KS.sh;
    TK *yout = (MODE == SM_V) ? KS.v : KS.t;
    const TK *other = (MODE == SM_V) ? KS.rh : KS.s;
    GAS TK *yo = G(yout);
    const GAS TK *ot = G(other);
    const GAS TK *idg = G(KS.inv_d);
    double acc[3] = {0.0, 0.0, 0.0};
    double S0[1] = {0.0};
    if (wave_on)
      sten_tile<TK, TK, 1>(geo, G(KS.gp_r), G(KS.gm_r), G(KS.gp_t), G(KS.gm_t), G(xin), G(xin), G(xin), G(xin),
                           inv_rw, inv_dth, bnode, S0,
                           [&](int idx) {
                             // FP64 forms 1/diag from its faces; FP32 loads its rounded copy
                             return Pre2{sizeof(TK) == 8 ? 0.0 : (double)idg[idx], (double)ot[idx]};
                           },
                           [&](int, int, int idx, const double *xc, const double *Lx, double ld, Pre2 q) {
                             const double ia = sizeof(TK) == 8 ? 1.0 / diag_of(inv_dt, th, ld) : q.a;
                             const double y = (inv_dt * xc[0] + th * Lx[0]) * ia;
                             const TK ys = (TK)y;
                             yo[idx] = ys;
                             const double yd = (double)ys;
                             acc[0] += q.b * yd;
                             acc[1] += yd * yd;
                           });
    if (MODE == SM_V) {
      double pv[2] = {acc[0], S0[0]};
      produce<2>(pv, I.part_v, I.nb_sten, mp.y);
    } else {
      acc[2] = S0[0];
      produce<3>(acc, I.part_t, I.nb_sten, mp.y);
    }
  } else if (MODE == SM_EST) {
    // f = -L x + S(t) + c N(t) at the start (x_0) or at the end of a level
    // (x_{k+1}), and the ring part of ||d||², ||x_{k+1}||² and S0
    const bool f0 = sc->need_f0 != 0;
    const int k = sc->level;
    const double t = f0 ? sc->t_now : sc->t1, th = sc->theta, dt = sc->dt;
    const bool est = !f0 && k >= 1;
    const double dtp = est ? I.t_table[k] - I.t_table[k - 1] : 1.0;
    const GAS double *xv = G((const double *)I.sol[sol_slot(sc->rot, f0 ? 0 : -1)]);
    const GAS double *x0 = G((const double *)I.sol[sol_slot(sc->rot, 0)]);
    const GAS double *fk = G((const double *)I.fdot[k % 3]), *fkm = G((const double *)I.fdot[(k + 2) % 3]);
    GAS double *fo = G(I.fdot[(k + (f0 ? 0 : 1)) % 3]);
    const GAS double *gmr = G(I.k64.gm_r), *gsrc = G(I.g), *nbv = G(I.nb);
    double tq[PD_MAXSRC];
    for (int q = 0; q < PD_MAXSRC; ++q) tq[q] = q < I.nsrc ? tau_q(I.lam[q], I.tpow[q], t) : 0.0;
    const int nsrc = I.nsrc, npad = I.npad;
    double acc[3] = {0.0, 0.0, 0.0};
    double S0[1] = {0.0};
    if (wave_on)
      sten_tile<double, double, 1>(geo, G(I.k64.gp_r), G(I.k64.gm_r), G(I.k64.gp_t), G(I.k64.gm_t), xv, xv,
                                   xv, xv, inv_rw, inv_dth, bnode, S0, no_pre,
                                   [&](int i, int j, int idx, const double *xc, const double *Lx, double, Nil) {
                                     double f = -Lx[0];
                                     for (int q = 0; q < nsrc; ++q) f += tq[q] * gsrc[q * npad + idx];
                                     if (i == m) {
                                       double Nm = 0.0;
                                       for (int q = 0; q < nsrc; ++q) Nm += tq[q] * nbv[q * n + j];
                                       f += inv_rw[i] * inv_dth[j] * gmr[m * n + j] * Nm;
                                     }
                                     fo[idx] = f;
                                     if (est) {
                                       const double d = est_d(xc[0], x0[idx], f, fk[idx], fkm[idx], dt, dtp, th);
                                       acc[0] += d * d;
                                     }
                                     acc[1] += xc[0] * xc[0];
                                   });
    acc[2] = S0[0];
    produce<3>(acc, I.part_e, I.nb_sten, mp.y);
  } else if (MODE == SM_RES) {
    const double inv_dt = sc->inv_dt, th = sc->theta;
    const GAS double *xv = G((const double *)I.sol[sol_slot(sc->rot, -1)]);
    const GAS double *bv = G((const double *)I.bvec);
    double rs[2 * PD_RB];   // per ring of the wave's tile (at most 2 PD_RB rings)
#pragma unroll
    for (int u = 0; u < 2 * PD_RB; ++u) rs[u] = 0.0;
    double S0[1] = {0.0};
    if (wave_on)
      sten_tile<double, double, 1>(geo, G(I.k64.gp_r), G(I.k64.gm_r), G(I.k64.gp_t), G(I.k64.gm_t), xv, xv,
                                   xv, xv, inv_rw, inv_dth, bnode, S0,
                                   [&](int idx) { return Pre2{bv[idx], 0.0}; },
                                   [&](int i, int j, int, const double *xc, const double *Lx, double, Pre2 q) {
                                     const double r = q.a - (inv_dt * xc[0] + th * Lx[0]);
                                     const double v = r * (1.0 / (inv_rw[i] * inv_dth[j]));
                                     const int k = i - geo.i0;
#pragma unroll
                                     for (int u = 0; u < 2 * PD_RB; ++u)
                                       if (u == k) rs[u] += v;
                                   });
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < 2 * PD_RB; ++u) {
      const double tsum = wave_sum(rs[u]);   // every lane takes part; idle columns hold 0
      if (wave_on && lane == 0 && u < I.rb && geo.i0 + u <= geo.i1)
        I.part_c[(size_t)(geo.i0 + u - 1) * I.ncg + cg] = tsum;
    }
    produce<1>(S0, I.part_c0, I.nb_sten, mp.y);
  } else if (MODE == SM_UR) {
    // FP64 operator applied to the FP32 correction d
    const double inv_dt = sc->inv_dt, th = sc->theta;
    double *x = I.sol[sol_slot(sc->rot, -1)];
    GAS double *xg = G(x), *rout = G(I.rout);
    GAS float *r32 = G(I.k32.r), *rh32 = G(I.k32.rh);
    double acc[2] = {0.0, 0.0};
    double S0[1] = {0.0};
    if (wave_on)
      sten_tile<double, float, 1>(geo, G(I.k64.gp_r), G(I.k64.gm_r), G(I.k64.gp_t), G(I.k64.gm_t),
                                  G((const float *)I.k32.d), G((const float *)I.k32.d),
                                  G((const float *)I.k32.d), G((const float *)I.k32.d), inv_rw,
                                  inv_dth, bnode, S0,
                                  [&](int idx) { return Pre2{rout[idx], xg[idx]}; },
                                  [&](int, int, int idx, const double *xc, const double *Lx, double ld, Pre2 q) {
                                    const double r = q.a - (inv_dt * xc[0] + th * Lx[0]);
                                    const double rs = r * (1.0 / diag_of(inv_dt, th, ld));
                                    rout[idx] = r;
                                    xg[idx] = q.b + xc[0];
                                    r32[idx] = (float)rs;
                                    rh32[idx] = (float)rs;
                                    acc[0] += rs * rs;
                                  });
    acc[1] = S0[0];
    produce<2>(acc, I.part_ur, I.nb_sten, mp.y);
  }
}

// ------------------------------------------------------------ ring-mean correction
//
// When a level has converged, its iterate x is corrected once within the
// ring-constant vectors: x <- x + P c with P^T V A P c = P^T V (b - A x),
// the Galerkin projection of the level's system onto one value per ring
// (and the origin), V the cell volumes.  That tridiagonal system of m+1
// unknowns has the ring sums of PdInst::crs as coefficients.  It removes
// what the Krylov iteration converges slowest on these meshes: the θ-mean
// of the error on the rings next to the origin, where a handful of rows of
// the diagonally scaled residual carry coefficients near 1/(r_1 Δθ)².  The
// scheme's solution is unchanged (the correction only moves the iterate
// towards it).
//
// k_ring_total sums SM_RES's partials of every ring (one wave per ring, its
// column groups over the lanes, a fixed butterfly).  k_coarse (one block
// per instance) closes the origin row and solves the tridiagonal system by
// segments: every thread owns a contiguous run of rows; the pivots follow
// from the continuants q_i = d_i q_{i-1} - a_i c_{i-1} q_{i-2} (2x2 matrix
// products, rescaled by powers of two), and the forward and back
// substitutions are affine recurrences; each is joined across the threads
// by a scan in LDS.  k_cadd adds c to the iterate.

__global__ __launch_bounds__(256) void k_ring_total(const PdInst *insts, const int2 *map) {
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  if (!level_converged(I.sc)) return;
  const int i = mp.y * 4 + (threadIdx.x >> 6) + 1;
  if (i > I.m) return;                         // the whole wave
  const int lane = threadIdx.x & 63, ncg = I.ncg;   // ncg <= 32 (n <= 2048)
  double v = lane < ncg ? I.part_c[(size_t)(i - 1) * ncg + lane] : 0.0;
  v = wave_sum(v);
  if (lane == 0) I.cr_f[i] = v;
}

constexpr int PD_CC_THREADS = 256;
constexpr int PD_CC_ROWS = 9;   // rows per thread: 256 x 9 >= 2049 = the most rings plus the origin

// Exclusive scan over the block's threads at positions pos (a permutation of
// 0..blockDim-1): returns op-composition of the values at all smaller
// positions (later position on the left), ident at position 0.
template <typename V, class Op>
__device__ __forceinline__ V block_exclusive_scan(V v, int pos, V ident, Op op, V *sh) {
  const int T = blockDim.x;
  sh[pos] = v;
  __syncthreads();
  for (int o = 1; o < T; o <<= 1) {
    const V other = pos >= o ? sh[pos - o] : ident;
    __syncthreads();
    if (pos >= o) v = op(v, other);
    sh[pos] = v;
    __syncthreads();
  }
  const V ex = pos > 0 ? sh[pos - 1] : ident;
  __syncthreads();
  return ex;
}

// The ring-mean system for the right-hand side (f0 at the origin, known to
// thread 0; fr[i] for ring i), solved into out[0..m].  One block of
// PD_CC_THREADS threads; every thread calls it.
__device__ void ring_solve(const double *crs, int m, double inv_dt, double th, double f0, const double *fr,
                           double *out) {
  __shared__ Mat2 shm[PD_CC_THREADS];
  __shared__ Aff sha[PD_CC_THREADS];
  const int M1 = m + 1;
  const double *cU = crs + 4 * M1;
  const int t = threadIdx.x;
  const int S = (M1 + blockDim.x - 1) / blockDim.x;   // <= PD_CC_ROWS
  const int r0 = t * S;
  const int cnt = max(0, min(S, M1 - r0));
  double d[PD_CC_ROWS], a[PD_CC_ROWS], c[PD_CC_ROWS], f[PD_CC_ROWS];
  // every row's coefficients, all loads issued (rows past the end reread the
  // last row, masked below)
  {
    const GAS double *gc = G(crs), *gf = G(fr);
    double v[7][PD_CC_ROWS];
#pragma unroll
    for (int k = 0; k < PD_CC_ROWS; ++k) {
      const int i = min(r0 + k, M1 - 1);
#pragma unroll
      for (int q = 0; q < 6; ++q) v[q][k] = gc[q * M1 + i];
      v[6][k] = gf[i];
    }
#pragma unroll
    for (int k = 0; k < PD_CC_ROWS; ++k) {
      const bool own = k < cnt;
      d[k] = own ? v[0][k] * inv_dt + th * (v[1][k] + v[2][k] + v[3][k]) : 1.0;
      c[k] = own ? -th * v[4][k] : 0.0;
      a[k] = own ? -th * v[5][k] : 0.0;
      f[k] = own ? (r0 + k == 0 ? f0 : v[6][k]) : 0.0;
    }
  }
  const double cprev = (cnt > 0 && r0 > 0) ? -th * cU[r0 - 1] : 0.0;   // c_{r0-1}
  // pivots: the segment's continuant product, joined over the threads
  Mat2 P = {1.0, 0.0, 0.0, 1.0};
#pragma unroll
  for (int k = 0; k < PD_CC_ROWS; ++k) {
    if (k < cnt) {
      const double cm = k == 0 ? cprev : c[k - 1];
      P = norm2(mul2(Mat2{d[k], -a[k] * cm, 1.0, 0.0}, P));
    }
  }
  const Mat2 Pin = block_exclusive_scan(P, t, Mat2{1.0, 0.0, 0.0, 1.0},
                                        [](Mat2 later, Mat2 earlier) { return norm2(mul2(later, earlier)); }, shm);
  // 1/u of the row before the segment: q_{r0-2}/q_{r0-1} (0 before row 0)
  const double rho = Pin.a != 0.0 ? Pin.c / Pin.a : 0.0;
  double uinv[PD_CC_ROWS], l[PD_CC_ROWS];
  double up = rho;   // 1/u of the previous row
#pragma unroll
  for (int k = 0; k < PD_CC_ROWS; ++k) {
    uinv[k] = 1.0;
    l[k] = 0.0;
    if (k < cnt) {
      const double cm = k == 0 ? cprev : c[k - 1];
      const double u = d[k] - a[k] * cm * up;
      l[k] = a[k] * up;
      uinv[k] = 1.0 / u;
      up = uinv[k];
    }
  }
  // forward substitution y_i = f_i - l_i y_{i-1}
  Aff F = {1.0, 0.0};
#pragma unroll
  for (int k = 0; k < PD_CC_ROWS; ++k)
    if (k < cnt) F = compose(Aff{-l[k], f[k]}, F);
  const Aff Fin = block_exclusive_scan(F, t, Aff{1.0, 0.0}, [](Aff later, Aff earlier) { return compose(later, earlier); },
                                       sha);
  double y = Fin.e;   // y_{r0-1} (0 before row 0)
#pragma unroll
  for (int k = 0; k < PD_CC_ROWS; ++k) {
    if (k < cnt) {
      y = f[k] - l[k] * y;
      f[k] = y;
    }
  }
  // back substitution x_i = (y_i - c_i x_{i+1}) / u_i, joined from the last thread down
  Aff B = {1.0, 0.0};
#pragma unroll
  for (int k = PD_CC_ROWS - 1; k >= 0; --k)
    if (k < cnt) B = compose(Aff{-c[k] * uinv[k], f[k] * uinv[k]}, B);
  const int rpos = blockDim.x - 1 - t;
  const Aff Bin = block_exclusive_scan(B, rpos, Aff{1.0, 0.0}, [](Aff later, Aff earlier) { return compose(later, earlier); },
                                       sha);
  double xn = Bin.e;   // x_{r0+cnt} (0 past the last row)
#pragma unroll
  for (int k = PD_CC_ROWS - 1; k >= 0; --k) {
    if (k < cnt) {
      xn = (f[k] - c[k] * xn) * uinv[k];
      out[r0 + k] = xn;
    }
  }
}

__global__ __launch_bounds__(PD_CC_THREADS) void k_coarse(const PdInst *insts) {
  const PdInst &I = insts[blockIdx.x];
  const PdScalars *sc = I.sc;
  if (!level_converged(sc)) return;   // the same for every thread of the block
  const int n = I.n, orig = I.m * n;
  const double inv_dt = sc->inv_dt, th = sc->theta;
  double s0[1];
  consume<1>(I.part_c0, I.nb_sten, s0);
  // the origin's residual (thread 0 only)
  double f0 = 0.0;
  if (threadIdx.x == 0) {
    const double x0 = I.sol[sol_slot(sc->rot, -1)][orig];
    const double bo = I.has_b ? I.b_node[orig] : 0.0;
    const double r = I.bvec[orig] - (inv_dt * x0 + th * (I.inv_V0 * s0[0] + bo * x0));
    f0 = I.crs[0] * r;
  }
  ring_solve(I.crs, I.m, inv_dt, th, f0, I.cr_f, I.cr_c);
}

// x <- x + P c for the instances whose level has converged (elementwise).
__global__ __launch_bounds__(256) void k_cadd(const PdInst *insts, const int2 *map) {
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  if (!level_converged(I.sc)) return;
  double *x = I.sol[sol_slot(I.sc->rot, -1)];
  const int n = I.n, orig = I.m * I.n;
  const double *c = I.cr_c;
  const int base = mp.y * PD_ELEM_PER_BLOCK;
  for (int k = threadIdx.x; k < PD_ELEM_PER_BLOCK; k += blockDim.x) {
    const int idx = base + k;
    if (idx < orig) x[idx] += c[idx / n + 1];
    else if (idx == orig) x[idx] += c[0];
  }
}

// ------------------------------------------------------------ multigrid
//
// The θ-semi-coarsening V-cycle (PdMgLevel) as the preconditioner of one
// FP64 instance's Krylov system D^{-1}A: z ≈ (D^{-1}A)^{-1} y.  Every level
// smooths with one step of its own alternating-line sweeps,
//   x <- x + M_l^{-1} D_l^{-1} (g_l - A_l x),
// from x = 0 on the way down and again after the coarse correction on the
// way up; the ring means at the bottom are solved directly (ring_solve with
// the instance's ring sums: merging lines does not change them).  Level 0's
// right-hand side is diag(A) y and its pre-smoothed iterate is the Krylov
// vector z = M^{-1} y that the instance's own sweeps have just written.
//
// Vectors of a level l >= 1: g_l (right-hand side per volume); sh_l holds
// the pre-smoothed iterate, then x_l = sh_l + P e_{l+1} after the coarse
// correction, and sh_l the post-smoothing correction, so that the level
// returns e_l = x_l + sh_l.  The kernels run only while the instance
// iterates (the same gate as its own sweeps).

// Coarse line of line j of a level with nc coarse lines.
__device__ __forceinline__ int mg_coarse(int j, int nc) { return min(j >> 1, nc - 1); }

// (A_l x) at ring node (i, j) of a level, x(ii, jj) its values, x0 the origin's.
template <class X>
__device__ __forceinline__ double mg_apply(const PdMgLevel &L, int i, int j, double inv_dt, double th, X x,
                                           double x0) {
  const int n = L.n, m = L.m, row = (i - 1) * n;
  const int jl = j == 0 ? n - 1 : j - 1, jr = j == n - 1 ? 0 : j + 1;
  // every neighbour is loaded (rows clamped into the mesh) and the origin
  // and the boundary selected afterwards: a load under a per-lane condition
  // becomes a branch that waits for it
  const double xc = x(i, j);
  const double xiv = x(max(i - 1, 1), j), xov = x(min(i + 1, m), j);
  const double xl = x(i, jl), xr = x(i, jr);
  const double xi = i == 1 ? x0 : xiv;
  const double xo = i == m ? 0.0 : xov;
  const double fo = L.gp_r[i * n + j] * xc - L.gm_r[i * n + j] * xo;
  const double fi = L.gp_r[row + j] * xi - L.gm_r[row + j] * xc;
  const double fu = L.gp_t[row + j] * xc - L.gm_t[row + j] * xr;
  const double fl = L.gp_t[row + jl] * xl - L.gm_t[row + jl] * xc;
  const double ivV = L.inv_rw[i] * L.inv_dth[j];
  const double bP = L.has_b ? L.b_node[row + j] : 0.0;
  return inv_dt * xc + th * (ivV * ((fo - fi) + (fu - fl)) + bP * xc);
}

// Block sum in a fixed order (wave butterflies, then the waves in turn);
// every thread of the block calls it and receives the total.
__device__ __forceinline__ double mg_block_sum(double v) {
  __shared__ double red[16];
  __shared__ double tot;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w];
    tot = t;
  }
  __syncthreads();
  return tot;
}

// (A_l x)_0 at the origin from its faces to ring 1 (the calling block sums).
template <class X>
__device__ __forceinline__ double mg_apply_origin(const PdMgLevel &L, double inv_dt, double th, X x, double x0) {
  double s = 0.0;
  for (int j = threadIdx.x; j < L.n; j += blockDim.x) s += L.gp_r[j] * x0 - L.gm_r[j] * x(1, j);
  s = mg_block_sum(s);
  const double b0 = L.has_b ? L.b_node[L.m * L.n] : 0.0;
  return inv_dt * x0 + th * (L.inv_V0 * s + b0 * x0);
}

// Coarse faces, widths and reaction of level l+1 from level l (set-up, once
// per solve call): one thread per coarse (face row, line).
__global__ __launch_bounds__(256) void k_mg_faces(const PdMgLevel *lev, int l, double *gp_r, double *gm_r,
                                                  double *gp_t, double *gm_t, double *inv_dth, double *b_node) {
  const PdMgLevel F = lev[l];
  const int m = F.m, nf = F.n, nc = nf / 2;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (m + 1) * nc) return;
  const int i = gid / nc, J = gid % nc;
  const int j0 = 2 * J, cnt = J == nc - 1 ? nf - j0 : 2;
  double sp = 0.0, sm = 0.0, w = 0.0, vb = 0.0;
  for (int k = 0; k < cnt; ++k) {
    const int j = j0 + k;
    sp += F.gp_r[i * nf + j];
    sm += F.gm_r[i * nf + j];
    const double dw = 1.0 / F.inv_dth[j];
    w += dw;
    if (i >= 1 && F.has_b) vb += dw * F.b_node[(i - 1) * nf + j];
  }
  gp_r[i * nc + J] = sp;
  gm_r[i * nc + J] = sm;
  if (i == 0) {
    inv_dth[J] = 1.0 / w;
    if (F.has_b && J == 0) b_node[m * nc] = F.b_node[m * nf];
    return;
  }
  const int jl = j0 + cnt - 1;   // the line's last fine line: its upper face bounds the merged cell
  gp_t[(i - 1) * nc + J] = F.gp_t[(i - 1) * nf + jl];
  gm_t[(i - 1) * nc + J] = F.gm_t[(i - 1) * nf + jl];
  if (F.has_b) b_node[(i - 1) * nc + J] = vb / w;
}

// Down: the volume-weighted residual of level lc-1 summed over each coarse
// cell, as level lc's right-hand side g (per volume) and its sweep input
// r = g / diag.  Level 0: g = diag y, iterate z; else g and sh of the level.
// One thread per coarse ring node; the last block takes the origin.
__global__ __launch_bounds__(256) void k_mg_down(const PdScalars *sc, const PdMgLevel *lev, int lc,
                                                 const double *y, const double *z) {
  if (!inner_active(sc)) return;   // the same for the whole grid
  const PdMgLevel Fl = lev[lc - 1], Cl = lev[lc];
  const double inv_dt = sc->inv_dt, th = sc->theta;
  const bool top = lc == 1;
  const double *xf = top ? z : Fl.sh;
  const int m = Cl.m, nc = Cl.n, nf = Fl.n;
  const double x0 = xf[m * nf];
  auto xv = [&](int ii, int jj) { return xf[(ii - 1) * nf + jj]; };
  if (blockIdx.x == gridDim.x - 1) {
    const double ax = mg_apply_origin(Fl, inv_dt, th, xv, x0);
    if (threadIdx.x == 0) {
      const double g = top ? Fl.diag[m * nf] * y[m * nf] : Fl.g[m * nf];
      const double gc = g - ax;   // the origin cell is kept: same volume
      Cl.g[m * nc] = gc;
      Cl.r[m * nc] = gc * Cl.inv_diag[m * nc];
    }
    return;
  }
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= m * nc) return;
  const int i = gid / nc + 1, J = gid % nc;
  const int j0 = 2 * J, cnt = J == nc - 1 ? nf - j0 : 2;
  // three fine lines at most, all loaded (the third clamped) and masked
  double f = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int j = j0 + min(k, cnt - 1), idx = (i - 1) * nf + j;
    const double g = top ? Fl.diag[idx] * y[idx] : Fl.g[idx];
    const double v = (g - mg_apply(Fl, i, j, inv_dt, th, xv, x0)) / (Fl.inv_rw[i] * Fl.inv_dth[j]);
    f += k < cnt ? v : 0.0;
  }
  const int cidx = (i - 1) * nc + J;
  const double gc = f * (Cl.inv_rw[i] * Cl.inv_dth[J]);
  Cl.g[cidx] = gc;
  Cl.r[cidx] = gc * Cl.inv_diag[cidx];
}

// Bottom: ring totals of level lb's volume-weighted residual (tot[i], the
// origin at tot[0]); one thread per ring (thread 0 of block 0: the origin).
__global__ __launch_bounds__(256) void k_mg_ringtot(const PdScalars *sc, const PdMgLevel *lev, int lb,
                                                    const double *y, const double *z, double *tot) {
  if (!inner_active(sc)) return;
  const PdMgLevel B = lev[lb];
  const double inv_dt = sc->inv_dt, th = sc->theta;
  const bool top = lb == 0;
  const double *xb = top ? z : B.sh;
  const int m = B.m, n = B.n;
  const double x0 = xb[m * n];
  auto xv = [&](int ii, int jj) { return xb[(ii - 1) * n + jj]; };
  auto gv = [&](int idx) { return top ? B.diag[idx] * y[idx] : B.g[idx]; };
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > m) return;
  if (i == 0) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += B.gp_r[j] * x0 - B.gm_r[j] * xv(1, j);
    const double b0 = B.has_b ? B.b_node[m * n] : 0.0;
    const double ax = inv_dt * x0 + th * (B.inv_V0 * s + b0 * x0);
    tot[0] = (gv(m * n) - ax) / B.inv_V0;
    return;
  }
  double f = 0.0;
  for (int j = 0; j < n; ++j)
    f += (gv((i - 1) * n + j) - mg_apply(B, i, j, inv_dt, th, xv, x0)) / (B.inv_rw[i] * B.inv_dth[j]);
  tot[i] = f;
}

// Bottom: the ring-mean system solved for the totals (one block).
__global__ __launch_bounds__(PD_CC_THREADS) void k_mg_solve(const PdScalars *sc, const double *crs, int m,
                                                            const double *tot, double *c) {
  if (!inner_active(sc)) return;
  ring_solve(crs, m, sc->inv_dt, sc->theta, tot[0], tot, c);
}

// Up, level l (nlev coarse levels; below level nlev the ring means c): the
// coarse correction e from level l+1 added to the level's pre-smoothed
// iterate (x_l, stored for l >= 1), and the post-smoothing sweep input
// r = (g - A_l x_l) / diag.  Neighbours' x_l are formed on the fly (no
// thread reads another's store).  The last block takes the origin.
__global__ __launch_bounds__(256) void k_mg_up(const PdScalars *sc, const PdMgLevel *lev, int l, int nlev,
                                               const double *cring, const double *y, const double *z) {
  if (!inner_active(sc)) return;
  const PdMgLevel L = lev[l];
  const bool ring = l == nlev;
  const PdMgLevel E = lev[ring ? l : l + 1];
  const double inv_dt = sc->inv_dt, th = sc->theta;
  const bool top = l == 0;
  const double *base = top ? z : L.sh;
  const int m = L.m, n = L.n, nc = E.n;
  auto ev = [&](int ii, int jj) -> double {   // e at the coarse cell of (ii, jj)
    if (ring) return cring[ii];
    const int c = (ii - 1) * nc + mg_coarse(jj, nc);
    return E.x[c] + E.sh[c];
  };
  const double e0 = ring ? cring[0] : E.x[m * nc] + E.sh[m * nc];
  const double x0 = base[m * n] + e0;
  auto xv = [&](int ii, int jj) { return base[(ii - 1) * n + jj] + ev(ii, jj); };
  if (blockIdx.x == gridDim.x - 1) {
    const double ax = mg_apply_origin(L, inv_dt, th, xv, x0);
    if (threadIdx.x == 0) {
      const int o = m * n;
      const double g = top ? L.diag[o] * y[o] : L.g[o];
      if (!top) L.x[o] = x0;
      L.r[o] = (g - ax) * L.inv_diag[o];
    }
    return;
  }
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= m * n) return;
  const int i = gid / n + 1, j = gid % n;
  const double g = top ? L.diag[gid] * y[gid] : L.g[gid];
  if (!top) L.x[gid] = xv(i, j);
  L.r[gid] = (g - mg_apply(L, i, j, inv_dt, th, xv, x0)) * L.inv_diag[gid];
}

// Level 0's result: z <- z + P e_1 + (its post-smoothing correction).
__global__ __launch_bounds__(256) void k_mg_fin(const PdScalars *sc, const PdMgLevel *lev, int nlev,
                                                const double *cring, double *z) {
  if (!inner_active(sc)) return;
  const PdMgLevel L = lev[0];
  const bool ring = nlev == 0;
  const PdMgLevel E = lev[ring ? 0 : 1];
  const int m = L.m, n = L.n, nc = E.n;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid > m * n) return;
  double e;
  if (gid == m * n) {
    e = ring ? cring[0] : E.x[m * nc] + E.sh[m * nc];
  } else {
    const int i = gid / n + 1, j = gid % n;
    if (ring) {
      e = cring[i];
    } else {
      const int c = (i - 1) * nc + mg_coarse(j, nc);
      e = E.x[c] + E.sh[c];
    }
  }
  z[gid] += e + L.sh[gid];
}

// Origin of a diagnostic operator apply (one thread per instance).
template <typename TK>
__global__ void k_apply_origin(const PdInst *insts, int ninst, double a_dt, double a_th, const TK *ax,
                               TK *ay) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ninst) return;
  const PdInst &I = insts[q];
  double s0 = 0.0;
  for (int b = 0; b < I.nb_sten; ++b) s0 += I.part_a[b];
  const int orig = I.m * I.n;
  ay[orig] = (TK)origin_apply<TK>(I, 1.0 / a_dt, a_th, (double)ax[orig], s0, 1.0);
}

// Origin of the level begin without a Krylov phase (right-hand side only).
__global__ void k_begin_origin(const PdInst *insts, int ninst) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ninst) return;
  const PdInst &I = insts[q];
  double tot[PD_NBEGIN];
#pragma unroll
  for (int k = 0; k < PD_NBEGIN; ++k) tot[k] = 0.0;
#pragma unroll 4
  for (int b = 0; b < I.nb_sten; ++b) {
#pragma unroll
    for (int k = 0; k < PD_NBEGIN; ++k) tot[k] += I.part_b[k * I.nb_sten + b];
  }
  const OriginBegin O = origin_begin(I, I.sc, tot);
  origin_begin_store(I, I.sc, O);
}

// ------------------------------------------------------------ radial sweep
//
// w = (I + D^{-1}R)^{-1} y for every θ-column of an instance.  A block owns
// CW consecutive columns (16, or 8 in the 1024-thread class) and splits every
// column into NT/CW segments: thread t takes column t % CW and segment
// t / CW, so a wave holds 64/CW consecutive segments of the block's columns
// (row pieces of CW values per load).  Every operand of a thread's rows is
// loaded at the start, before the launch's partial sums are read.  Each
// thread runs the forward and backward substitution of its segment in
// registers; the segments' affine maps are joined by a scan over the
// segments of a wave (lane shuffles), then over the waves of the block
// (wave totals through LDS), and each thread corrects its rows.  The origin
// row passes through (unit diagonal).
//
// RM_P:  y = p = r + β (p - ω v)   (p = r on a (re)start; r̂ = r on a restart)
// RM_S:  y = s = r - α v
// RM_Y:  y = r (diagnostic application of the preconditioner; no scalars)

enum { RM_P = 0, RM_S = 1, RM_Y = 2 };

// C: the sweep's arithmetic type, its storage type T (FP64, or FP32 for the
// inner solve of mixed precision).
template <typename C, int BM>
struct RadRegs {
  C a[BM], b[BM];               // P: r, p - ω v   S: r, v
  float u[BM], f[BM], g[BM];    // pivot inverse and multipliers, as stored (converted at use)
};

template <typename T, int MODE, int BM>
__device__ __forceinline__ void rad_load(int n, int j, int rb, int klast, double omega,
                                         const GAS T *__restrict__ a, const GAS T *__restrict__ b,
                                         const GAS T *__restrict__ c,
                                         const GAS float *__restrict__ uinv,
                                         const GAS float *__restrict__ f, RadRegs<T, BM> &R) {
  const T om = (T)omega;
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    // rows past the segment's end repeat its last row (clamped, always issued)
    const int idx = (rb + min(k, klast)) * n + j;
    R.a[k] = a[idx];
    if (MODE == RM_P) R.b[k] = b[idx] - om * c[idx];
    if (MODE == RM_S) R.b[k] = b[idx];
    if (MODE == RM_Y) R.b[k] = (T)0;
    R.u[k] = uinv[idx];
    R.f[k] = f[idx];
  }
}

// The backward multipliers, loaded once the launch's partial sums are read
// (they are first needed after the forward join, and holding them through
// the closure of the p-sweep would cost registers).
template <typename C, int BM>
__device__ __forceinline__ void rad_load_g(int n, int j, int rb, int klast,
                                           const GAS float *__restrict__ g, RadRegs<C, BM> &R) {
#pragma unroll
  for (int k = 0; k < BM; ++k) R.g[k] = g[(rb + min(k, klast)) * n + j];
}

// Joins of the segments of a block's columns (NW waves; a wave holds
// 64/CW consecutive segments of the block's CW columns).  Forward: the value
// entering segment s from above is the composition of the maps of segments
// 0..s-1 applied to 0; backward: of the segments below s.  lane/CW is the
// segment within the wave.
template <typename C, int NW, int CW>
__device__ __forceinline__ C rad_join(AffT<C> A, bool fwd, int c, int lane, int wave,
                                      C (&lp)[NW][CW], C (&le)[NW][CW]) {
  constexpr int SPW = 64 / CW;
  const int sub = lane / CW;
  // inclusive scan over the wave's segments
#pragma unroll
  for (int d = 1; d < SPW; d <<= 1) {
    const AffT<C> o = fwd ? AffT<C>{__shfl_up(A.P, CW * d, 64), __shfl_up(A.e, CW * d, 64)}
                          : AffT<C>{__shfl_down(A.P, CW * d, 64), __shfl_down(A.e, CW * d, 64)};
    if (fwd ? sub >= d : sub + d < SPW) A = compose(A, o);
  }
  // the part of the wave before (forward) or after (backward) the segment
  const AffT<C> ex = fwd ? AffT<C>{__shfl_up(A.P, CW, 64), __shfl_up(A.e, CW, 64)}
                         : AffT<C>{__shfl_down(A.P, CW, 64), __shfl_down(A.e, CW, 64)};
  const bool edge = fwd ? sub == 0 : sub == SPW - 1;
  if (sub == (fwd ? SPW - 1 : 0)) {
    lp[wave][c] = A.P;
    le[wave][c] = A.e;
  }
  __syncthreads();
  C W = (C)0;
  if (fwd) {
    for (int w = 0; w < wave; ++w) W = lp[w][c] * W + le[w][c];
  } else {
    for (int w = NW - 1; w > wave; --w) W = lp[w][c] * W + le[w][c];
  }
  __syncthreads();   // the tables are reused by the next join
  return edge ? W : ex.P * W + ex.e;
}

template <typename T, int MODE, int BM, int NT, int CW>
__device__ __forceinline__ void rad_solve(int m, int n, int j, int c, int i_begin, int cnt,
                                          bool origin_thread, double beta, double omega,
                                          double alpha, bool first, bool reset, RadRegs<T, BM> &R,
                                          const GAS T *__restrict__ r, GAS T *__restrict__ p,
                                          const GAS T *__restrict__ v, GAS T *__restrict__ rh,
                                          GAS T *__restrict__ s, GAS T *__restrict__ out) {
  constexpr int NW = NT / 64;
  __shared__ T lp[NW][CW], le[NW][CW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  // RM_P: b = p - ω v, so that p = r + β b (in T: FP32 for the inner solve)
  const T be = (T)beta, al = (T)alpha;
  auto input = [&](T a, T b) -> T {
    if (MODE == RM_P) return first ? a : a + be * b;
    if (MODE == RM_S) return a - al * b;
    return a;
  };
  if (origin_thread) {
    const int o = m * n;
    if (MODE == RM_P) {
      const T ps = input(r[o], (T)((double)p[o] - omega * (double)v[o]));
      p[o] = ps;
      if (reset) rh[o] = r[o];
      out[o] = ps;
    } else {
      const T ss = input(r[o], v[o]);
      if (MODE == RM_S) s[o] = ss;
      out[o] = ss;
    }
  }

  // right-hand side of the sweep (stored in the Krylov vector it defines),
  // then the local forward pass
  T wl[BM];
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    const T ys = input(R.a[k], R.b[k]);
    if (k < cnt) {
      const int idx = (i_begin + k) * n + j;
      if (MODE == RM_P) {
        p[idx] = ys;
        if (reset) rh[idx] = R.a[k];
      } else if (MODE == RM_S) {
        s[idx] = ys;
      }
    }
    wl[k] = k < cnt ? (T)R.u[k] * ys : (T)0;
    if (k >= cnt) R.f[k] = 0.0f;  // the forward fix-up then leaves such rows alone
  }
  AffT<T> A{(T)1, (T)0};
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    if (k < cnt) {
      A.e = wl[k] - (T)R.f[k] * A.e;
      A.P *= -(T)R.f[k];
      wl[k] = A.e;
    }
  }
  const T Win = rad_join<T, NW, CW>(A, true, c, lane, wave, lp, le);
  T P = (T)1;
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    P *= -(T)R.f[k];
    wl[k] += P * Win;
  }
  AffT<T> Bk{(T)1, (T)0};
#pragma unroll
  for (int k = BM - 1; k >= 0; --k) {
    if (k < cnt) {
      Bk.e = wl[k] - (T)R.g[k] * Bk.e;
      Bk.P *= -(T)R.g[k];
      wl[k] = Bk.e;
    }
  }
  const T Xin = rad_join<T, NW, CW>(Bk, false, c, lane, wave, lp, le);
  T Q = (T)1;
#pragma unroll
  for (int k = BM - 1; k >= 0; --k) {
    if (k < cnt) {
      Q *= -(T)R.g[k];
      out[(i_begin + k) * n + j] = wl[k] + Q * Xin;
    }
  }
}

// NT threads per block of CW columns x NT/CW segments (the three classes of
// rad_class); at most 128 VGPRs, so that two 512-thread blocks share a CU.
template <typename T, int MODE, int BM, int NT, int CW>
__global__ __launch_bounds__(NT, 4) void k_rad(const PdInst *insts, const int2 *map) {
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  PdScalars *sc = I.sc;
  if (!prec_match<T>(I)) return;
  if (block_status(sc) != ST_ACTIVE) return;   // the p- and s-sweeps change the status
  // the descriptor's fields are read before the first store (they then stay
  // scalar; read after a store that may alias them they would be vector
  // loads, and every later store would wait for the wave's memory traffic)
  const KSet<T> KS = kset<T>(I);
  const float *rfu = I.rf_uinv, *rff = I.rf_f, *rfg = I.rf_g;
  const double *part_x = I.part_x, *part_v = I.part_v;
  const int nb_elem = I.nb_elem, nb_sten = I.nb_sten, mixed = I.mixed;
  // the scalars the update closure reads (this launch writes none of them)
  const double sc_omega = sc->omega, sc_alpha = sc->alpha, sc_rho_cur = sc->rho_cur;
  const double sc_tol = sc->tol, sc_bnorm2 = sc->bnorm2;
  const int sc_iters = sc->iters, sc_maxit = sc->maxit, sc_reset = sc->reset_rh;
  constexpr int cw = CW, NSEG = NT / CW;
  const int m = I.m, n = I.n, orig = m * n, B = (m + NSEG - 1) / NSEG;
  const bool b0 = mp.y == 0 && threadIdx.x == 0;
  // this thread's rows: column j, segment seg (threads without rows read row 0)
  const int c = threadIdx.x % cw, seg = threadIdx.x / cw;
  const int j = mp.y * cw + c;
  const bool act = j < n;
  const int cnt = act ? max(0, min(B, m - seg * B)) : 0;
  const int jj = act ? j : 0;
  const int rb = cnt > 0 ? seg * B : 0, klast = cnt > 0 ? cnt - 1 : 0;
  RadRegs<T, BM> R;
  auto load = [&]() {
    const T *a = KS.r;
    const T *bb = (MODE == RM_P) ? KS.p : KS.v;
    rad_load<T, MODE, BM>(n, jj, rb, klast, sc_omega, G(a), G((const T *)bb), G((const T *)KS.v),
                          G(rfu), G(rff), R);
  };
  // the loads are issued before the partial sums are read, except on the
  // rare closures of a level begin or a refinement, whose origin arithmetic
  // would otherwise hold registers together with them
  const int pend = (MODE == RM_P) ? sc->pend : PEND_UPDATE;
  if (pend == PEND_UPDATE) load();
  double beta = 0.0, omega = 0.0, alpha = 0.0;
  bool first = false, reset = false;
  if (MODE == RM_P) {
    // close what the previous launches left: a level begin, a refinement or
    // an update step (ρ = r̂·r, convergence, restart, β)
    int st = ST_ACTIVE;
    double rho = 0.0, rel = -1.0;
    if (pend == PEND_BEGIN) {
      double tot[PD_NBEGIN];
      consume<PD_NBEGIN>(I.part_b, I.nb_sten, tot);
      const OriginBegin O = origin_begin(I, sc, tot);
      if (b0) {
        origin_begin_store(I, sc, O);
        sc->stage = STAGE_ITER;   // the level's factorisation and rhs are done
        sc->bnorm2 = O.bb;
        sc->r0norm2 = O.rr;
        sc->inner_first = 1;
        sc->inner_iters = 0;
        sc->rout0[0] = O.r;
      }
      rho = O.rr;
      first = true;
      rel = O.bb > 0.0 ? sqrt(O.rr / O.bb) : 0.0;
      if (!(O.rr == O.rr) || !(O.bb == O.bb)) st = ST_BREAKDOWN;
      else if (O.rr <= sc->tol * sc->tol * O.bb) st = ST_DONE;
    } else if (pend == PEND_REFINE) {
      double tot[2];
      consume<2>(I.part_ur, I.nb_sten, tot);
      const OriginRefine O = origin_refine(I, sc, tot);
      if (b0) {
        sc->rout0[sc->outer & 1] = O.r;
        I.sol[sol_slot(sc->rot, -1)][orig] += O.d0;
        I.k32.r[orig] = (float)O.rs;
        I.k32.rh[orig] = (float)O.rs;
        sc->r0norm2 = O.rr;
        sc->inner_first = 1;
        sc->inner_iters = 0;
      }
      rho = O.rr;
      first = true;
      rel = sqrt(O.rr / sc->bnorm2);
      if (!(O.rr == O.rr)) st = ST_BREAKDOWN;
      else if (O.rr <= sc->tol * sc->tol * sc->bnorm2) st = ST_DONE;
      else if (sc->outer >= sc->max_outer || sc->iters >= sc->maxit) st = ST_NOCONV;
    } else {
      double tot[2];
      consume<2>(part_x, nb_elem, tot);
      const double rr = tot[1];
      rho = tot[0];
      if (!(rr == rr) || !(rho == rho)) {
        st = ST_BREAKDOWN;
      } else if (!mixed) {
        rel = sqrt(rr / sc_bnorm2);
        if (rr <= sc_tol * sc_tol * sc_bnorm2) st = ST_DONE;
        else if (sc_iters >= sc_maxit) st = ST_NOCONV;
      }
      if (st == ST_ACTIVE) {
        if (sc_reset || fabs(rho) <= 1e-30 * rr) {
          first = true;                  // restart from the iterate: r̂ = r, p = r
          reset = true;
          rho = rr;
          if (b0) sc->restarted = 1;
        } else {
          beta = (rho / sc_rho_cur) * (sc_alpha / sc_omega);
        }
      }
      if (b0) sc->inner_first = 0;
    }
    omega = sc_omega;
    if (b0) {
      sc->rho_next = rho;
      if (rel >= 0.0) sc->rel_resid = rel;
      if (st != ST_ACTIVE) finish_instance(I, sc, st);
    }
    if (st != ST_ACTIVE) return;
  } else if (MODE == RM_S) {
    // α = ρ / (r̂·v), closing the v-stencil with its origin row
    double tot[2];
    consume<2>(part_v, nb_sten, tot);
    const double ph0 = (double)KS.ph[orig];
    const double invd0 = sizeof(T) == 8 ? origin_invd(I, sc->inv_dt, sc->theta) : (double)KS.inv_d[orig];
    const T v0 = (T)origin_apply<T>(I, sc->inv_dt, sc->theta, ph0, tot[1], invd0);
    const double dot = tot[0] + (double)KS.rh[orig] * (double)v0;
    const double rho = sc->rho_next;
    int st = ST_ACTIVE;
    bool brk = false;
    if (!(dot == dot)) {
      st = ST_BREAKDOWN;
    } else if (fabs(dot) <= 1e-300 || fabs(rho) <= 1e-300) {
      alpha = 0.0;                         // restart at the next p-sweep
      brk = true;
    } else {
      alpha = rho / dot;
    }
    if (b0) {
      KS.v[orig] = v0;
      sc->alpha = alpha;
      sc->rho_cur = rho;
      if (brk) sc->reset_rh = 1;
      if (st != ST_ACTIVE) finish_instance(I, sc, st);
    }
    if (st != ST_ACTIVE) return;
  }
  if (pend != PEND_UPDATE) load();
  rad_load_g<T, BM>(n, jj, rb, klast, G(rfg), R);
  rad_solve<T, MODE, BM, NT, CW>(m, n, jj, c, seg * B, cnt, b0, beta, omega, alpha, first, reset, R,
                         G((const T *)KS.r), G(KS.p), G((const T *)KS.v), G(KS.rh), G(KS.s), G(KS.w));
}

// ------------------------------------------------------------ angular sweep
//
// z = (I + D^{-1}Θ)^{-1} w for every ring: one wave per ring, lane L owns
// the bang consecutive nodes j in [L*bang, (L+1)*bang).  The ring's input is
// read with coalesced loads and handed to the owning lanes through LDS (and
// the result back the same way); the factors are stored in the lanes' order
// and read directly.  Local substitution in registers, then the lanes' affine
// maps are composed by a Kogge-Stone scan across the wave (prefix for the
// forward, suffix for the backward substitution), then the Sherman-Morrison
// correction closes the period.  Ring 1's wave then closes the origin row
// of the arrow system (ring 1 with the origin): z_0 = (w_0 - c̃·u)/σ and
// z_1 = u - q z_0, from the vectors and scalar its factorisation stored.
//
// AM_P: input w, output p̂;  AM_S: output ŝ (ring 1's wave also closes the origin).
enum { AM_P = 0, AM_S = 1 };

// Orders the LDS accesses of one wave (its lanes exchange values through LDS).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The sweep computes in its storage type T (FP64, or FP32 for the inner
// solve of mixed precision).
template <typename T, int BM>
__device__ __forceinline__ void ang_body(int m, int n, int B, int i, int lane, double kappa_d,
                                         double alpha0_d, const GAS T *__restrict__ in,
                                         GAS T *__restrict__ out,
                                         const GAS float *__restrict__ uinv,
                                         const GAS float *__restrict__ f,
                                         const GAS float *__restrict__ g,
                                         const GAS float *__restrict__ z,
                                         const GAS float *__restrict__ qa,
                                         const GAS float *__restrict__ ca,
                                         const GAS double *__restrict__ sigma, T *tb,
                                         float *abuf) {
  using C = T;
  const C kappa = (C)kappa_d, alpha0 = (C)alpha0_d;
  const int row = (i - 1) * n, frow = (i - 1) * 64 * B;
  const int j0 = lane * B;
  const int cnt = max(0, min(B, n - j0));
  const bool arrow = i == 1;   // ring 1 closes the origin row (wave-uniform)

  // every load first, issued together (a load under a per-lane condition
  // becomes a branch that waits for it): the ring's input (coalesced, node
  // lane + 64k) and this lane's factors (node j0 + k, stored at 64k + lane)
  C xin[BM], ul[BM], fl[BM], gl[BM], zl[BM];
  const C w0 = (C)in[m * n], sg = (C)sigma[0];
  float aq[BM], ac[BM];   // ring 1: its arrow vectors, parked in LDS (abuf) with the input
#pragma unroll
  for (int k = 0; k < BM; ++k) aq[k] = ac[k] = 0.0f;
  if (arrow) {
#pragma unroll
    for (int k = 0; k < BM; ++k) {
      if (k < B) {
        aq[k] = qa[64 * k + lane];   // in the arrays; entries past the ring end go unused
        ac[k] = ca[64 * k + lane];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    // k >= B (the kernel's span beyond the instance's) rereads the last slots
    const int kk = min(k, B - 1);
    const int jn = min(lane + 64 * kk, n - 1);
    const int fi = frow + 64 * kk + lane;
    const C xv = (C)in[row + jn], uv = (C)uinv[fi], fv = (C)f[fi], gv = (C)g[fi], zv = (C)z[fi];
    const bool in_span = k < B;
    xin[k] = in_span ? xv : (C)0;
    ul[k] = in_span ? uv : (C)0;
    fl[k] = in_span ? fv : (C)0;
    gl[k] = in_span ? gv : (C)0;
    zl[k] = in_span ? zv : (C)0;
  }
  // node j sits at j + j/B in LDS: lane L's nodes are contiguous, one gap after each lane
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    const int j = lane + 64 * k;
    if (k < B && j < n) tb[j + j / B] = xin[k];
    if (arrow) {
      abuf[64 * k + lane] = aq[k];            // read back by this lane only
      abuf[64 * (BM + k) + lane] = ac[k];
    }
  }
  wave_sync();
  C wl[BM];
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    const bool own = k < cnt;
    wl[k] = own ? ul[k] * tb[lane * (B + 1) + k] : (C)0;
    fl[k] = own ? fl[k] : (C)0;
    gl[k] = own ? gl[k] : (C)0;
    zl[k] = own ? zl[k] : (C)0;
  }
  wave_sync();

  AffT<C> A{(C)1, (C)0};
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    if (k < cnt) {
      A.e = wl[k] - fl[k] * A.e;
      A.P *= -fl[k];
      wl[k] = A.e;
    }
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const AffT<C> o{__shfl_up(A.P, d, 64), __shfl_up(A.e, d, 64)};
    if (lane >= d) A = compose(A, o);
  }
  C Win = __shfl_up(A.e, 1, 64);
  if (lane == 0) Win = (C)0;
  C P = (C)1;
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    P *= -fl[k];
    wl[k] += P * Win;
  }
  AffT<C> Bk{(C)1, (C)0};
#pragma unroll
  for (int k = BM - 1; k >= 0; --k) {
    if (k < cnt) {
      Bk.e = wl[k] - gl[k] * Bk.e;
      Bk.P *= -gl[k];
      wl[k] = Bk.e;
    }
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const AffT<C> o{__shfl_down(Bk.P, d, 64), __shfl_down(Bk.e, d, 64)};
    if (lane + d < 64) Bk = compose(Bk, o);
  }
  C Xin = __shfl_down(Bk.e, 1, 64);
  if (lane == 63) Xin = (C)0;
  C Q = (C)1, ylast = (C)0;
#pragma unroll
  for (int k = BM - 1; k >= 0; --k) {
    if (k < cnt) {
      Q *= -gl[k];
      wl[k] += Q * Xin;
      if (j0 + k == n - 1) ylast = wl[k];
    }
  }
  const C y0 = __shfl(wl[0], 0, 64);
  const C yl = __shfl(ylast, (n - 1) / B, 64);
  const C sfac = kappa * (y0 - alpha0 * yl);
#pragma unroll
  for (int k = 0; k < BM; ++k) wl[k] -= sfac * zl[k];
  if (arrow) {
    // z_0 = (w_0 - c̃·u)/σ, z_1 = u - q z_0 (fixed-order wave sum)
    C dot = (C)0;
#pragma unroll
    for (int k = 0; k < BM; ++k)
      if (k < cnt) dot += (C)abuf[64 * (BM + k) + lane] * wl[k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) dot += __shfl_xor(dot, d, 64);
    const C z0 = (w0 - dot) / sg;
#pragma unroll
    for (int k = 0; k < BM; ++k)
      if (k < cnt) wl[k] -= (C)abuf[64 * k + lane] * z0;
    if (lane == 0) out[m * n] = (T)z0;
  }
  // back to node order through LDS, then coalesced stores
#pragma unroll
  for (int k = 0; k < BM; ++k)
    if (k < cnt) tb[lane * (B + 1) + k] = wl[k];
  wave_sync();
#pragma unroll
  for (int k = 0; k < BM; ++k) {
    const int j = lane + 64 * k;
    if (k < B && j < n) out[row + j] = (T)tb[j + j / B];
  }
}

template <typename T, int MODE, int BM>
__global__ __launch_bounds__(256) void k_ang(const PdInst *insts, const int2 *map) {
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  PdScalars *sc = I.sc;
  if (!inner_active(sc) || !prec_match<T>(I)) return;
  // the descriptor is read before the first store (read after a store that
  // may alias it, its fields would be vector loads that later stores wait on)
  const KSet<T> KS = kset<T>(I);
  const int m = I.m, n = I.n, B = I.bang;
  const int lane = threadIdx.x & 63;
  const int i = mp.y * 4 + (threadIdx.x >> 6) + 1;
  const int ic = i <= m ? i : 1;
  const double kappa = I.af_kappa[ic - 1], alpha0 = I.af_alpha0[ic - 1];
  const float *fu = I.af_uinv, *ff = I.af_f, *fg = I.af_g, *fz = I.af_z, *fq = I.af_q, *fc = I.af_c;
  const double *sig = I.af_sigma;
  // the p-sweep before this launch consumed the restart flag and the
  // pending closure; only this block's thread 0 touches these fields here
  if (MODE == AM_P && mp.y == 0 && threadIdx.x == 0) {
    if (sc->restarted) {
      sc->restarts += 1;
      sc->restarted = 0;
    }
    sc->reset_rh = 0;
    sc->pend = PEND_UPDATE;
  }
  if (i > m) return;                                 // whole wave exits together
  __shared__ T tbuf[4][64 * (BM + 1)];               // one exchange buffer per wave
  __shared__ float abuf[2 * 64 * BM];                // ring 1's arrow vectors (its wave only)
  const T *in = KS.w;
  T *out = (MODE == AM_P) ? KS.ph : KS.sh;
  ang_body<T, BM>(m, n, B, i, lane, kappa, alpha0, G(in), G(out), G(fu), G(ff), G(fg), G(fz), G(fq),
                  G(fc), G(sig), tbuf[threadIdx.x >> 6], abuf);
}

// Ring sweep of rings with more than 1024 nodes: aw = 4 waves per ring (the
// kernel also takes aw = 2).
// Each of the ring's 64*aw threads owns the 8 consecutive nodes 8t..8t+7
// (factors stored thread-major, afac_index).  The segments' affine maps are
// scanned over the lanes of each wave, then joined across the ring's waves
// through LDS (forward: the waves before, backward: the waves after); the
// Sherman-Morrison closure reads the ring's first and last values from LDS,
// and ring 1's arrow closure sums its dot product over the waves in a fixed
// order.  A block of 256 threads holds 4/aw rings; every thread reaches
// every barrier (rings past m only skip their memory accesses).
template <typename T, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_angw(const PdInst *insts, const int2 *map) {
  using C = T;
  constexpr int BW = 8;                          // nodes per thread
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  PdScalars *sc = I.sc;
  if (!inner_active(sc) || !prec_match<T>(I)) return;   // the same for the whole block
  // every field of the descriptor is read before the first store, so that
  // the reads stay scalar: a read after a store that may alias it becomes a
  // vector load, and each later store would then wait for all memory
  // traffic of the wave
  const KSet<T> KS = kset<T>(I);
  const int m = I.m, n = I.n, aw = I.aw, B = I.bang;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rpb = 4 / aw;
  const int slot = wv / aw, wr = wv % aw;        // ring of the block, wave of the ring
  const int nt = 64 * aw, t = wr * 64 + lane;    // threads of a ring, this thread
  const int i = mp.y * rpb + slot + 1;
  const bool on = i <= m;
  const int ic = on ? i : 1;                     // rings past m read ring 1's data (unused)
  const double kappa_d = I.af_kappa[ic - 1], alpha0_d = I.af_alpha0[ic - 1];
  const double sigma_d = I.af_sigma[0];
  const GAS T *in = G((const T *)KS.w);
  GAS T *out = G(MODE == AM_P ? KS.ph : KS.sh);
  const GAS float *uinv = G((const float *)I.af_uinv), *f = G((const float *)I.af_f);
  const GAS float *g = G((const float *)I.af_g), *z = G((const float *)I.af_z);
  const GAS float *aq = G((const float *)I.af_q), *ac = G((const float *)I.af_c);
  // the p-sweep before this launch consumed the restart flag and the
  // pending closure; only this block's thread 0 touches these fields here
  if (MODE == AM_P && mp.y == 0 && threadIdx.x == 0) {
    if (sc->restarted) {
      sc->restarts += 1;
      sc->restarted = 0;
    }
    sc->reset_rh = 0;
    sc->pend = PEND_UPDATE;
  }
  __shared__ C tb[2304];                         // node order, one gap after every 8 nodes
  __shared__ C fP[4], fE[4], bP[4], bE[4];       // wave totals of the forward and backward maps
  __shared__ C ends[4][2];                       // per ring: first and last value
  __shared__ C dsum[4];                          // per wave: ring 1's arrow dot product
  C *rbuf = tb + slot * 576 * aw;
  const int row = (ic - 1) * n, frow = (ic - 1) * 64 * B;
  const int j0 = BW * t;
  const int cnt = on ? max(0, min(BW, n - j0)) : 0;
  const bool arrow = on && i == 1;

  // every load first, all of them issued (indexes clamped into the ring,
  // values masked afterwards: a load under a per-lane condition becomes a
  // branch that waits for it): the ring's input (coalesced, node t + nt k)
  // and this thread's factors (node 8t + k at k nt + t)
  C xin[BW];
  float ul[BW], fl[BW], gl[BW], zl[BW];   // factors as stored, converted at use
  const C w0 = (C)in[m * n], sg = (C)sigma_d;
#pragma unroll
  for (int k = 0; k < BW; ++k) {
    const int jn = t + nt * k;
    const bool own = k < cnt;                   // implies on
    const int fi = frow + min(k * nt + t, 64 * B - 1);
    const C xv = (C)in[row + min(jn, n - 1)];
    const float uv = uinv[fi], fv = f[fi], gv = g[fi], zv = z[fi];
    xin[k] = jn < n ? xv : (C)0;   // rings past m hold ring 1's values, never stored
    ul[k] = own ? uv : 0.0f;
    fl[k] = own ? fv : 0.0f;
    gl[k] = own ? gv : 0.0f;
    zl[k] = own ? zv : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < BW; ++k) {
    const int jn = t + nt * k;
    if (on && jn < n) rbuf[jn + jn / BW] = xin[k];
  }
  __syncthreads();
  C wl[BW];
#pragma unroll
  for (int k = 0; k < BW; ++k) {
    const C v = rbuf[j0 + k + t];   // in the buffer for every thread; unset past the ring's end
    wl[k] = k < cnt ? (C)ul[k] * v : (C)0;
  }
  __syncthreads();   // the buffer is rewritten with the result

  // forward substitution: local, over the wave, over the ring's earlier waves
  AffT<C> A{(C)1, (C)0};
#pragma unroll
  for (int k = 0; k < BW; ++k) {
    if (k < cnt) {
      A.e = wl[k] - (C)fl[k] * A.e;
      A.P *= -(C)fl[k];
      wl[k] = A.e;
    }
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const AffT<C> o{__shfl_up(A.P, d, 64), __shfl_up(A.e, d, 64)};
    if (lane >= d) A = compose(A, o);
  }
  AffT<C> X{__shfl_up(A.P, 1, 64), __shfl_up(A.e, 1, 64)};
  if (lane == 0) X = AffT<C>{(C)1, (C)0};
  if (lane == 63) {
    fP[wv] = A.P;
    fE[wv] = A.e;
  }
  __syncthreads();
  C E = (C)0;
  for (int w = 0; w < wr; ++w) E = fP[slot * aw + w] * E + fE[slot * aw + w];
  const C Win = X.P * E + X.e;
  C P = (C)1;
#pragma unroll
  for (int k = 0; k < BW; ++k) {
    P *= -(C)fl[k];
    wl[k] += P * Win;
  }
  // backward substitution: local, over the wave, over the ring's later waves
  AffT<C> Bk{(C)1, (C)0};
#pragma unroll
  for (int k = BW - 1; k >= 0; --k) {
    if (k < cnt) {
      Bk.e = wl[k] - (C)gl[k] * Bk.e;
      Bk.P *= -(C)gl[k];
      wl[k] = Bk.e;
    }
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const AffT<C> o{__shfl_down(Bk.P, d, 64), __shfl_down(Bk.e, d, 64)};
    if (lane + d < 64) Bk = compose(Bk, o);
  }
  AffT<C> Y{__shfl_down(Bk.P, 1, 64), __shfl_down(Bk.e, 1, 64)};
  if (lane == 63) Y = AffT<C>{(C)1, (C)0};
  if (lane == 0) {
    bP[wv] = Bk.P;
    bE[wv] = Bk.e;
  }
  __syncthreads();
  C F = (C)0;
  for (int w = aw - 1; w > wr; --w) F = bP[slot * aw + w] * F + bE[slot * aw + w];
  const C Xin = Y.P * F + Y.e;
  C Q = (C)1, ylast = (C)0;
#pragma unroll
  for (int k = BW - 1; k >= 0; --k) {
    if (k < cnt) {
      Q *= -(C)gl[k];
      wl[k] += Q * Xin;
      if (j0 + k == n - 1) ylast = wl[k];
    }
  }
  // ring 1 closes the origin row: z_0 = (w_0 - c.u)/σ, z_1 = u - q z_0 (only
  // the block holding ring 1 takes this branch and its barrier; its arrow
  // vectors are loaded here, before the Sherman-Morrison barrier, all
  // issued: frow = 0 for ring 1)
  float cq[BW], qq[BW];
  if (mp.y == 0) {
#pragma unroll
    for (int k = 0; k < BW; ++k) {
      const int ai = min(k * nt + t, 64 * B - 1);
      cq[k] = ac[ai];
      qq[k] = aq[ai];
    }
  }
  // Sherman-Morrison closure of the period
  if (on && t == 0) ends[slot][0] = wl[0];
  if (on && t == (n - 1) / BW) ends[slot][1] = ylast;
  __syncthreads();
  if (on) {
    const C kappa = (C)kappa_d, alpha0 = (C)alpha0_d;
    const C sfac = kappa * (ends[slot][0] - alpha0 * ends[slot][1]);
#pragma unroll
    for (int k = 0; k < BW; ++k) wl[k] -= sfac * (C)zl[k];
  }
  if (mp.y == 0) {
    C dot = (C)0;
#pragma unroll
    for (int k = 0; k < BW; ++k)
      if (arrow && k < cnt) dot += (C)cq[k] * wl[k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) dot += __shfl_xor(dot, d, 64);
    if (lane == 0) dsum[wv] = dot;
    __syncthreads();
    if (arrow) {
      C tot = (C)0;
      for (int w = 0; w < aw; ++w) tot += dsum[slot * aw + w];
      const C z0 = (w0 - tot) / sg;
#pragma unroll
      for (int k = 0; k < BW; ++k)
        if (k < cnt) wl[k] -= (C)qq[k] * z0;
      if (t == 0) out[m * n] = (T)z0;
    }
  }
  // back to node order through LDS, then coalesced stores
#pragma unroll
  for (int k = 0; k < BW; ++k)
    if (k < cnt) rbuf[j0 + k + t] = wl[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < BW; ++k) {
    const int jn = t + nt * k;
    if (on && jn < n) out[row + jn] = (T)rbuf[jn + jn / BW];
  }
}

// ------------------------------------------------------------ update kernel
//
// x += α p̂ + ω ŝ (x = ... on the first inner iteration of a refinement),
// r = s - ω t, partials r̂·r and r·r; the last block decides convergence,
// breakdown or restart for the instance.

template <int E>
struct ElemRegs {
  double ph[E], sh[E], s[E], t[E], rh[E], x[E];
};

// Every operand of the thread's E unknowns (clamped indices: every load is
// issued unconditionally, tails masked later).
template <typename T, int E>
__device__ __forceinline__ void elem_load(int N, int base, const GAS T *__restrict__ ph,
                                          const GAS T *__restrict__ sh, const GAS T *__restrict__ s,
                                          const GAS T *__restrict__ t, const GAS T *__restrict__ rh,
                                          const GAS T *__restrict__ x, ElemRegs<E> &R) {
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int idx = base + k * 256 + threadIdx.x;
    const int li = idx < N ? idx : N - 1;
    R.ph[k] = (double)ph[li];
    R.sh[k] = (double)sh[li];
    R.s[k] = (double)s[li];
    R.t[k] = (double)t[li];
    R.rh[k] = (double)rh[li];
    R.x[k] = (double)x[li];
  }
}

template <typename T, int E>
__device__ __forceinline__ void elem_update(int N, int base, double al, double om, bool setx,
                                            int orig, double t0, const ElemRegs<E> &R,
                                            GAS T *__restrict__ x, GAS T *__restrict__ r,
                                            double (&acc)[2]) {
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int idx = base + k * 256 + threadIdx.x;
    const double tv = (idx == orig) ? t0 : R.t[k];
    const double xv = setx ? 0.0 : R.x[k];
    const T xs = (T)(xv + al * R.ph[k] + om * R.sh[k]);
    const T rs = (T)(R.s[k] - om * tv);
    const double rd = (double)rs;
    if (idx < N) {
      x[idx] = xs;
      r[idx] = rs;
      acc[0] += R.rh[k] * rd;
      acc[1] += rd * rd;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_elem_x(const PdInst *insts, const int2 *map) {
  constexpr int E = PD_ELEM_PER_BLOCK / 256;
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  PdScalars *sc = I.sc;
  if (!prec_match<T>(I)) return;
  if (block_status(sc) != ST_ACTIVE) return;   // this kernel changes the status
  // the descriptor's fields and the scalars are read before the first store
  // (read after it they would be vector loads that every later store waits on)
  const KSet<T> KS = kset<T>(I);
  const int orig = I.m * I.n;
  const bool b0 = mp.y == 0 && threadIdx.x == 0;
  T *x = iterate_ptr<T>(I, sc);
  double *part_x = I.part_x;
  const int nb_elem = I.nb_elem;
  const double sc_alpha = sc->alpha;
  const bool setx = I.mixed && sc->inner_first != 0;
  const int base = mp.y * 256 * E;
  // the vectors first, then the partial sums of the t-stencil
  ElemRegs<E> R;
  elem_load<T, E>(orig + 1, base, G((const T *)KS.ph), G((const T *)KS.sh), G((const T *)KS.s),
                  G((const T *)KS.t), G((const T *)KS.rh), G((const T *)x), R);
  // ω = (t·s)/(t·t), closing the t-stencil with its origin row
  double tot[3];
  consume<3>(I.part_t, I.nb_sten, tot);
  const double invd0 = sizeof(T) == 8 ? origin_invd(I, sc->inv_dt, sc->theta) : (double)KS.inv_d[orig];
  const T t0 = (T)origin_apply<T>(I, sc->inv_dt, sc->theta, (double)KS.sh[orig], tot[2], invd0);
  const double s0 = (double)KS.s[orig];
  const double ts = tot[0] + s0 * (double)t0, tt = tot[1] + (double)t0 * (double)t0;
  double om = 0.0;
  int st = ST_ACTIVE;
  bool brk = false;
  if (!(ts == ts) || !(tt == tt)) {
    st = ST_BREAKDOWN;
  } else if (tt <= 1e-300) {
    brk = true;                           // x += α p̂ only; restart at the next p-sweep
  } else {
    om = ts / tt;
  }
  if (b0) {
    sc->omega = om;
    sc->iters += 1;
    sc->inner_iters += 1;
    if (brk) sc->reset_rh = 1;
    if (st != ST_ACTIVE) finish_instance(I, sc, st);
  }
  if (st != ST_ACTIVE) return;
  double acc[2] = {0.0, 0.0};
  elem_update<T, E>(orig + 1, base, sc_alpha, om, setx, orig, (double)t0, R, G(x), G(KS.r), acc);
  produce<2>(acc, part_x, nb_elem, mp.y);
}

// ------------------------------------------------------------ adaptivity
//
// Error indicator and state transfer between meshes (the paper ties its
// adaptivity to the exponent p of the stretch (2.4), α = pσ of Theorem 2.1,
// and leaves the indicator open).  Indicator at ring node (i, j) from the
// second divided differences on the non-uniform mesh:
//   δ_r² n = 2[(n_{i+1,j} - n_{i,j})/h_{i+1} - (n_{i,j} - n_{i-1,j})/h_i]/(h_i + h_{i+1})
//   δ_θ² n = 2[(n_{i,j+1} - n_{i,j})/μ_{j+1} - (n_{i,j} - n_{i,j-1})/μ_j]/(μ_j + μ_{j+1})
// with ring 0 the origin, ring m+1 the Dirichlet value N(t, θ_j) (zero flux:
// ring m repeated) and j periodic;
//   η = max(ĥ_i² |δ_r² n|, Δθ_j² |δ_θ² n|),  ĥ_i = (h_i + h_{i+1})/2,  Δθ_j = (μ_j + μ_{j+1})/2.
// One wave per ring; per ring: κ_i = max_j |δ_r² n|, max_j η (first j of
// the maximum) and Σ_j η, summed in a fixed order.

__device__ __forceinline__ double boundary_value(const double *nb, const double *lam, const int *tpow,
                                                 int nsrc, int n, int j, double t) {
  double v = 0.0;
  for (int q = 0; q < nsrc; ++q) v += tau_q(lam[q], tpow[q], t) * nb[q * n + j];
  return v;
}

__global__ __launch_bounds__(256) void k_indicator(const double *__restrict__ x, int m, int n,
                                                   const double *__restrict__ r,
                                                   const double *__restrict__ th,
                                                   const double *nb, const double *lam,
                                                   const int *tpow, int nsrc, double t, int dirichlet,
                                                   double *__restrict__ ring_out,
                                                   double *__restrict__ eta_out) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6) + 1;
  if (i > m) return;                                   // whole wave exits together
  const double hi = r[i] - r[i - 1], ho = r[i + 1] - r[i];
  const double hloc = 0.5 * (hi + ho);
  const double x0 = x[m * n];
  double kap = 0.0, emax = -1.0, esum = 0.0;
  int jmax = 0;
  for (int j = lane; j < n; j += 64) {
    const double c = x[(i - 1) * n + j];
    const double below = (i == 1) ? x0 : x[(i - 2) * n + j];
    double above;
    if (i < m) above = x[i * n + j];
    else above = dirichlet ? boundary_value(nb, lam, tpow, nsrc, n, j, t) : c;
    const double d2r = 2.0 * ((above - c) / ho - (c - below) / hi) / (hi + ho);
    const int jl = (j == 0) ? n - 1 : j - 1, jr = (j == n - 1) ? 0 : j + 1;
    const double mu_j = (j == 0) ? th[n] - th[n - 1] : th[j] - th[j - 1];   // μ_0 = μ_n
    const double mu_j1 = th[j + 1] - th[j];
    const double left = x[(i - 1) * n + jl], right = x[(i - 1) * n + jr];
    const double d2t = 2.0 * ((right - c) / mu_j1 - (c - left) / mu_j) / (mu_j + mu_j1);
    const double dth = 0.5 * (mu_j + mu_j1);
    const double e = fmax(hloc * hloc * fabs(d2r), dth * dth * fabs(d2t));
    if (eta_out) eta_out[(i - 1) * n + j] = e;
    kap = fmax(kap, fabs(d2r));
    if (e > emax) {
      emax = e;
      jmax = j;
    }
    esum += e;
  }
  // wave reductions: max with the first index of the maximum, fixed-order sum
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    kap = fmax(kap, __shfl_xor(kap, o, 64));
    const double eo = __shfl_xor(emax, o, 64);
    const int jo = __shfl_xor(jmax, o, 64);
    if (eo > emax || (eo == emax && jo < jmax)) {
      emax = eo;
      jmax = jo;
    }
  }
  esum = wave_sum(esum);
  if (lane == 0) {
    ring_out[4 * (i - 1) + 0] = kap;
    ring_out[4 * (i - 1) + 1] = emax;
    ring_out[4 * (i - 1) + 2] = (double)jmax;
    ring_out[4 * (i - 1) + 3] = esum;
  }
}

// Cubic Lagrange polynomial through (xs[a], ys[a]), a = 0..3, at x.
__device__ __forceinline__ double lagrange4(const double (&xs)[4], const double (&ys)[4], double x) {
  double total = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double w = 1.0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (b != a) w *= (x - xs[b]) / (xs[a] - xs[b]);
    total += w * ys[a];
  }
  return total;
}

// First of the four consecutive entries of nodes[0..cnt) whose middle
// interval holds v (shifted inwards at the ends); nodes increasing.
__device__ __forceinline__ int window4(const double *nodes, int cnt, double v) {
  int lo = 0, hi = cnt - 1;               // last k with nodes[k] <= v, clamped to [0, cnt-2]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (nodes[mid] <= v) lo = mid;
    else hi = mid;
  }
  int k = (v >= nodes[cnt - 1]) ? cnt - 2 : lo;
  k = min(max(k, 0), cnt - 2);
  return min(max(k - 1, 0), cnt - 4);
}

// State transfer: tensor cubic Lagrange, radial along each old θ-line on
// the nodes 0 (origin value), r_1..r_m and, for Dirichlet data, 1 (boundary
// value), then periodic in θ.  One thread per target ring node; the origin
// value is kept.
__global__ __launch_bounds__(256) void k_transfer(const double *__restrict__ x, int m, int n,
                                                  const double *__restrict__ r,
                                                  const double *__restrict__ th,
                                                  const double *nb, const double *lam,
                                                  const int *tpow, int nsrc, double t, int dirichlet,
                                                  const double *__restrict__ r2,
                                                  const double *__restrict__ th2, int m2, int n2,
                                                  double *__restrict__ y) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id == 0) y[m2 * n2] = x[m * n];
  if (id >= m2 * n2) return;
  const int i2 = id / n2 + 1, j2 = id % n2;
  const double rq = r2[i2], tq = th2[j2];
  const int cnt = dirichlet ? m + 2 : m + 1;           // radial nodes r_0..r_{m(+1)}
  const int k = window4(r, cnt, rq);
  double rs[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) rs[a] = r[k + a];
  // the old node at or before tq: the last j with th[j] <= tq among 0..n-1
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (th[mid] <= tq) lo = mid;
    else hi = mid;
  }
  const int jb = lo;
  double ts[4], col[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int jj = jb - 1 + s;
    const int wrap = (jj < 0) ? -1 : (jj >= n ? 1 : 0);
    const int j = jj - wrap * n;
    ts[s] = th[j] + 2.0 * 3.14159265358979323846 * wrap;
    double ys[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int ii = k + a;                            // radial node index
      double v;
      if (ii == 0) v = x[m * n];
      else if (ii <= m) v = x[(ii - 1) * n + j];
      else v = boundary_value(nb, lam, tpow, nsrc, n, j, t);
      ys[a] = v;
    }
    col[s] = lagrange4(rs, ys, rq);
  }
  y[(i2 - 1) * n2 + j2] = lagrange4(ts, col, tq);
}

}  // namespace pd

// ------------------------------------------------------------ launchers

#include "pd_launch.h"

namespace pd {

KTimer *g_timer = nullptr;

static inline dim3 g1(int n) { return dim3((unsigned)n); }

// Launches a kernel; while kernel timing is on, through hipExtLaunchKernel
// with a pair of events that the dispatch itself stamps.
template <typename... KArgs, typename... Args>
static inline void go(int fam, void (*k)(KArgs...), dim3 grid, dim3 block, hipStream_t s,
                      Args... args) {
  hipEvent_t a, b;
  if (g_timer && g_timer->pair(fam, &a, &b))
    hipExtLaunchKernelGGL(k, grid, block, 0, s, a, b, 0, args...);
  else
    k<<<grid, block, 0, s>>>(args...);
}
enum { KF_BEGIN = 0, KF_FACTOR = 1, KF_RAD_P = 2, KF_ANG_P = 3, KF_STEN_V = 4, KF_RAD_S = 5,
       KF_ANG_S = 6, KF_STEN_T = 7, KF_UPDATE = 8, KF_REFINE = 9, KF_CONTROL = 10, KF_LEVEL_END = 11,
       KF_MG = 12 };

void launch_level_begin(const LaunchSet &L, hipStream_t s) {
  go(KF_CONTROL, k_level_begin, dim3((L.ninst + 63) / 64), dim3(64), s, L.insts, L.ninst);
}
void launch_ctl(const LaunchSet &L, hipStream_t s) {
  go(KF_CONTROL, k_ctl, dim3((L.ninst + 63) / 64), dim3(64), s, L.insts, L.ninst);
}
// Register-array length of the segmented sweeps: the smallest of 4, 8, 16,
// 32 that holds the longest segment of the batch.
static inline int seg_len(int b) { return b <= 4 ? 4 : (b <= 8 ? 8 : (b <= 16 ? 16 : 32)); }

#define PD_DISPATCH_BM(b, CALL)          \
  switch (seg_len(b)) {                  \
    case 4: { constexpr int BM = 4; CALL; } break;   \
    case 8: { constexpr int BM = 8; CALL; } break;   \
    case 16: { constexpr int BM = 16; CALL; } break; \
    default: { constexpr int BM = 32; CALL; } break; \
  }

void launch_factor(const LaunchSet &L, hipStream_t s) {
  if (L.nb_rad)
    PD_DISPATCH_BM(L.max_bfrad, (go(KF_FACTOR, k_fact_rad<BM>, g1(L.nb_rad), dim3(PD_RAD_THREADS), s, L.insts, L.map_rad)));
  if (L.nb_ang)
    PD_DISPATCH_BM(L.max_bang, (go(KF_FACTOR, k_fact_ang<BM>, g1(L.nb_ang), dim3(256), s, L.insts, L.map_ang)));
  // the coarse levels of a multigrid preconditioner factor their own lines
  // (gated, like the instance's, on the instance starting a level)
  for (int q = 0; q < L.nmg; ++q)
    for (int l = 1; l <= L.mg[q]->nlev; ++l) launch_factor(L.mg[q]->lev[l], s);
}
void launch_begin(const LaunchSet &L, hipStream_t s) {
  go(KF_BEGIN, k_sten<double, SM_GRAM>, g1(L.nb_sten), dim3(256), s, L.insts, L.map_sten, 0.0, 0.0,
     (const double *)nullptr, (double *)nullptr);
  go(KF_BEGIN, k_gram_total, dim3(L.ninst * PD_NGRAM), dim3(256), s, L.insts, L.ninst);
  go(KF_BEGIN, k_sten<double, SM_BEGIN>, g1(L.nb_sten), dim3(256), s, L.insts, L.map_sten, 0.0, 0.0,
     (const double *)nullptr, (double *)nullptr);
}

template <typename T, int MODE>
static void rad(const LaunchSet &L, hipStream_t s, int fam_as = -1) {
  const int fam = fam_as >= 0 ? fam_as : (MODE == RM_S ? KF_RAD_S : (MODE == RM_P ? KF_RAD_P : KF_CONTROL));
  if (L.nb_rs[0]) {
    PD_DISPATCH_BM(L.max_brs[0], (go(fam, k_rad<T, MODE, BM, 512, 16>, g1(L.nb_rs[0]), dim3(512), s, L.insts, L.map_rs[0])));
  }
  if (L.nb_rs[1]) {
    PD_DISPATCH_BM(L.max_brs[1], (go(fam, k_rad<T, MODE, BM, 1024, 16>, g1(L.nb_rs[1]), dim3(1024), s, L.insts, L.map_rs[1])));
  }
  if (L.nb_rs[2]) {
    PD_DISPATCH_BM(L.max_brs[2], (go(fam, k_rad<T, MODE, BM, 1024, 8>, g1(L.nb_rs[2]), dim3(1024), s, L.insts, L.map_rs[2])));
  }
}
template <typename T, int MODE>
static void ang(const LaunchSet &L, hipStream_t s, int fam_as = -1) {
  const int fam = fam_as >= 0 ? fam_as : (MODE == AM_S ? KF_ANG_S : KF_ANG_P);
  if (L.nb_angs[0])
    PD_DISPATCH_BM(L.max_bang1, (go(fam, k_ang<T, MODE, BM>, g1(L.nb_angs[0]), dim3(256), s, L.insts, L.map_angs[0])));
  if (L.nb_angs[1]) go(fam, k_angw<T, MODE>, g1(L.nb_angs[1]), dim3(256), s, L.insts, L.map_angs[1]);
}
template <typename T, int MODE>
static void sten(int fam, const LaunchSet &L, hipStream_t s) {
  go(fam, k_sten<T, MODE>, g1(L.nb_sten), dim3(256), s, L.insts, L.map_sten, 0.0, 0.0,
     (const T *)nullptr, (T *)nullptr);
}

// The rest of a V-cycle once level 0 holds z = M^{-1} y (the multigrid
// kernels' comment): down through the coarse levels, the ring means, up.
static void mg_vcycle(const MgSet &M, const double *y, double *z, hipStream_t s) {
  const int L = M.nlev, m = M.m;
  const PdMgLevel *dl = M.dlev;
  auto blocks = [&](int l) { return g1((m * M.n[l] + 255) / 256 + 1); };   // + the origin's block
  for (int l = 1; l <= L; ++l) {
    go(KF_MG, k_mg_down, blocks(l), dim3(256), s, M.sc, dl, l, y, (const double *)z);
    rad<double, RM_Y>(M.lev[l], s, KF_MG);
    ang<double, AM_S>(M.lev[l], s, KF_MG);
  }
  go(KF_MG, k_mg_ringtot, g1((m + 1 + 255) / 256), dim3(256), s, M.sc, dl, L, y, (const double *)z, M.btot);
  go(KF_MG, k_mg_solve, g1(1), dim3(PD_CC_THREADS), s, M.sc, M.crs, m, (const double *)M.btot, M.cring);
  for (int l = L; l >= 0; --l) {
    go(KF_MG, k_mg_up, blocks(l), dim3(256), s, M.sc, dl, l, L, (const double *)M.cring, y, (const double *)z);
    rad<double, RM_Y>(M.lev[l], s, KF_MG);
    ang<double, AM_S>(M.lev[l], s, KF_MG);
  }
  go(KF_MG, k_mg_fin, g1((m * M.n[0] + 1 + 255) / 256), dim3(256), s, M.sc, dl, L, (const double *)M.cring, z);
}

// A Krylov iteration of an FP64 batch in which some instances use the
// V-cycle: the batch's sweeps give their level 0's pre-smoothing (and are
// the whole preconditioner of the others), each V-cycle the rest.
static void cycle_mg(const LaunchSet &L, hipStream_t s) {
  rad<double, RM_P>(L, s);
  ang<double, AM_P>(L, s);
  for (int q = 0; q < L.nmg; ++q) mg_vcycle(*L.mg[q], L.mg[q]->p, L.mg[q]->ph, s);
  sten<double, SM_V>(KF_STEN_V, L, s);
  rad<double, RM_S>(L, s);
  ang<double, AM_S>(L, s);
  for (int q = 0; q < L.nmg; ++q) mg_vcycle(*L.mg[q], L.mg[q]->s, L.mg[q]->sh, s);
  sten<double, SM_T>(KF_STEN_T, L, s);
  go(KF_UPDATE, k_elem_x<double>, g1(L.nb_elem), dim3(256), s, L.insts, L.map_elem);
}

template <typename T>
static void cycle_t(const LaunchSet &L, hipStream_t s) {
  rad<T, RM_P>(L, s);
  ang<T, AM_P>(L, s);
  sten<T, SM_V>(KF_STEN_V, L, s);
  rad<T, RM_S>(L, s);
  ang<T, AM_S>(L, s);
  sten<T, SM_T>(KF_STEN_T, L, s);
  go(KF_UPDATE, k_elem_x<T>, g1(L.nb_elem), dim3(256), s, L.insts, L.map_elem);
}

// One round of asynchronous levels: the ring-mean correction of the levels
// that have just converged, level control (an instance whose level ended
// starts its next one), the factorisations and right-hand sides of the
// instances starting a level, then `cycles` Krylov iterations of every
// active instance.
void launch_level_end(const LaunchSet &L, hipStream_t s) {
  go(KF_LEVEL_END, k_sten<double, SM_RES>, g1(L.nb_sten), dim3(256), s, L.insts, L.map_sten, 0.0, 0.0,
     (const double *)nullptr, (double *)nullptr);
  go(KF_LEVEL_END, k_ring_total, g1(L.nb_ang), dim3(256), s, (const PdInst *)L.insts,
     (const int2 *)L.map_ang);
  go(KF_LEVEL_END, k_coarse, g1(L.ninst), dim3(PD_CC_THREADS), s, (const PdInst *)L.insts);
  go(KF_LEVEL_END, k_cadd, g1(L.nb_elem), dim3(256), s, (const PdInst *)L.insts, (const int2 *)L.map_elem);
}

void launch_round(const LaunchSet &L, int cycles, hipStream_t s) {
  launch_level_end(L, s);
  if (L.adaptive_any)
    go(KF_CONTROL, k_sten<double, SM_EST>, g1(L.nb_sten), dim3(256), s, L.insts, L.map_sten, 0.0, 0.0,
       (const double *)nullptr, (double *)nullptr);
  launch_ctl(L, s);
  launch_factor(L, s);
  launch_begin(L, s);
  for (int c = 0; c < cycles; ++c) launch_cycle(L, s);
}

// z = M^{-1} y of the preconditioner (diagnostic): y in the Krylov set's r,
// the radial sweep into w, the ring sweep (with the origin's arrow closure)
// into p̂.
void launch_precond_apply(const LaunchSet &L, int fp32, hipStream_t s) {
  if (fp32) {
    rad<float, RM_Y>(L, s);
    ang<float, AM_P>(L, s);
  } else {
    rad<double, RM_Y>(L, s);
    ang<double, AM_P>(L, s);
    for (int q = 0; q < L.nmg; ++q) mg_vcycle(*L.mg[q], L.mg[q]->r, L.mg[q]->ph, s);
  }
}

void launch_cycle(const LaunchSet &L, hipStream_t s) {
  if (L.nmg) {   // an FP64 batch
    cycle_mg(L, s);
    return;
  }
  if (L.mixed_any) sten<float, SM_UR>(KF_REFINE, L, s);
  if (L.mixed_any && !L.fp64_any) {
    cycle_t<float>(L, s);
  } else if (!L.mixed_any) {
    cycle_t<double>(L, s);
  } else {
    // a batch mixing both precisions runs both inner cycles; each instance
    // only takes part in the one matching its precision
    cycle_t<double>(L, s);
    cycle_t<float>(L, s);
  }
}

void launch_apply(const LaunchSet &L, double dt, double th, const void *x, void *y, int fp32,
                  hipStream_t s) {
  const dim3 go_orig((L.ninst + 63) / 64);
  if (fp32) {
    go(KF_CONTROL, k_sten<float, SM_APPLY>, g1(L.nb_sten), dim3(256), s, L.insts, L.map_sten, dt, th,
       (const float *)x, (float *)y);
    go(KF_CONTROL, k_apply_origin<float>, go_orig, dim3(64), s, L.insts, L.ninst, dt, th,
       (const float *)x, (float *)y);
  } else {
    go(KF_CONTROL, k_sten<double, SM_APPLY>, g1(L.nb_sten), dim3(256), s, L.insts, L.map_sten, dt, th,
       (const double *)x, (double *)y);
    go(KF_CONTROL, k_apply_origin<double>, go_orig, dim3(64), s, L.insts, L.ninst, dt, th,
       (const double *)x, (double *)y);
  }
}

void launch_mg_faces(const PdMgLevel *dlev, int l, int m, int nc, double *gp_r, double *gm_r, double *gp_t,
                     double *gm_t, double *inv_dth, double *b_node, hipStream_t s) {
  go(KF_MG, k_mg_faces, g1(((m + 1) * nc + 255) / 256), dim3(256), s, dlev, l, gp_r, gm_r, gp_t, gm_t, inv_dth,
     b_node);
}

void launch_begin_origin(const LaunchSet &L, hipStream_t s) {
  go(KF_BEGIN, k_begin_origin, dim3((L.ninst + 63) / 64), dim3(64), s, L.insts, L.ninst);
}

// ------------------------------------------------------------ two carriers
//
// A carrier of the coupled system (electrons or holes, (3.1) with the drift
// velocity s μ 𝓔 of §3.1's continuity equations, 𝓔 = -∇ψ) takes the drift
// of a potential ψ computed on the same mesh.  Per face, from the inner (or
// lower-θ) node P to the outer (or higher-θ) node Q,
//   K = c (ψ_P - ψ_Q),  c = s μ (face length) / (distance of P and Q),
// c and the conductance G kept from the set-up, and the face pair formed
// as at creation: central gp = G + K/2, gm = G - K/2, or upwind.  ψ_Q of the
// outer faces is the potential's Dirichlet value; P of the faces i = 1/2 is
// the origin.  One thread per face, radial faces first.
__global__ __launch_bounds__(256) void k_drift(int m, int n, int flux, const double *__restrict__ G_r,
                                               const double *__restrict__ c_r, const double *__restrict__ G_t,
                                               const double *__restrict__ c_t, const double *__restrict__ psi,
                                               const double *__restrict__ nb, const double *__restrict__ lam,
                                               const int *__restrict__ tpow, int nsrc,
                                               double *__restrict__ gp_r, double *__restrict__ gm_r,
                                               double *__restrict__ gp_t, double *__restrict__ gm_t) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  const int nr = (m + 1) * n, nt = m * n;
  double G, K;
  double *gp, *gm;
  if (k < nr) {
    const int i = k / n, j = k - i * n;
    const double pp = i == 0 ? psi[m * n] : psi[(i - 1) * n + j];
    const double pq = i == m ? boundary_value(nb, lam, tpow, nsrc, n, j, 0.0) : psi[i * n + j];
    G = G_r[k];
    K = c_r[k] * (pp - pq);
    gp = gp_r + k;
    gm = gm_r + k;
  } else if (k < nr + nt) {
    const int f = k - nr, i1 = f / n, j = f - i1 * n;   // ring i1 + 1
    const int jq = j + 1 == n ? 0 : j + 1;
    G = G_t[f];
    K = c_t[f] * (psi[i1 * n + j] - psi[i1 * n + jq]);
    gp = gp_t + f;
    gm = gm_t + f;
  } else {
    return;
  }
  if (flux == 0) {
    *gp = G + 0.5 * K;
    *gm = G - 0.5 * K;
  } else {
    *gp = G + fmax(K, 0.0);
    *gm = G - fmin(K, 0.0);
  }
}

// The face sums of the ring-mean correction that depend on the radial faces
// (PdInst::crs rows 2-5) after a drift update, one wave per ring i = 0..m
// (a fixed lane-strided order and butterfly), and the origin's diagonal of
// L, inv_V0 Σ_j gp_r(1/2, j) + b_0, into *l0.
__global__ __launch_bounds__(256) void k_drift_rings(int m, int n, const double *__restrict__ gp_r,
                                                     const double *__restrict__ gm_r, double *__restrict__ crs,
                                                     double inv_V0, double b0, double *__restrict__ l0) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i > m) return;                                   // the whole wave
  const int lane = threadIdx.x & 63, M1 = m + 1;
  double sO = 0.0, sU = 0.0, sI = 0.0, sL = 0.0;
  for (int j = lane; j < n; j += 64) {
    sO += gp_r[(size_t)i * n + j];
    if (i < m) sU += gm_r[(size_t)i * n + j];
    if (i >= 1) {
      sI += gm_r[(size_t)(i - 1) * n + j];
      sL += gp_r[(size_t)(i - 1) * n + j];
    }
  }
  sO = wave_sum(sO);
  sU = wave_sum(sU);
  sI = wave_sum(sI);
  sL = wave_sum(sL);
  if (lane == 0) {
    crs[2 * M1 + i] = sO;
    crs[3 * M1 + i] = sI;
    crs[4 * M1 + i] = sU;
    crs[5 * M1 + i] = sL;
    if (i == 0) *l0 = fma(inv_V0, sO, b0);
  }
}

// out = a - b over N values (the coupled system's charge p - n).
__global__ __launch_bounds__(256) void k_sub(const double *__restrict__ a, const double *__restrict__ b,
                                             double *__restrict__ out, int N) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < N) out[k] = a[k] - b[k];
}

// max |a - b| and max |a| over N values: per-block maxima, then one block
// takes the maxima of those (out[0], out[1]).
__global__ __launch_bounds__(256) void k_maxdiff(const double *__restrict__ a, const double *__restrict__ b,
                                                 int N, double *__restrict__ part) {
  __shared__ double sd[4], sa[4];
  double d = 0.0, x = 0.0;
  for (int k = blockIdx.x * 256 + threadIdx.x; k < N; k += gridDim.x * 256) {
    d = fmax(d, fabs(a[k] - b[k]));
    x = fmax(x, fabs(a[k]));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    d = fmax(d, __shfl_xor(d, o, 64));
    x = fmax(x, __shfl_xor(x, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    sd[threadIdx.x >> 6] = d;
    sa[threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = fmax(fmax(sd[0], sd[1]), fmax(sd[2], sd[3]));
    part[2 * blockIdx.x + 1] = fmax(fmax(sa[0], sa[1]), fmax(sa[2], sa[3]));
  }
}
__global__ __launch_bounds__(256) void k_maxdiff_final(const double *__restrict__ part, int nblk,
                                                       double *__restrict__ out) {
  __shared__ double sd[4], sa[4];
  double d = 0.0, x = 0.0;
  for (int k = threadIdx.x; k < nblk; k += 256) {
    d = fmax(d, part[2 * k]);
    x = fmax(x, part[2 * k + 1]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    d = fmax(d, __shfl_xor(d, o, 64));
    x = fmax(x, __shfl_xor(x, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    sd[threadIdx.x >> 6] = d;
    sa[threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = fmax(fmax(sd[0], sd[1]), fmax(sd[2], sd[3]));
    out[1] = fmax(fmax(sa[0], sa[1]), fmax(sa[2], sa[3]));
  }
}

void launch_drift(int m, int n, int flux, const double *G_r, const double *c_r, const double *G_t,
                  const double *c_t, const double *psi, const double *nb, const double *lam, const int *tpow,
                  int nsrc, double *gp_r, double *gm_r, double *gp_t, double *gm_t, double *crs, double inv_V0,
                  double b0, double *l0, hipStream_t s) {
  const int faces = (2 * m + 1) * n;
  go(KF_CONTROL, k_drift, dim3((faces + 255) / 256), dim3(256), s, m, n, flux, G_r, c_r, G_t, c_t, psi, nb,
     lam, tpow, nsrc, gp_r, gm_r, gp_t, gm_t);
  go(KF_CONTROL, k_drift_rings, dim3((m + 1 + 3) / 4), dim3(256), s, m, n, (const double *)gp_r,
     (const double *)gm_r, crs, inv_V0, b0, l0);
}

void launch_sub(const double *a, const double *b, double *out, int N, hipStream_t s) {
  go(KF_CONTROL, k_sub, dim3((N + 255) / 256), dim3(256), s, a, b, out, N);
}

void launch_maxdiff(const double *a, const double *b, int N, double *part, int nblk, double *out,
                    hipStream_t s) {
  go(KF_CONTROL, k_maxdiff, dim3(nblk), dim3(256), s, a, b, N, part);
  go(KF_CONTROL, k_maxdiff_final, dim3(1), dim3(256), s, (const double *)part, nblk, out);
}

void launch_indicator(const double *x, int m, int n, const double *r, const double *th,
                      const double *nb, const double *lam, const int *tpow, int nsrc, double t,
                      int dirichlet, double *ring_out, double *eta_out, hipStream_t s) {
  go(KF_CONTROL, k_indicator, dim3((m + 3) / 4), dim3(256), s, x, m, n, r, th, nb, lam, tpow, nsrc, t,
     dirichlet, ring_out, eta_out);
}

void launch_transfer(const double *x, int m, int n, const double *r, const double *th, const double *nb,
                     const double *lam, const int *tpow, int nsrc, double t, int dirichlet,
                     const double *r2, const double *th2, int m2, int n2, double *y, hipStream_t s) {
  const int cnt = m2 * n2;
  go(KF_CONTROL, k_transfer, dim3((cnt + 255) / 256), dim3(256), s, x, m, n, r, th, nb, lam, tpow, nsrc, t,
     dirichlet, r2, th2, m2, n2, y);
}

}  // namespace pd
