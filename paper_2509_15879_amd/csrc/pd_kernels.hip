// HIP kernels (gfx950 / CDNA4) of the polar-disk θ-scheme solver.
//
// Every kernel is batched: a block map turns blockIdx.x into (instance,
// local block), so one launch advances every instance of a batch, whatever
// its mesh size or PDE type.  Per-instance Krylov scalars live in device
// memory and are finalised by the last block of each reducing kernel, in a
// fixed order that depends only on the instance's own tiling (a result does
// not depend on which other instances share the launch).
//
// One time level (scheme (2.5) of §2.1, Ch. 3 scheme of §3.2.1, system
// (2.11)/(2.12)) is
//   k_level_begin   per-instance set-up: Δt, θ, source weights, extrapolation
//   k_fact_rad      radial-line LU of (D + R) per θ-column (when Δt/θ change)
//   k_fact_ang      ring-periodic LU of (I + D^{-1} Θ) per ring, Sherman-Morrison
//   k_sten<BEGIN>   rhs, extrapolated initial guess and its residual
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
// periodic) couplings of A; the origin row is left as is (unit diagonal).
// The radial blocks are the tridiagonal A_j of (2.12).
//
// Arithmetic is FP64 throughout; the FP32 inner solve of the mixed-precision
// mode only stores its vectors, faces and multipliers in FP32 (pivots stay
// FP64).

#include "pd_device.h"

#include <math.h>

namespace pd {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ double ld(const T *p, int i) { return (double)p[i]; }

__device__ __forceinline__ double tau_q(double lam, int tp, double t) {
  double v = exp(lam * t);
  for (int k = 0; k < tp; ++k) v *= t;
  return v;
}

// Block-wide reduction of NS partial sums into a per-instance partial array,
// followed by a deterministic reduction of all partials by the last block of
// the instance.  Returns true in that last block, with the totals in tot.
template <int NS>
__device__ bool block_commit(double (&v)[NS], double *part, int nblk, int blk, unsigned *counter,
                             double (&tot)[NS]) {
  __shared__ double red[NS][16];
  __shared__ int s_last;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    double x = wave_sum(v[k]);
    if (lane == 0) red[k][wave] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[k][w];
      __hip_atomic_store(&part[k * nblk + blk], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __threadfence();
    unsigned t = atomicAdd(counter, 1u);
    s_last = (t == (unsigned)(nblk - 1)) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  double acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
      s += __hip_atomic_load(&part[k * nblk + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    acc[k] = wave_sum(s);
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) red[k][wave] = acc[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[k][w];
    tot[k] = s;
  }
  if (threadIdx.x == 0) atomicExch(counter, 0u);
  return true;
}

__device__ __forceinline__ void finish_instance(const PdInst &I, PdScalars *sc, int status) {
  sc->status = status;
  atomicSub(I.n_active, 1);
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
  return I.sol[(sc->rot + 2) % 3];
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

// ------------------------------------------------------------ level control

// Per-instance set-up of a time level t_k -> t_{k+1} (one thread per instance).
__global__ void k_level_begin(PdInst *insts, int ninst) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ninst) return;
  PdInst &I = insts[q];
  PdScalars *sc = I.sc;
  if (sc->status == ST_IDLE) return;          // not stepping in this level
  const int k = sc->level;
  const double t0 = I.t_table[k], t1 = I.t_table[k + 1];
  const double dt = t1 - t0, th = sc->theta;
  sc->t0 = t0;
  sc->t1 = t1;
  sc->dt = dt;
  sc->inv_dt = 1.0 / dt;
  sc->refactor = (dt != sc->fact_dt || th != sc->fact_theta) ? 1 : 0;
  sc->extrap = sc->have_prev ? dt / sc->prev_dt : 0.0;
  for (int s = 0; s < PD_MAXSRC; ++s) sc->cq[s] = 0.0;
  for (int s = 0; s < I.nsrc; ++s)
    sc->cq[s] = (1.0 - th) * tau_q(I.lam[s], I.tpow[s], t0) + th * tau_q(I.lam[s], I.tpow[s], t1);
  sc->status = ST_ACTIVE;
  atomicAdd(I.n_active, 1);
  sc->phase = PH_INNER;
  sc->iters = 0;
  sc->outer = 0;
  sc->inner_iters = 0;
  sc->restarts = 0;
  sc->first = 1;
  sc->reset_rh = 0;
  sc->inner_first = I.mixed ? 1 : 0;
  sc->alpha = sc->omega = 1.0;
  sc->rho_old = sc->rho_new = 1.0;
}

// Records the level, rotates the solution buffers (iterate -> n^{k+1}).
__global__ void k_level_end(PdInst *insts, int ninst) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ninst) return;
  PdInst &I = insts[q];
  PdScalars *sc = I.sc;
  if (sc->status == ST_IDLE) return;
  const int k = sc->level;
  double *st = I.level_stats + 8 * k;
  st[0] = sc->iters;
  st[1] = sc->outer;
  st[2] = sc->status;
  st[3] = sc->rel_resid;
  st[4] = sc->dt;
  st[5] = sc->t1;
  st[6] = sc->restarts;
  st[7] = 0.0;
  sc->total_iters += sc->iters;
  const bool ok = sc->status == ST_DONE;
  if (!ok) sc->nfail += 1;
  sc->rot = (sc->rot + 1) % 3;       // old iterate slot becomes n^k
  sc->prev_dt = sc->dt;
  sc->have_prev = 1;
  sc->t_now = sc->t1;
  sc->level = k + 1;
  if (sc->refactor) {
    sc->fact_dt = sc->dt;
    sc->fact_theta = sc->theta;
  }
  sc->status = (ok && k + 1 < sc->K) ? ST_DONE : ST_IDLE;
}

// ------------------------------------------------------------ factorisations

// Diagonal of A = I/dt + θ L_h at ring node (i, j) (i = 1..m).
__device__ __forceinline__ double diag_at(const PdInst &I, int i, int j, double inv_dt, double th) {
  const int n = I.n;
  const int jl = (j == 0) ? n - 1 : j - 1;
  const double *gpr = I.k64.gp_r, *gmr = I.k64.gm_r, *gpt = I.k64.gp_t, *gmt = I.k64.gm_t;
  const int row = (i - 1) * n;
  double s = gpr[i * n + j] + gmr[(i - 1) * n + j] + gpt[row + j] + gmt[row + jl];
  double v = I.inv_rw[i] * I.inv_dth[j] * s;
  if (I.has_b) v += I.b_node[row + j];
  return inv_dt + th * v;
}

// Radial-line LU of (I + D^{-1}R) for column j:  rows i = 1..m, diagonal 1,
// sub-diagonal a_i = -θ gp_r(i-1/2)/(V d_i) (i >= 2), super
// c_i = -θ gm_r(i+1/2)/(V d_i).  Stored: uinv_i = 1/u_i, f_i = a_i/u_i,
// g_i = c_i/u_i, so that forward  w_i = uinv_i y_i - f_i w_{i-1},
// backward  x_i = w_i - g_i x_{i+1}.  Also stores d and 1/d.
__global__ void k_fact_rad(const PdInst *insts, const int2 *map) {
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  const PdScalars *sc = I.sc;
  if (sc->status != ST_ACTIVE || !sc->refactor) return;
  const int j = mp.y * blockDim.x + threadIdx.x;
  const int m = I.m, n = I.n;
  const double th = sc->theta, inv_dt = sc->inv_dt;
  if (j < n) {
    double u_prev = 1.0, c_prev = 0.0;
    for (int i = 1; i <= m; ++i) {
      const int idx = (i - 1) * n + j;
      const double d = diag_at(I, i, j, inv_dt, th);
      const double id = 1.0 / d;
      const double ivV = I.inv_rw[i] * I.inv_dth[j] * id;
      const double a = (i >= 2) ? -th * ivV * I.k64.gp_r[(i - 1) * n + j] : 0.0;
      const double c = (i < m) ? -th * ivV * I.k64.gm_r[i * n + j] : 0.0;
      const double u = 1.0 - a * c_prev / u_prev;
      const double ui = 1.0 / u;
      I.diag[idx] = d;
      I.inv_diag[idx] = id;
      if (I.mixed) I.inv_diag32[idx] = (float)id;
      I.rf_uinv[idx] = ui;
      I.k64.rf_f[idx] = a * ui;
      I.k64.rf_g[idx] = c * ui;
      if (I.mixed) {
        I.k32.rf_f[idx] = (float)(a * ui);
        I.k32.rf_g[idx] = (float)(c * ui);
      }
      u_prev = u;
      c_prev = c;
    }
  }
  if (mp.y == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int jj = 0; jj < n; ++jj) s += I.k64.gp_r[jj];
    double v = I.inv_V0 * s;
    if (I.has_b) v += I.b_node[m * n];
    const double d0 = inv_dt + th * v;
    I.diag[m * n] = d0;
    I.inv_diag[m * n] = 1.0 / d0;
    if (I.mixed) I.inv_diag32[m * n] = (float)(1.0 / d0);
  }
}

// Ring-periodic LU of (I + D^{-1}Θ) for ring i: row j has diagonal 1,
// sub α_j = -θ gp_t(j-1/2)/(V d_j), super γ_j = -θ gm_t(j+1/2)/(V d_j),
// periodic corners α_0 (row 0, column n-1) and γ_{n-1} (row n-1, column 0).
// Sherman-Morrison with u = (-1, 0.., γ_{n-1}), v = (1, 0.., -α_0): the
// non-periodic T0 has diagonal 2 at row 0 and 1 + γ_{n-1} α_0 at row n-1;
// z = T0^{-1} u and κ = 1/(1 + z_0 - α_0 z_{n-1}) are stored so that
// x = y - κ (y_0 - α_0 y_{n-1}) z with y = T0^{-1} d.
__global__ void k_fact_ang(const PdInst *insts, const int2 *map) {
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  const PdScalars *sc = I.sc;
  if (sc->status != ST_ACTIVE || !sc->refactor) return;
  const int i = mp.y * blockDim.x + threadIdx.x + 1;
  const int m = I.m, n = I.n;
  if (i > m) return;
  const double th = sc->theta;
  const int row = (i - 1) * n;
  const double irw = I.inv_rw[i];
  auto alpha_j = [&](int j) {
    const int jl = (j == 0) ? n - 1 : j - 1;
    return -th * irw * I.inv_dth[j] * I.k64.gp_t[row + jl] / I.diag[row + j];
  };
  auto gamma_j = [&](int j) {
    return -th * irw * I.inv_dth[j] * I.k64.gm_t[row + j] / I.diag[row + j];
  };
  const double a0 = alpha_j(0);
  const double gl = gamma_j(n - 1);
  // factor T0 and solve T0 z = u on the fly (forward), then backward for z
  double u_prev = 1.0, c_prev = 0.0, zf_prev = 0.0;
  for (int j = 0; j < n; ++j) {
    const double a = (j >= 1) ? alpha_j(j) : 0.0;
    const double c = (j < n - 1) ? gamma_j(j) : 0.0;
    double dj = 1.0;
    if (j == 0) dj = 2.0;
    if (j == n - 1) dj = 1.0 + gl * a0;
    const double u = dj - a * c_prev / u_prev;
    const double ui = 1.0 / u;
    const double f = a * ui, g = c * ui;
    I.af_uinv[row + j] = ui;
    I.k64.af_f[row + j] = f;
    I.k64.af_g[row + j] = g;
    const double uj = (j == 0) ? -1.0 : ((j == n - 1) ? gl : 0.0);
    const double zf = ui * uj - f * zf_prev;   // forward substitution of u
    I.k64.af_z[row + j] = zf;
    zf_prev = zf;
    u_prev = u;
    c_prev = c;
  }
  double xn = 0.0;
  double z0 = 0.0, zl = 0.0;
  for (int j = n - 1; j >= 0; --j) {
    const double x = I.k64.af_z[row + j] - I.k64.af_g[row + j] * xn;
    I.k64.af_z[row + j] = x;
    if (j == n - 1) zl = x;
    if (j == 0) z0 = x;
    xn = x;
  }
  I.af_kappa[i - 1] = 1.0 / (1.0 + z0 - a0 * zl);
  I.af_alpha0[i - 1] = a0;
  if (I.mixed) {
    for (int j = 0; j < n; ++j) {
      I.k32.af_f[row + j] = (float)I.k64.af_f[row + j];
      I.k32.af_g[row + j] = (float)I.k64.af_g[row + j];
      I.k32.af_z[row + j] = (float)I.k64.af_z[row + j];
    }
  }
}

// ------------------------------------------------------------ stencil march
//
// One wave owns 64 consecutive θ-columns and PD_RB consecutive rings and
// marches outward in r, keeping the radial neighbours and the shared radial
// faces in registers; the θ-neighbours come from the adjacent lanes by
// cross-lane permutes, and only the two wave-edge columns (including the
// periodic seam j = n-1 <-> 0) are fetched from memory.  The origin row is a
// sum over ring 1 accumulated per block and closed by the instance's last
// block.

template <typename TF, typename TX, int NV, class Epi>
__device__ __forceinline__ void sten_tile(const PdInst &I, const TF *gp_r, const TF *gm_r,
                                          const TF *gp_t, const TF *gm_t, const TX *const (&X)[NV],
                                          int cg, int rg, double (&S0)[NV], Epi &&epi) {
  const int m = I.m, n = I.n, lane = threadIdx.x & 63;
  const int j = cg * 64 + lane;
  const bool act = j < n;
  const int jc = act ? j : n - 1;
  const int jl = (jc == 0) ? n - 1 : jc - 1;
  const int jr = (jc == n - 1) ? 0 : jc + 1;
  const bool need_l = (lane == 0);
  const bool need_r = (lane == 63) || (j + 1 >= n);
  const int i0 = rg * PD_RB + 1;
  const int i1 = min(i0 + PD_RB - 1, m);
  const double idth = I.inv_dth[jc];
  const int orig = m * n;

  double xb[NV], xc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    xb[v] = (i0 == 1) ? ld(X[v], orig) : ld(X[v], (i0 - 2) * n + jc);
    xc[v] = ld(X[v], (i0 - 1) * n + jc);
  }
  double gpi = ld(gp_r, (i0 - 1) * n + jc), gmi = ld(gm_r, (i0 - 1) * n + jc);
  for (int i = i0; i <= i1; ++i) {
    const int row = (i - 1) * n;
    const double gpo = ld(gp_r, i * n + jc), gmo = ld(gm_r, i * n + jc);
    const double gpt = ld(gp_t, row + jc), gmt = ld(gm_t, row + jc);
    double gptl = __shfl_up(gpt, 1, 64), gmtl = __shfl_up(gmt, 1, 64);
    if (need_l) {
      gptl = ld(gp_t, row + jl);
      gmtl = ld(gm_t, row + jl);
    }
    const double ivV = I.inv_rw[i] * idth;
    const double bP = I.has_b ? I.b_node[row + jc] : 0.0;
    double Lx[NV], xa[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      xa[v] = (i < m) ? ld(X[v], i * n + jc) : 0.0;
      double xl = __shfl_up(xc[v], 1, 64), xr = __shfl_down(xc[v], 1, 64);
      if (need_l) xl = ld(X[v], row + jl);
      if (need_r) xr = ld(X[v], row + jr);
      const double fs = gpo * xc[v] - gmo * xa[v] + gmi * xc[v] - gpi * xb[v] + gpt * xc[v] -
                        gmt * xr + gmtl * xc[v] - gptl * xl;
      Lx[v] = ivV * fs + bP * xc[v];
      if (i == 1 && act) S0[v] += gpi * xb[v] - gmi * xc[v];
    }
    if (act) epi(i, jc, row + jc, xc, Lx);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      xb[v] = xc[v];
      xc[v] = xa[v];
    }
    gpi = gpo;
    gmi = gmo;
  }
}

enum { SM_APPLY = 0, SM_BEGIN = 1, SM_V = 2, SM_T = 3, SM_UR = 4 };

// Stencil kernels.  TK: storage type of the Krylov set the mode works on.
//  SM_APPLY: y = x/dt + θ L x (diagnostic; dt, θ, x, y passed explicitly)
//  SM_BEGIN: b = x^k/dt - (1-θ) L x^k + Σ_q c_q g_q + boundary;
//            x0 = x^k + ρ (x^k - x^{k-1});  r = b - A x0;  r̂ = r
//  SM_V:     v = A p̂,  partial r̂·v
//  SM_T:     t = A ŝ,  partials t·s, t·t
//  SM_UR:    (mixed) r ← r - A d in FP64, x ← x + d; r32 = r̂32 = r
template <typename TK, int MODE>
__global__ __launch_bounds__(256) void k_sten(const PdInst *insts, const int2 *map, double a_dt,
                                              double a_th, const TK *ax, TK *ay) {
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  PdScalars *sc = I.sc;
  if (MODE == SM_V || MODE == SM_T) {
    if (!inner_active(sc) || !prec_match<TK>(I)) return;
  } else if (MODE == SM_BEGIN) {
    if (sc->status != ST_ACTIVE) return;
  } else if (MODE == SM_UR) {
    if (sc->status != ST_ACTIVE || sc->phase != PH_OUTER) return;
  }
  const int wave = threadIdx.x >> 6;
  const int tile = mp.y * PD_STEN_WAVES + wave;
  const bool wave_on = tile < I.ncg * I.nrg;
  const int cg = wave_on ? tile % I.ncg : 0, rg = wave_on ? tile / I.ncg : 0;
  const int m = I.m, n = I.n, orig = m * n;
  const KSet<TK> &KS = kset<TK>(I);

  if (MODE == SM_APPLY) {
    const double inv_dt = 1.0 / a_dt, th = a_th;
    double S0[1] = {0.0};
    const TK *X[1] = {ax};
    if (wave_on)
      sten_tile<TK, TK, 1>(I, KS.gp_r, KS.gm_r, KS.gp_t, KS.gm_t, X, cg, rg, S0,
                           [&](int, int, int idx, const double *xc, const double *Lx) {
                             ay[idx] = (TK)(inv_dt * xc[0] + th * Lx[0]);
                           });
    double tot[1];
    if (block_commit<1>(S0, I.partials, I.nb_sten, mp.y, I.counters + CNT_APPLY, tot) &&
        threadIdx.x == 0) {
      const double x0 = ld(ax, orig);
      const double bo = I.has_b ? I.b_node[orig] : 0.0;
      ay[orig] = (TK)(inv_dt * x0 + th * (I.inv_V0 * tot[0] + bo * x0));
    }
  } else if (MODE == SM_BEGIN) {
    // FP64 operator on x^k and x^{k-1}
    const double inv_dt = sc->inv_dt, th = sc->theta, rho = sc->extrap;
    const double *xk = I.sol[(sc->rot + 1) % 3];
    const double *xkm = I.sol[sc->rot % 3];
    double *x0 = I.sol[(sc->rot + 2) % 3];
    const bool ex = rho != 0.0;
    double cq[PD_MAXSRC];
    for (int s = 0; s < PD_MAXSRC; ++s) cq[s] = sc->cq[s];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};   // ||b||^2, ||r||^2, S0(x^k), S0(x^{k-1})
    double S0[2] = {0.0, 0.0};
    const double *X[2] = {xk, ex ? xkm : xk};
    const double *gpr = I.k64.gp_r, *gmr = I.k64.gm_r;
    if (wave_on)
      sten_tile<double, double, 2>(
          I, gpr, gmr, I.k64.gp_t, I.k64.gm_t, X, cg, rg, S0,
          [&](int i, int j, int idx, const double *xc, const double *Lx) {
            double b = inv_dt * xc[0] - (1.0 - th) * Lx[0];
            for (int s = 0; s < I.nsrc; ++s) b += cq[s] * I.g[s * I.npad + idx];
            if (i == m) {
              double Nm = 0.0;
              for (int s = 0; s < I.nsrc; ++s) Nm += cq[s] * I.nb[s * n + j];
              b += I.inv_rw[i] * I.inv_dth[j] * gmr[m * n + j] * Nm;
            }
            const double xg = ex ? xc[0] + rho * (xc[0] - xc[1]) : xc[0];
            const double Lg = ex ? Lx[0] + rho * (Lx[0] - Lx[1]) : Lx[0];
            const double r = b - (inv_dt * xg + th * Lg);
            const double idg = I.inv_diag[idx];
            const double rs = r * idg, bs = b * idg;
            I.bvec[idx] = b;
            x0[idx] = xg;
            if (I.mixed) {
              I.rout[idx] = r;
              I.k32.r[idx] = (float)rs;
              I.k32.rh[idx] = (float)rs;
            } else {
              I.k64.r[idx] = rs;
              I.k64.rh[idx] = rs;
            }
            acc[0] += bs * bs;
            acc[1] += rs * rs;
          });
    acc[2] = S0[0];
    acc[3] = S0[1];
    double tot[4];
    if (block_commit<4>(acc, I.partials, I.nb_sten, mp.y, I.counters + CNT_BEGIN, tot) &&
        threadIdx.x == 0) {
      const double bo = I.has_b ? I.b_node[orig] : 0.0;
      const double xk0 = xk[orig], xkm0 = ex ? xkm[orig] : xk0;
      const double L0 = I.inv_V0 * tot[2] + bo * xk0;
      const double L1 = I.inv_V0 * tot[3] + bo * xkm0;
      double b = inv_dt * xk0 - (1.0 - th) * L0;
      for (int s = 0; s < I.nsrc; ++s) b += cq[s] * I.g[s * I.npad + orig];
      const double xg = ex ? xk0 + rho * (xk0 - xkm0) : xk0;
      const double Lg = ex ? L0 + rho * (L0 - L1) : L0;
      const double r = b - (inv_dt * xg + th * Lg);
      const double idg = I.inv_diag[orig];
      const double rs = r * idg, bs = b * idg;
      I.bvec[orig] = b;
      x0[orig] = xg;
      if (I.mixed) {
        I.rout[orig] = r;
        I.k32.r[orig] = (float)rs;
        I.k32.rh[orig] = (float)rs;
      } else {
        I.k64.r[orig] = rs;
        I.k64.rh[orig] = rs;
      }
      const double bb = tot[0] + bs * bs, rr = tot[1] + rs * rs;
      sc->bnorm2 = bb;
      sc->rnorm2 = rr;
      sc->r0norm2 = rr;
      sc->rho_new = rr;
      sc->rel_resid = bb > 0.0 ? sqrt(rr / bb) : 0.0;
      if (!(rr == rr) || !(bb == bb)) {
        finish_instance(I, sc, ST_BREAKDOWN);
      } else if (rr <= sc->tol * sc->tol * bb) {
        finish_instance(I, sc, ST_DONE);
      }
    }
  } else if (MODE == SM_V || MODE == SM_T) {
    const double inv_dt = sc->inv_dt, th = sc->theta;
    const TK *xin = (MODE == SM_V) ? KS.ph : KS.sh;
    TK *yout = (MODE == SM_V) ? KS.v : KS.t;
    const TK *other = (MODE == SM_V) ? KS.rh : KS.s;
    double acc[3] = {0.0, 0.0, 0.0};
    double S0[1] = {0.0};
    const TK *X[1] = {xin};
    if (wave_on)
      sten_tile<TK, TK, 1>(I, KS.gp_r, KS.gm_r, KS.gp_t, KS.gm_t, X, cg, rg, S0,
                           [&](int, int, int idx, const double *xc, const double *Lx) {
                             const double y = (inv_dt * xc[0] + th * Lx[0]) * ld(KS.inv_d, idx);
                             const TK ys = (TK)y;
                             yout[idx] = ys;
                             const double yd = (double)ys;
                             acc[0] += ld(other, idx) * yd;
                             acc[1] += yd * yd;
                           });
    acc[2] = S0[0];
    double tot[3];
    if (block_commit<3>(acc, I.partials, I.nb_sten, mp.y,
                        I.counters + (MODE == SM_V ? CNT_V : CNT_T), tot) &&
        threadIdx.x == 0) {
      const double bo = I.has_b ? I.b_node[orig] : 0.0;
      const double x0 = ld(xin, orig);
      const double y0 = (inv_dt * x0 + th * (I.inv_V0 * tot[2] + bo * x0)) * ld(KS.inv_d, orig);
      const TK ys = (TK)y0;
      yout[orig] = ys;
      const double yd = (double)ys;
      const double dot = tot[0] + ld(other, orig) * yd;
      const double yy = tot[1] + yd * yd;
      if (MODE == SM_V) {
        // α = ρ / (r̂·v)
        if (!(dot == dot)) {
          finish_instance(I, sc, ST_BREAKDOWN);
        } else if (fabs(dot) <= 1e-300 || fabs(sc->rho_new) <= 1e-300) {
          sc->alpha = 0.0;
          sc->reset_rh = 1;     // restart: r̂ = r, p = r
        } else {
          sc->alpha = sc->rho_new / dot;
        }
        sc->first = 0;
      } else {
        // ω = (t·s)/(t·t)
        if (!(dot == dot) || !(yy == yy)) {
          finish_instance(I, sc, ST_BREAKDOWN);
        } else if (yy <= 1e-300) {
          sc->omega = 0.0;
          sc->reset_rh = 1;
        } else {
          sc->omega = dot / yy;
        }
      }
    }
  } else if (MODE == SM_UR) {
    // FP64 operator applied to the FP32 correction d
    const double inv_dt = sc->inv_dt, th = sc->theta;
    double *x = I.sol[(sc->rot + 2) % 3];
    double acc[2] = {0.0, 0.0};
    double S0[1] = {0.0};
    const float *X[1] = {I.k32.d};
    if (wave_on)
      sten_tile<double, float, 1>(I, I.k64.gp_r, I.k64.gm_r, I.k64.gp_t, I.k64.gm_t, X, cg, rg, S0,
                                  [&](int, int, int idx, const double *xc, const double *Lx) {
                                    const double r = I.rout[idx] - (inv_dt * xc[0] + th * Lx[0]);
                                    const double rs = r * I.inv_diag[idx];
                                    I.rout[idx] = r;
                                    x[idx] += xc[0];
                                    I.k32.r[idx] = (float)rs;
                                    I.k32.rh[idx] = (float)rs;
                                    acc[0] += rs * rs;
                                  });
    acc[1] = S0[0];
    double tot[2];
    if (block_commit<2>(acc, I.partials, I.nb_sten, mp.y, I.counters + CNT_UR, tot) &&
        threadIdx.x == 0) {
      const double bo = I.has_b ? I.b_node[orig] : 0.0;
      const double d0 = (double)I.k32.d[orig];
      const double r = I.rout[orig] - (inv_dt * d0 + th * (I.inv_V0 * tot[1] + bo * d0));
      const double rs = r * I.inv_diag[orig];
      I.rout[orig] = r;
      x[orig] += d0;
      I.k32.r[orig] = (float)rs;
      I.k32.rh[orig] = (float)rs;
      const double rr = tot[0] + rs * rs;
      sc->rnorm2 = rr;
      sc->outer += 1;
      sc->rel_resid = sqrt(rr / sc->bnorm2);
      if (!(rr == rr)) {
        finish_instance(I, sc, ST_BREAKDOWN);
      } else if (rr <= sc->tol * sc->tol * sc->bnorm2) {
        finish_instance(I, sc, ST_DONE);
      } else if (sc->outer >= sc->max_outer) {
        finish_instance(I, sc, ST_NOCONV);
      } else {
        sc->phase = PH_INNER;
        sc->first = 1;
        sc->inner_first = 1;
        sc->inner_iters = 0;
        sc->r0norm2 = rr;
        sc->rho_new = rr;
        sc->alpha = sc->omega = 1.0;
      }
    }
  }
}

// ------------------------------------------------------------ radial sweep
//
// w = (D + R)^{-1} y for every θ-column of an instance.  A block owns cw
// consecutive columns; its 1024 threads split every column into nseg
// segments of brad rows (lane = column within the block, segment = the rest
// of the thread index).  Each thread runs the forward and backward
// substitution of its segment locally, holding the segment in registers;
// the segments are then joined by composing their affine maps
// w -> P w + e across segments through LDS (a segmented scan), and each
// thread corrects its rows.  The origin is scaled by its diagonal.
//
// RM_P:  y = p = r + β (p - ω v)   (p = r on a (re)start; r̂ = r on a restart)
// RM_S:  y = s = r - α v
// RM_PLAIN: y = x (diagnostic)

enum { RM_P = 0, RM_S = 1, RM_PLAIN = 2 };

template <typename T, int MODE>
__global__ __launch_bounds__(PD_RAD_THREADS) void k_rad(const PdInst *insts, const int2 *map,
                                                        const T *plain_in, T *plain_out) {
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  PdScalars *sc = I.sc;
  if (MODE != RM_PLAIN && (!inner_active(sc) || !prec_match<T>(I))) return;
  const KSet<T> &KS = kset<T>(I);
  const int m = I.m, n = I.n, cw = I.cw, B = I.brad;
  const int c = threadIdx.x % cw, seg = threadIdx.x / cw;
  const int j = mp.y * cw + c;
  const bool act = j < n;
  const int i_begin = seg * B;                       // 0-based row
  const int cnt = act ? max(0, min(B, m - i_begin)) : 0;

  __shared__ double lds_a[PD_RAD_THREADS];
  __shared__ double lds_b[PD_RAD_THREADS];

  double beta = 0.0, omega = 0.0, alpha = 0.0;
  bool first = false, reset = false;
  if (MODE == RM_P) {
    first = sc->first || sc->reset_rh;
    reset = sc->reset_rh;
    omega = sc->omega;
    beta = first ? 0.0 : (sc->rho_new / sc->rho_old) * (sc->alpha / sc->omega);
  } else if (MODE == RM_S) {
    alpha = sc->alpha;
  }
  T *out = (MODE == RM_PLAIN) ? plain_out : KS.w;

  auto input = [&](int idx) -> double {
    if (MODE == RM_P) {
      const double r = ld(KS.r, idx);
      double p = first ? r : r + beta * (ld(KS.p, idx) - omega * ld(KS.v, idx));
      const T ps = (T)p;
      KS.p[idx] = ps;
      if (reset) KS.rh[idx] = (T)r;
      return (double)ps;
    } else if (MODE == RM_S) {
      const double s = ld(KS.r, idx) - alpha * ld(KS.v, idx);
      const T ss = (T)s;
      KS.s[idx] = ss;
      return (double)ss;
    } else {
      return ld(plain_in, idx);
    }
  };

  // origin (one thread of the instance's first block): unit diagonal
  if (mp.y == 0 && threadIdx.x == 0) {
    const int o = m * n;
    out[o] = (T)input(o);
  }

  // forward local pass
  double wl[PD_RAD_BMAX] = {};
  double W = 0.0, P = 1.0;
#pragma unroll
  for (int k = 0; k < PD_RAD_BMAX; ++k) {
    if (k < cnt) {
      const int idx = (i_begin + k) * n + j;
      const double y = input(idx);
      const double f = ld(KS.rf_f, idx);
      W = I.rf_uinv[idx] * y - f * W;
      P *= -f;
      wl[k] = W;
    }
  }
  lds_a[threadIdx.x] = W;
  lds_b[threadIdx.x] = P;
  __syncthreads();
  double Win = 0.0;
  for (int s2 = 0; s2 < seg; ++s2) Win = lds_b[s2 * cw + c] * Win + lds_a[s2 * cw + c];
  __syncthreads();
  // fix-up of the forward pass, then local backward pass
  P = 1.0;
#pragma unroll
  for (int k = 0; k < PD_RAD_BMAX; ++k) {
    if (k < cnt) {
      P *= -ld(KS.rf_f, (i_begin + k) * n + j);
      wl[k] += P * Win;
    }
  }
  double X = 0.0, Q = 1.0;
#pragma unroll
  for (int k = PD_RAD_BMAX - 1; k >= 0; --k) {
    if (k < cnt) {
      const double g = ld(KS.rf_g, (i_begin + k) * n + j);
      X = wl[k] - g * X;
      Q *= -g;
      wl[k] = X;
    }
  }
  lds_a[threadIdx.x] = X;
  lds_b[threadIdx.x] = Q;
  __syncthreads();
  const int nseg = I.nseg;
  double Xin = 0.0;
  for (int s2 = nseg - 1; s2 > seg; --s2) Xin = lds_b[s2 * cw + c] * Xin + lds_a[s2 * cw + c];
  Q = 1.0;
#pragma unroll
  for (int k = PD_RAD_BMAX - 1; k >= 0; --k) {
    if (k < cnt) {
      const int idx = (i_begin + k) * n + j;
      Q *= -ld(KS.rf_g, idx);
      out[idx] = (T)(wl[k] + Q * Xin);
    }
  }
}

// ------------------------------------------------------------ angular sweep
//
// z = (I + D^{-1}Θ)^{-1} w for every ring: one wave per ring, lane L owns
// the bang consecutive nodes j in [L*bang, (L+1)*bang).  Local substitution
// in registers, then the lanes' affine maps are composed by a Kogge-Stone
// scan across the wave (prefix for the forward, suffix for the backward
// substitution), then the Sherman-Morrison correction closes the period.
//
// AM_P: input w, output p̂ (origin copied);  AM_S: output ŝ;  AM_PLAIN: diagnostic.
enum { AM_P = 0, AM_S = 1, AM_PLAIN = 2 };

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_ang(const PdInst *insts, const int2 *map,
                                             const T *plain_in, T *plain_out) {
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  const PdScalars *sc = I.sc;
  if (MODE != AM_PLAIN && (!inner_active(sc) || !prec_match<T>(I))) return;
  const KSet<T> &KS = kset<T>(I);
  const int m = I.m, n = I.n, B = I.bang;
  const int lane = threadIdx.x & 63;
  const int i = mp.y * 4 + (threadIdx.x >> 6) + 1;
  if (i > m) return;                                 // whole wave exits together
  const T *in = (MODE == AM_PLAIN) ? plain_in : KS.w;
  T *out = (MODE == AM_PLAIN) ? plain_out : ((MODE == AM_P) ? KS.ph : KS.sh);
  const int row = (i - 1) * n;
  const int j0 = lane * B;
  const int cnt = max(0, min(B, n - j0));

  if (i == 1 && lane == 0) out[m * n] = in[m * n];

  double wl[PD_ANG_BMAX] = {};
  double W = 0.0, P = 1.0;
#pragma unroll
  for (int k = 0; k < PD_ANG_BMAX; ++k) {
    if (k < cnt) {
      const int idx = row + j0 + k;
      const double f = ld(KS.af_f, idx);
      W = I.af_uinv[idx] * ld(in, idx) - f * W;
      P *= -f;
      wl[k] = W;
    }
  }
  // inclusive prefix composition of (P, W) over lanes
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double Pp = __shfl_up(P, d, 64), Wp = __shfl_up(W, d, 64);
    if (lane >= d) {
      W = P * Wp + W;
      P = P * Pp;
    }
  }
  double Win = __shfl_up(W, 1, 64);
  if (lane == 0) Win = 0.0;
  P = 1.0;
#pragma unroll
  for (int k = 0; k < PD_ANG_BMAX; ++k) {
    if (k < cnt) {
      P *= -ld(KS.af_f, row + j0 + k);
      wl[k] += P * Win;
    }
  }
  double X = 0.0, Q = 1.0;
#pragma unroll
  for (int k = PD_ANG_BMAX - 1; k >= 0; --k) {
    if (k < cnt) {
      const double g = ld(KS.af_g, row + j0 + k);
      X = wl[k] - g * X;
      Q *= -g;
      wl[k] = X;
    }
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double Qn = __shfl_down(Q, d, 64), Xn = __shfl_down(X, d, 64);
    if (lane + d < 64) {
      X = Q * Xn + X;
      Q = Q * Qn;
    }
  }
  double Xin = __shfl_down(X, 1, 64);
  if (lane == 63) Xin = 0.0;
  Q = 1.0;
  double ylast = 0.0;
#pragma unroll
  for (int k = PD_ANG_BMAX - 1; k >= 0; --k) {
    if (k < cnt) {
      Q *= -ld(KS.af_g, row + j0 + k);
      wl[k] += Q * Xin;
      if (j0 + k == n - 1) ylast = wl[k];
    }
  }
  const int llast = (n - 1) / B;
  const double y0 = __shfl(wl[0], 0, 64);
  const double yl = __shfl(ylast, llast, 64);
  const double sfac = I.af_kappa[i - 1] * (y0 - I.af_alpha0[i - 1] * yl);
#pragma unroll
  for (int k = 0; k < PD_ANG_BMAX; ++k) {
    if (k < cnt) {
      const int idx = row + j0 + k;
      out[idx] = (T)(wl[k] - sfac * ld(KS.af_z, idx));
    }
  }
}

// ------------------------------------------------------------ update kernel
//
// x += α p̂ + ω ŝ (x = ... on the first inner iteration of a refinement),
// r = s - ω t, partials r̂·r and r·r; the last block decides convergence,
// breakdown or restart for the instance.

template <typename T>
__global__ __launch_bounds__(256) void k_elem_x(const PdInst *insts, const int2 *map) {
  const int2 mp = map[blockIdx.x];
  const PdInst &I = insts[mp.x];
  PdScalars *sc = I.sc;
  if (!inner_active(sc) || !prec_match<T>(I)) return;
  const KSet<T> &KS = kset<T>(I);
  T *x = iterate_ptr<T>(I, sc);
  const double al = sc->alpha, om = sc->omega;
  const bool setx = sc->inner_first;
  const int N = I.m * I.n + 1;
  double acc[2] = {0.0, 0.0};
  const int base = mp.y * PD_ELEM_PER_BLOCK;
#pragma unroll
  for (int k = 0; k < PD_ELEM_PER_BLOCK / 256; ++k) {
    const int idx = base + k * 256 + threadIdx.x;
    if (idx < N) {
      const double dx = al * ld(KS.ph, idx) + om * ld(KS.sh, idx);
      x[idx] = (T)(setx ? dx : ld(x, idx) + dx);
      const T rs = (T)(ld(KS.s, idx) - om * ld(KS.t, idx));
      KS.r[idx] = rs;
      const double rd = (double)rs;
      acc[0] += ld(KS.rh, idx) * rd;
      acc[1] += rd * rd;
    }
  }
  double tot[2];
  if (block_commit<2>(acc, I.partials, I.nb_elem, mp.y, I.counters + CNT_X, tot) &&
      threadIdx.x == 0) {
    const double rr = tot[1];
    sc->iters += 1;
    sc->inner_iters += 1;
    sc->inner_first = 0;
    sc->rho_old = sc->rho_new;
    sc->rho_new = tot[0];
    sc->rnorm2 = rr;
    if (!(rr == rr) || !(tot[0] == tot[0])) {
      finish_instance(I, sc, ST_BREAKDOWN);
      return;
    }
    if (!I.mixed) {
      sc->rel_resid = sqrt(rr / sc->bnorm2);
      if (rr <= sc->tol * sc->tol * sc->bnorm2) {
        finish_instance(I, sc, ST_DONE);
        return;
      }
      if (sc->iters >= sc->maxit) {
        finish_instance(I, sc, ST_NOCONV);
        return;
      }
    } else {
      if (rr <= sc->tol_inner * sc->tol_inner * sc->r0norm2 || sc->inner_iters >= sc->maxit_inner ||
          sc->iters >= sc->maxit) {
        sc->phase = PH_OUTER;
      }
    }
    if (sc->reset_rh || fabs(tot[0]) <= 1e-30 * rr) {
      // restart from the current iterate: r̂ = r, p = r
      sc->reset_rh = 1;
      sc->restarts += 1;
      sc->rho_new = rr;
      if (sc->restarts > 50) finish_instance(I, sc, ST_BREAKDOWN);
    }
  }
}

// Clears the restart flag after the radial sweep that consumed it; resets
// counters of an instance after an aborted launch.
__global__ void k_clear_reset(PdInst *insts, int ninst) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ninst) return;
  insts[q].sc->reset_rh = 0;
}

}  // namespace pd

// ------------------------------------------------------------ launchers

#include "pd_launch.h"

namespace pd {

KTimer *g_timer = nullptr;

static inline dim3 g1(int n) { return dim3((unsigned)n); }

struct Mark {
  int f;
  hipStream_t s;
  Mark(int fam, hipStream_t st) : f(fam), s(st) {
    if (g_timer) g_timer->mark(f, true, s);
  }
  ~Mark() {
    if (g_timer) g_timer->mark(f, false, s);
  }
};
enum { KF_BEGIN = 0, KF_FACTOR = 1, KF_RAD = 2, KF_ANG = 3, KF_STEN_V = 4, KF_STEN_T = 5,
       KF_UPDATE = 6, KF_REFINE = 7, KF_CONTROL = 8 };

void launch_level_begin(const LaunchSet &L, hipStream_t s) {
  Mark mk(KF_CONTROL, s);
  k_level_begin<<<(L.ninst + 63) / 64, 64, 0, s>>>(L.insts, L.ninst);
}
void launch_level_end(const LaunchSet &L, hipStream_t s) {
  Mark mk(KF_CONTROL, s);
  k_level_end<<<(L.ninst + 63) / 64, 64, 0, s>>>(L.insts, L.ninst);
}
void launch_factor(const LaunchSet &L, hipStream_t s) {
  Mark mk(KF_FACTOR, s);
  if (L.nb_frad) k_fact_rad<<<g1(L.nb_frad), 64, 0, s>>>(L.insts, L.map_frad);
  if (L.nb_fang) k_fact_ang<<<g1(L.nb_fang), 64, 0, s>>>(L.insts, L.map_fang);
}
void launch_begin(const LaunchSet &L, hipStream_t s) {
  Mark mk(KF_BEGIN, s);
  k_sten<double, SM_BEGIN><<<g1(L.nb_sten), 256, 0, s>>>(L.insts, L.map_sten, 0, 0, nullptr, nullptr);
}

template <typename T>
static void cycle_t(const LaunchSet &L, hipStream_t s) {
  { Mark mk(KF_RAD, s); k_rad<T, RM_P><<<g1(L.nb_rad), PD_RAD_THREADS, 0, s>>>(L.insts, L.map_rad, nullptr, nullptr); }
  { Mark mk(KF_CONTROL, s); k_clear_reset<<<(L.ninst + 63) / 64, 64, 0, s>>>(L.insts, L.ninst); }
  { Mark mk(KF_ANG, s); k_ang<T, AM_P><<<g1(L.nb_ang), 256, 0, s>>>(L.insts, L.map_ang, nullptr, nullptr); }
  { Mark mk(KF_STEN_V, s); k_sten<T, SM_V><<<g1(L.nb_sten), 256, 0, s>>>(L.insts, L.map_sten, 0, 0, nullptr, nullptr); }
  { Mark mk(KF_RAD, s); k_rad<T, RM_S><<<g1(L.nb_rad), PD_RAD_THREADS, 0, s>>>(L.insts, L.map_rad, nullptr, nullptr); }
  { Mark mk(KF_ANG, s); k_ang<T, AM_S><<<g1(L.nb_ang), 256, 0, s>>>(L.insts, L.map_ang, nullptr, nullptr); }
  { Mark mk(KF_STEN_T, s); k_sten<T, SM_T><<<g1(L.nb_sten), 256, 0, s>>>(L.insts, L.map_sten, 0, 0, nullptr, nullptr); }
  { Mark mk(KF_UPDATE, s); k_elem_x<T><<<g1(L.nb_elem), 256, 0, s>>>(L.insts, L.map_elem); }
}

void launch_cycle(const LaunchSet &L, hipStream_t s) {
  if (L.mixed_any) {
    Mark mk(KF_REFINE, s);
    k_sten<float, SM_UR><<<g1(L.nb_sten), 256, 0, s>>>(L.insts, L.map_sten, 0, 0, nullptr, nullptr);
  }
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
  if (fp32)
    k_sten<float, SM_APPLY><<<g1(L.nb_sten), 256, 0, s>>>(L.insts, L.map_sten, dt, th,
                                                          (const float *)x, (float *)y);
  else
    k_sten<double, SM_APPLY><<<g1(L.nb_sten), 256, 0, s>>>(L.insts, L.map_sten, dt, th,
                                                           (const double *)x, (double *)y);
}

void launch_precond_plain(const LaunchSet &L, const double *x, double *tmp, double *y,
                          hipStream_t s) {
  k_rad<double, RM_PLAIN><<<g1(L.nb_rad), PD_RAD_THREADS, 0, s>>>(L.insts, L.map_rad, x, tmp);
  k_ang<double, AM_PLAIN><<<g1(L.nb_ang), 256, 0, s>>>(L.insts, L.map_ang, tmp, y);
}

}  // namespace pd
