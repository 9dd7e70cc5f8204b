// Launch interface between the host runtime and the HIP kernels.
#pragma once

#include "pd_device.h"

namespace pd {

#define PD_MG_MAXLEV 12   // coarse θ-levels of a multigrid preconditioner (2048 lines need 8)

struct MgSet;

// Device-side description of one batched launch: the instance array and,
// per kernel family, a block map (instance index, block index within it).
struct LaunchSet {
  PdInst *insts = nullptr;
  int ninst = 0;
  int2 *map_sten = nullptr, *map_elem = nullptr, *map_rad = nullptr, *map_ang = nullptr;
  int nb_sten = 0, nb_elem = 0, nb_rad = 0, nb_ang = 0;
  int mixed_any = 0, fp64_any = 0;
  int adaptive_any = 0;             // some instance steps adaptively (level-end pass in the round head)
  int max_bang = 1;                 // longest angular lane span of the batch (factorisation)
  int max_bang1 = 1;                // longest lane span of the one-wave ring sweeps
  // ring sweeps: [0] one wave per ring (4 rings per block), [1] rings of 2 or
  // 4 waves (4/aw rings per block)
  int2 *map_angs[2] = {nullptr, nullptr};
  int nb_angs[2] = {0, 0};
  int max_bfrad = 1;                // longest radial segment of the factorisation
  // Radial sweeps, three classes by ring count (rad_class).  The class
  // depends on the instance alone, so its arithmetic does not depend on the
  // rest of the batch.
  int2 *map_rs[3] = {nullptr, nullptr, nullptr};
  int nb_rs[3] = {0, 0, 0};
  int max_brs[3] = {1, 1, 1};       // longest radial segment per class
  // the multigrid preconditioners of the plan's instances that use one
  // (then every instance of the plan is FP64)
  const MgSet *const *mg = nullptr;
  int nmg = 0;
};

// Launches of a θ-semi-coarsening V-cycle (PdMgLevel) for one FP64
// instance: per level a launch set of its line sweeps (level 0: the
// instance's own factors with the V-cycle's vectors; level l: the level's
// faces and factors), all gated on the instance's scalars.
struct MgSet {
  int nlev = 0;                      // coarse θ-levels 1..nlev (the ring means below)
  int m = 0;
  int n[PD_MG_MAXLEV + 1] = {};      // θ-lines per level
  LaunchSet lev[PD_MG_MAXLEV + 1];
  const PdMgLevel *dlev = nullptr;   // device [nlev + 1]
  const PdScalars *sc = nullptr;     // the instance's scalars
  const double *crs = nullptr;       // its ring sums (the ring-mean system)
  double *btot = nullptr, *cring = nullptr;   // ring totals and ring-mean correction [m + 1]
  // the instance's Krylov vectors: inputs p, s (and r for a diagnostic
  // application), outputs p̂, ŝ
  const double *p = nullptr, *s = nullptr, *r = nullptr;
  double *ph = nullptr, *sh = nullptr;
};

// Radial-sweep classes: 512-thread blocks of 16 columns x 32 segments for
// m <= 256; 1024-thread blocks of 16 columns x 64 segments for m <= 512;
// above, 1024-thread blocks of 8 columns x 128 segments, whose segments stay
// short enough for registers and which give twice the blocks.
inline int rad_class(int m) { return m <= 256 ? 0 : (m <= 512 ? 1 : 2); }
inline int rad_threads_of(int c) { return c == 0 ? 512 : 1024; }
inline int rad_cols_of(int c) { return c == 2 ? 8 : 16; }
inline int rad_rows(int m) {
  const int c = rad_class(m), seg = rad_threads_of(c) / rad_cols_of(c);
  return (m + seg - 1) / seg;
}
inline int rad_blocks(int m, int n) { return (n + rad_cols_of(rad_class(m)) - 1) / rad_cols_of(rad_class(m)); }

// Optional per-family event timing of launches (diagnostics).
struct KTimer {
  // Two events that the next launch of `family` stamps with its own start
  // and end (hipExtLaunchKernel), so that their difference is the kernel's
  // execution time alone.
  virtual bool pair(int family, hipEvent_t *start, hipEvent_t *stop) = 0;
  virtual ~KTimer() {}
};
extern KTimer *g_timer;

void launch_level_begin(const LaunchSet &L, hipStream_t s);
void launch_ctl(const LaunchSet &L, hipStream_t s);
void launch_level_end(const LaunchSet &L, hipStream_t s);
void launch_round(const LaunchSet &L, int cycles, hipStream_t s);
void launch_factor(const LaunchSet &L, hipStream_t s);
void launch_begin(const LaunchSet &L, hipStream_t s);
void launch_begin_origin(const LaunchSet &L, hipStream_t s);
// Faces, angular widths and reaction of multigrid level l+1 (nc lines) from
// level l of the device descriptors.
void launch_mg_faces(const PdMgLevel *dlev, int l, int m, int nc, double *gp_r, double *gm_r, double *gp_t,
                     double *gm_t, double *inv_dth, double *b_node, hipStream_t s);
void launch_cycle(const LaunchSet &L, hipStream_t s);
void launch_precond_apply(const LaunchSet &L, int fp32, hipStream_t s);
void launch_apply(const LaunchSet &L, double dt, double th, const void *x, void *y, int fp32,
                  hipStream_t s);
// Coupled carriers: drift faces from a potential (and the ring sums and
// origin diagonal that depend on them), a difference of two vectors, and
// max |a - b|, max |a| (out[0], out[1]; part: 2 nblk doubles).
void launch_drift(int m, int n, int flux, const double *G_r, const double *c_r, const double *G_t,
                  const double *c_t, const double *psi, const double *nb, const double *lam, const int *tpow,
                  int nsrc, double *gp_r, double *gm_r, double *gp_t, double *gm_t, double *crs, double inv_V0,
                  double b0, double *l0, hipStream_t s);
void launch_sub(const double *a, const double *b, double *out, int N, hipStream_t s);
void launch_maxdiff(const double *a, const double *b, int N, double *part, int nblk, double *out,
                    hipStream_t s);
void launch_indicator(const double *x, int m, int n, const double *r, const double *th,
                      const double *nb, const double *lam, const int *tpow, int nsrc, double t,
                      int dirichlet, double *ring_out, double *eta_out, hipStream_t s);
void launch_transfer(const double *x, int m, int n, const double *r, const double *th, const double *nb,
                     const double *lam, const int *tpow, int nsrc, double t, int dirichlet,
                     const double *r2, const double *th2, int m2, int n2, double *y, hipStream_t s);

}  // namespace pd
