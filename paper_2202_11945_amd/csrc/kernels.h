// Launch interface of the gfx950 kernels (kernels.hip).
#pragma once

#include "fewha_internal.h"

namespace fewha {

// source of the inverse transform (SRC_PJ: the search direction p_j as
// formed by the augmented PCG's direction kernel; problems with augmentation
// take it in place of SRC_PUPD0 / SRC_PUPD)
enum { SRC_IN = 0, SRC_STATE_C = 1, SRC_PUPD0 = 2, SRC_PUPD = 3, SRC_PJ = 4 };
// destination of the inverse transform
enum { OUT_PHI = 0, OUT_USER = 1, OUT_FIT = 2 };
// epilogue of the forward transform
enum { EPI_APPLYM = 0, EPI_PCG = 1, EPI_RHS = 2, EPI_PLAIN = 3, EPI_RHSQ = 4 };
// propagation + Shack-Hartmann output
//   PG_COMPACT : io.in -> compact slopes in io.out      (A x)
//   PG_DENSE   : phi -> slope buffer (row-span layout) + tip/tilt partials (inside M)
//   PG_DENSE_IN: io.in -> slope buffer + partials
//   PG_RESID_IN: slope buffer -= Gamma P io.in, + partials (data residual s - A x)
//   PG_POL_IN  : slope buffer = compact io.in + Gamma P a_prev (state), + partials
//                (closed loop: pseudo-open-loop slopes, two-step delay)
//   PG_APREV   : slope buffer = Gamma P a_prev (state), + partials (the mirrors'
//                part of the pseudo-open-loop slopes, before the measurement arrives)
enum { PG_COMPACT = 0, PG_DENSE = 1, PG_DENSE_IN = 2, PG_RESID_IN = 3, PG_POL_IN = 4, PG_APREV = 5 };
// Shack-Hartmann adjoint weighting
enum { GT_PLAIN = 0, GT_WEIGHTED = 1 };
// propagation adjoint destination
enum { PT_PHIADJ = 0, PT_USER = 1 };
// DM fitting CG phases
enum { FIT_INIT = 0, FIT_ITER = 1, FIT_FINAL = 2 };

struct LaunchArgs {
  const ProbDev* P;
  const LayerDev* L;
  const WfsDev* W;
  const IoDev* IO;
  Filter F;
  hipStream_t stream;
  int res_max;  // largest resident transform side of the plan (32, 64 or 128)
  const HatEnt* hats;     // hat tables of the propagation adjoint (plan-wide)
  int n_hats;             // entries of hats
  const BandRec* bands;   // band records of the propagation adjoint (plan-wide)
  const PtEnt* pents;     // sensor lists of the propagation-adjoint tiles (plan-wide)
  const int2* pgrows;     // propagation-stage tiles: per layer, (cell row, fraction) of the 17 window rows,
                          // then (cell column, fraction) of the 17 columns, at tile.level
  const int2* gtrows;     // Shack-Hartmann adjoint tiles: per window row (span base << 1 | active flag
                          // of window column 32, active flags of window columns 0 .. 31), at tile.level
  int pt_rows;         // node rows per thread of the propagation adjoint (4 or 8)
  int pt_wide;         // 1: some pair has K > 3 corners per node (the kernel with wide records)
  int pt_split;        // 1: tiles of one band record, the sensor list split over the waves
  int glob_fuse;       // 1: the last two global levels of a layer run as one tile (inverse transform)
};

void launch_idwt_res(const LaunchArgs& a, const Tile* tiles, int ntiles, int src_mode, int out_mode, int iter);
// the resident inverse levels over four workgroups per (problem, layer): tile.tx = quadrant
void launch_idwt_res4(const LaunchArgs& a, const Tile* tiles, int ntiles, int src_mode, int out_mode, int iter);
void launch_idwt_glob(const LaunchArgs& a, const Tile* tiles, int ntiles, int src_mode, int out_mode, int iter,
                      int step);
void launch_fdwt_glob(const LaunchArgs& a, const Tile* tiles, int ntiles, int epi, int iter, int step);
void launch_fdwt_res(const LaunchArgs& a, const Tile* tiles, int ntiles, int epi, int iter);
void launch_pgamma(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode);
// compact slopes io.in -> slope buffer + tip/tilt partials; add = 1: added to the
// buffer's current values (closed loop after PG_APREV)
void launch_slopes_in(const LaunchArgs& a, const Tile* tiles, int ntiles, int add = 0);
void launch_gammaT(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode);
void launch_pT(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode);
// x update of a PCG step: x += a_k p_k (ONE); none, left to the next step
// (DEFER); x += a_{k-1} p_{k-1} + a_k p_k, the previous step's deferred one
// first (PAIR; iter >= 1, C null)
enum { UPD_X_ONE = 0, UPD_X_DEFER = 1, UPD_X_PAIR = 2 };
// C: the coarse-level correction of a converged solve (rho includes it), else null
void launch_update(const LaunchArgs& a, const Tile* tiles, int ntiles, int iter, const CoarseDev* C = nullptr,
                   int xm = UPD_X_ONE);
// converged solves' coarse-level correction: y = E^{-1} Z^T r_k (tiles: problem x row block)
void launch_coarse(const LaunchArgs& a, const CoarseDev* C, const Tile* tiles, int ntiles, int k);
// p_k = J^{-1} r_k + Z y + beta_k p_{k-1} over the vector-update chunks
void launch_coarse_p(const LaunchArgs& a, const CoarseDev* C, const Tile* tiles, int ntiles, int iter);
// set-up of E = Z^T M Z, round t: unit vectors (store = false) or columns (store = true)
void launch_coarse_probe(const CoarseProbe* Q, int nprob, int t, bool store, hipStream_t s);
void launch_solve_init(const LaunchArgs& a, const Tile* tiles, int ntiles);
void launch_grad_height(const LaunchArgs& a, const Tile* tiles, int ntiles, int term);
void launch_grad_prior(const LaunchArgs& a, const GradIo* g, const Tile* tiles, int ntiles);
void launch_grad_final(const LaunchArgs& a, const GradIo* g, int nprob);
// Work lists of the FP64 residual chain (residual64.hip).
struct Resid64Tiles {
  const Tile* upd = nullptr;             // coefficient chunks (the vector-update list)
  int upd_n = 0;
  int n_steps = 0;                       // transform levels (max over layers)
  const Tile* inv[kMaxLevelsJ] = {};     // synthesis step s: blocks of side (n >> levels) << (s + 1)
  int inv_n[kMaxLevelsJ] = {};
  const Tile* fwd[kMaxLevelsJ] = {};     // analysis step s: blocks of side n >> s
  int fwd_n[kMaxLevelsJ] = {};
  const Tile* pg = nullptr;              // subaperture tiles
  int pg_n = 0;
  const Tile* wfs = nullptr;             // one per (problem, sensor)
  int wfs_n = 0;
  const Tile* gt = nullptr;              // corner tiles
  int gt_n = 0;
  const Tile* pt = nullptr;              // node tiles
  int pt_n = 0;
};

// r = b - M x64 in FP64 (io.in = b, io.out = r) + partial sums of r^2, b^2
void launch64_resid_chain(const LaunchArgs& a, const Resid64Tiles& rt, const Filter64& F);
// x64 = 0 (mode 0), x64 += io.in (1), io.state = (float) x64 (2)
void launch64_iterate(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode);
// augmented PCG over the vector-update chunks of augmented problems:
// partial sums of W^T r_0 and W^T A W; the projected start (x_0, r_0, rho_0,
// (A W)^T z_0); the direction p_j; the frame's directions into the state
void launch_aug_gram(const LaunchArgs& a, const Tile* tiles, int ntiles);
void launch_aug_init(const LaunchArgs& a, const Tile* tiles, int ntiles);
void launch_aug_p(const LaunchArgs& a, const Tile* tiles, int ntiles, int iter);
void launch_aug_store(const LaunchArgs& a, const Tile* tiles, int ntiles, int iters);
void launch_fit_fwd(const LaunchArgs& a, const Tile* tiles, int ntiles);
void launch_fit_cg(const LaunchArgs& a, const FitDev* F, int nfit, int phase);

}  // namespace fewha
