// Launch interface of the gfx950 kernels (kernels.hip).
#pragma once

#include "fewha_internal.h"

namespace fewha {

// source of the inverse transform
enum { SRC_IN = 0, SRC_STATE_C = 1, SRC_PUPD0 = 2, SRC_PUPD = 3 };
// destination of the inverse transform
enum { OUT_PHI = 0, OUT_USER = 1, OUT_FIT = 2 };
// epilogue of the forward transform
enum { EPI_APPLYM = 0, EPI_PCG = 1, EPI_RHS = 2, EPI_PLAIN = 3 };
// propagation + Shack-Hartmann output
enum { PG_COMPACT = 0, PG_DENSE = 1 };
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
};

void launch_idwt_res(const LaunchArgs& a, const Tile* tiles, int ntiles, int src_mode, int out_mode, int iter);
void launch_idwt_glob(const LaunchArgs& a, const Tile* tiles, int ntiles, int src_mode, int out_mode, int iter,
                      int step);
void launch_fdwt_glob(const LaunchArgs& a, const Tile* tiles, int ntiles, int epi, int iter, int step);
void launch_fdwt_res(const LaunchArgs& a, const Tile* tiles, int ntiles, int epi, int iter);
void launch_pgamma(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode);
void launch_slopes_in(const LaunchArgs& a, const Tile* tiles, int ntiles);
void launch_gammaT(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode);
void launch_pT(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode);
void launch_update(const LaunchArgs& a, const Tile* tiles, int ntiles, int iter);
void launch_fit_fwd(const LaunchArgs& a, const Tile* tiles, int ntiles);
void launch_fit_cg(const LaunchArgs& a, const FitDev* F, int nfit, int phase);

}  // namespace fewha
