// Internal data structures shared by the host set-up, the plan builder and
// the gfx950 kernels.  Everything a kernel reads is flat POD in device
// memory; per-problem buffers are carved out of one arena per plan.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fewha.h"

namespace fewha {

constexpr int kMaxLevelsJ = 16;   // j index range of the per-layer prior table
constexpr int kResMax = 128;      // largest block kept resident in LDS by the DWT kernels (default residency)
constexpr int kTileS = 16;        // subaperture / corner tile side of the sensor stages
constexpr int kGtS = 32;          // corner tile side of the noise-weighted sensor adjoint (4 corners per thread)
constexpr int kTileN = 32;        // node tile side of the FP64 propagation adjoint
constexpr int kPtW = 64;          // propagation adjoint tile: 64 node columns (one per lane) by
                                  // 4 x rows-per-thread node rows (tuning: 4 or 8 rows per thread)
// Corner rows (band) that rpt consecutive node rows of the propagation adjoint
// may touch with K corners per node: consecutive first corners differ by at
// most one (K = 2: corner spacing >= node spacing) or two (K = 3: spacing
// >= 2/3 of it); the host checks every row group against this bound.
constexpr int pt_band(int K, int rpt) { return K == 2 ? rpt + 2 : (3 * (rpt - 1)) / 2 + K + 2; }
constexpr int kBandRows = 4;                    // node rows of one band record
constexpr int kBandMax = pt_band(3, kBandRows);  // corner rows of the widest band
// Sensors sampling a layer finer than 2/3 of its spacing (rho in [1/3, 2/3))
// have K = 4, 5 or 6 corners per node and axis ("wide" pairs).  Consecutive
// first corners then differ by at most ceil(1 / rho), so kBandRows node rows
// touch at most ceil(3 / rho) + K corner rows: 10, 13 or 15.
constexpr int kWideMaxK = 6;
constexpr int pt_band_wide(int K) { return K == 4 ? 10 : (K == 5 ? 13 : 15); }
constexpr int kBandWideMax = pt_band_wide(kWideMaxK);
constexpr int kUpdChunk = 2048;   // coefficients per workgroup of the vector update
constexpr int kDotRing = 256;     // PCG iterations whose inner products are kept (ring, power of two)
constexpr int kGradChunk = 2048;  // coefficients per workgroup of the prior-term reductions
constexpr double kTie = 1e-9;     // |t - round(t)| below which a sample sits on a grid line
// Augmented PCG: at most kAugMax previous search directions per problem.
// FP64 partial-sum groups (one slot per vector-update chunk) of a frame:
// W^T r_0 (kAugMax), the lower triangle of W^T A W (row r, column k <= r:
// group r (r + 1) / 2 + k), rho_0 of the projected residual, and
// (A W)^T z_j for the two iteration parities.
constexpr int kAugMax = 4;
constexpr int kAugD = 0;
constexpr int kAugG = kAugD + kAugMax;
constexpr int kAugRho0 = kAugG + kAugMax * (kAugMax + 1) / 2;
constexpr int kAugT = kAugRho0 + 1;
constexpr int kAugGroups = kAugT + 2 * kAugMax;
constexpr int kAugFac = kAugMax * kAugMax + kAugMax;  // doubles: Cholesky factor, then the kept flags

// db3 analysis filters, passed by value to the transform kernels.
struct Filter {
  float h[6];
  float g[6];
};

// One layer of one problem.
struct LayerDev {
  int n, log2n, levels, res;  // res = min(n, kResMax)
  int off;                    // offset of the layer in N_c-sized vectors
  int tmp_off;                // offset of the layer's coarse-block scratch
  int n_glob_levels;          // levels with output side > kResMax
  int pad0;
  float inv_delta;            // 1 / delta_l
  float alpha_d[kMaxLevelsJ]; // alpha * D_j, j = log2(block side)
  // parameter gradients
  double d64[kMaxLevelsJ];    // D_j in FP64
  double cn2;                 // gamma_l
  int gp_off, gp_n;           // prior-term slots of this layer (from the start of the slot array)
  int gh_off, gh_n;           // height-term slots of this layer (from the start of one term's range)
  double inv_delta64;         // 1 / delta_l (residual in FP64)
};

// One sensor of one problem.
struct WfsDev {
  int N, nc;            // subapertures per side, corners per side
  int lgs, tt;          // laser guide star, tip/tilt removal
  int blocks;           // 1 = 2x2 block noise weights present
  int n_active;
  int s_off;            // dense FP64 slopes of the refined solves' residual: [s^x N*N | s^y N*N] at s_off
  int v_off;            // corner grids: nc*nc at v_off
  int cs_off;           // compact slopes of this sensor within the problem's slope vector
  int m_off;            // N*N compact-index map at m_off (-1 = inactive)
  int cinv_off;         // 3 floats (a, b, c) per subaperture at cinv_off (blocks only)
  int part_off;         // 4 floats per P-Gamma tile at part_off
  int n_tiles_s;        // tiles of the subaperture grid (= partial slots)
  int tiles_side;       // tiles per side of the subaperture grid
  int tab_off;          // per layer: interp/adjacency tables at tab_off + l * tab_stride
  int tab_stride;
  int gtab_off;         // per layer: derivative tables at gtab_off + l * 4 nc (gitab / gftab)
  int sp_off;           // FP32 slopes in row-span layout: [s^x | s^y] at sp_off, sp_len entries each,
  int sp_len;           //   row i holding its columns lo_i .. hi_i (the first and last active ones)
  int rb_off;           // row bases at rb_off of the problem's srow: subaperture (i, j) at srow[rb_off + i] + j
  float inv_sigma2;
  float inv_nM;
  float sum_cinv[4];    // sum over the mask of the 2x2 inverse blocks (row-major)
  double inv_sigma2_d;  // FP64 copies for the residual of refined solves
  double inv_nM_d;
};

// Per-(sensor, layer) table layout inside the int/float table arrays, relative
// to WfsDev::tab_off + l * tab_stride (tab_stride = 4 nc):
//   int   q0y[nc], q0x[nc]   bilinear cell of each corner row / column
//   float wy[nc],  wx[nc]    fractional offsets (float slots [2nc, 4nc))
// Derivative tables (gradient with respect to the layer height), relative to
// WfsDev::gtab_off + l * 4 nc:
//   int   qy[nc], qx[nc], tiey[nc], tiex[nc]   cell (the node itself on a grid line)
//   float wy[nc], wx[nc], dty[nc], dtx[nc]     fraction (0 on a grid line), dt/dh

// Propagation of one (sensor, layer) pair in node units: corner k of the
// sensor sits at t = t0 + k rho along each axis (rho = cone factor x pitch /
// layer spacing) and its bilinear weight on node p is the hat function
// max(0, 1 - |t - p|).  kmax = most corners within one node spacing of a
// node along an axis (2 when rho >= 1, 3 when rho >= 2/3, 4, 5, 6 when rho >=
// 1/2, 2/5, 1/3; 0 = finer, or a band that does not fit: general gather).
struct GLPar {
  double t0y, t0x, rho, inv_rho;
  int nc, v_off, kmax;
  int hat_off;   // hat tables of this pair: [rows n][columns n] HatEnt in the plan's hat array
  int band_off;  // band records of this pair (one per kBandRows node rows) in the plan's band array
  int pad_;
};

// The corners of one node along one axis: corner lo + k has weight w[k]
// (k < K = kmax; lo clamped so that lo + K - 1 < nc, unused weights 0);
// a node that no corner's cell touches has all weights 0 and lo =
// clamp(floor(c), 0, nc - K), so lo never decreases along an axis.  A wide
// pair (K > 3) has two entries per node: the second holds w[3 .. 5] (its lo
// repeats the first's).
struct HatEnt {
  int lo;
  float w[3];
};
static_assert(sizeof(HatEnt) == 16, "one 16-byte load per lane");

// Separable propagation adjoint of kBandRows consecutive node rows and one
// (sensor, layer) pair.  The band is a run of consecutive corner rows of the
// sensor's grid starting at row base (so0 = base nc 4, its byte offset).
// pat says how the first corners of the node rows step:
//   0 .. 7    : a step pattern.  base is the first node row's first corner;
//               bit u - 1 of pat is the step from node row u - 1 to u less
//               its least value (K = 2: steps 0 or 1, K = 3: 1 or 2), so node
//               row u reads the K band rows from d_u = sum of the steps, with
//               the weights wk[u][0 .. K - 1] (its y hat).
//   kPatZero  : every weight is zero (the rows lie outside the sensor's reach).
//   kPatDense : any other steps (grid edges, a short last group); band rows
//               base .. base + nrows - 1, all inside the grid, and node row u
//               weights band row s by w[u][s].
constexpr int kPatZero = 8, kPatDense = 9;
struct BandRec {
  int so0, pat, nrows, pad_;
  float wk[kBandRows][3];
  float w[kBandRows][kBandMax];
  int pad2_[12];
};
static_assert(sizeof(BandRec) == 256, "band record: 64 dwords");
// The band record of a wide pair, in the same 256 bytes of the band array:
// always dense (pat kPatDense or kPatZero), node row u weighting band row s
// by w[u][s].
struct BandRecW {
  int so0, pat, nrows, pad_;
  float w[kBandRows][kBandWideMax];
};
static_assert(sizeof(BandRecW) == sizeof(BandRec), "wide band record: 64 dwords");

// One sensor of a propagation-adjoint tile's list (the sensors whose
// footprint meets the tile, in sensor order), all a wave needs for it:
//   v_off : the sensor's corner grid in the problem's corner array
//   nck   : K > 0: corner grid side nc << 3 | K;
//           K = 0 (general gather): index of the pair's GLPar << 3
//   hx    : K > 0: hat-table index of the tile's first node column (its
//           first entry: two per node of a wide pair), else 0
//   band  : K > 0: band record of the tile's first kBandRows node rows, else 0
// Every list ends with one more entry {0, 2, 0, 0} that is never run (the
// sensor loop prefetches one entry ahead); the hat and band arrays hold at
// least 64 and 8 entries, so every prefetch address is valid.
struct PtEnt {
  int v_off, nck, hx, band;
};
static_assert(sizeof(PtEnt) == 16, "one 16-byte scalar load per sensor");

// One problem.
struct ProbDev {
  int L, G;
  int layer0, wfs0;        // first LayerDev / WfsDev index
  int n_c;                 // coefficients = layer nodes
  int n_slopes;            // compact slopes
  int n_act;
  int n_dots;              // dot-product slots per group
  int n_slots_fdwt;        // producers of rho_0 and pi_k
  int n_slots_upd;         // producers of rho_{k+1}
  int fitted;              // 1 = the DM commands come from the fitting step
  int closed;              // 1 = closed loop (pseudo-open-loop slopes, closed-loop control)
  float gain;
  float pad2;
  // internal buffers
  float* phi;      // layers (FE domain) N_c
  float* phiadj;   // A^T ... result N_c
  float* tmpa;     // coarse-block scratch (ping)
  float* tmpb;     // coarse-block scratch (pong)
  float* sd;       // slopes of the sensor stages (row-span layout, WfsDev::sp_off)
  float* vadj;     // corner-grid adjoint values
  float* part;     // tip/tilt partial sums
  float* pbuf0;    // search direction (ping)
  float* pbuf1;    // search direction (pong)
  float* q;        // M p
  double* dots;    // [group][n_dots] partial inner products
  const float* jinv;     // 1 / J
  const int* itab;       // int tables
  const float* ftab;     // float tables
  const int* cmap;       // compact-index maps
  const unsigned char* amap;  // active flags (1 byte per subaperture, the maps' layout)
  const int* srow;       // row bases of the row-span slope layout (WfsDev::rb_off)
  const float* cinv;     // 2x2 inverse noise blocks
  const GLPar* gl;       // [sensor][layer] propagation parameters
  // parameter gradients
  float* gphi;           // W^{-1} c
  float* glam;           // W^{-1} lambda
  double* gslots;        // [prior terms n_gp | height term 0 n_gh | height term 1 n_gh]
  const int* gitab;      // derivative tables
  const float* gftab;
  int n_gp, n_gh;
  double alpha;
  // FP64 residual b - M x of refined solves
  double* a64;           // N_c: coefficients -> layers -> adjoint -> coefficients
  double* b64;           // N_c: pass scratch
  double* sd64;          // slopes on the dense N x N grids (WfsDev::s_off)
  double* u64;           // corner grids, as vadj
  double* rslots;        // [upd slot][2]: sum r^2, sum b^2
  const double* cinv64;  // 2x2 inverse noise blocks, as cinv
  const double* ftab64;  // interpolation fractions, as ftab
  float* rbuf;           // N_c: residual (right-hand side of a correction solve)
  double* x64;           // N_c: the refined iterate
  // numerical-breakdown flag of the plan (host-mapped pinned memory): a
  // PCG step that finds p^T M p <= 0 with a nonzero residual, or a
  // non-finite or negative inner product, stores the problem index + 1
  int* numflag;
  // augmented PCG (Sec. 3.3): directions of the previous frame in the state
  // after a_prev / a (aug_keep of them, then their images, then a count),
  // this frame's first aug_keep directions and images, FP64 partial sums and
  // the factor of W^T A W
  int aug_keep;            // 0 = plain PCG
  int aug_pad;
  float* aug_pdir;         // aug_keep x N_c
  float* aug_qdir;         // aug_keep x N_c
  double* aug_slots;       // kAugGroups x n_slots_upd
  double* aug_fac;         // kAugFac
};

// db3 filters in FP64 for the residual transforms.
struct Filter64 {
  double h[6];
  double g[6];
};

// Per-call pointers of the parameter-gradient reductions of one problem.
struct GradIo {
  const float* c;
  const float* lam;
  double* out;  // [g_alpha | g_cn2 (L) | g_h (L)]
};

// Per-call input/output pointers of one problem.
struct IoDev {
  const float* in;     // slopes (reconstruct, apply_AT, rhs), layers (apply_A), c (apply_M)
  float* out;          // apply_* outputs
  float* state;        // [c | b | r | a_prev | a]
  float* layers_out;
  float* dm_out;
  const float* rs;     // FP64 residual: slopes of the right-hand side W^{-T} A^T C_hat^{-1} s (or NULL)
  const float* rg;     // FP64 residual: layer-domain term of the right-hand side W^{-T} g (or NULL)
};

// Coarse-level correction of the converged solves (fewha_solve and its
// kin; never the frame path, which is Algorithm 1's Jacobi PCG).  Z selects
// the top-left s x s block of every layer's Mallat layout (the coarsest
// levels, s = 16 by default, smaller when the problem would exceed
// kCoarseMax unknowns), E = Z^T M Z, and the preconditioner is
//   z = J^{-1} r + Z E^{-1} Z^T r,
// Jacobi plus an exact solve on the coarse block (additive two-level form).
// The weakly observed low-order modes of the layers, which keep Jacobi PCG
// slow, are resolved by the coarse solve.
constexpr int kCoarseSide = 16;   // default coarse block side per layer
constexpr int kCoarseMax = 1024;  // most coarse unknowns of one problem
constexpr int kCoarseRows = 64;   // rows of E^{-1} per workgroup of k_coarse
struct CoarseDev {
  const float* einv;  // E^{-1}, m x m row-major (one copy per distinct system)
  const int* idx;     // the m coarse coefficients: index in the problem's vector
  float* zc;          // N_c floats: E^{-1} Z^T r at the coarse indices, 0 elsewhere
  double* slots;      // kDotRing x n_slots: partials of (Z^T r)^T E^{-1} Z^T r
  int m, n_slots;     // n_slots = workgroups of k_coarse of the problem
  int pad_[2];
};
// Set-up of E: round t probes column t count + rank of the system's E with
// a unit vector in `in` (every instance of one system in a batch probes its
// own columns); M e_j comes back in `out`.
struct CoarseProbe {
  float* in;
  const float* out;
  const int* idx;
  float* E;  // m x m, column j = Z^T M e_j (owned by the system's first instance)
  int m, rank, count, pad_;
};

// Work item of a tiled launch: problem, item (layer or sensor), tile
// row/column, and the slot of the partial it produces.  Some kinds carry
// more, so that their descriptor loads need not wait for the problem's:
// propagation-adjoint tiles use slot / level for their sensor list (offset,
// count) and mask / pad1 for the layer's side and offset; the sensor-stage
// tiles carry the sensor's descriptor index in slot and the problem's first
// layer descriptor in mask; the transform tiles carry their layer's
// descriptor index in mask (and the global levels their level in level).
struct Tile {
  int prob, item, ty, tx;
  int slot, level, mask, pad1;
};

// ---- host-side description of one configured problem ----

struct WfsHost {
  fewha_wfs_desc d;
  std::vector<uint8_t> mask;   // N*N
  std::vector<int> cmap;       // N*N compact index or -1
  int n_active = 0;
  std::vector<double> cinv;    // 3 per subaperture (a, b, c), row-major N*N
  double sum_cinv[4] = {0, 0, 0, 0};
};

struct LayerHost {
  fewha_layer_desc d;
  double delta = 0;
  std::vector<double> dtab;  // D_j, j = 0..kMaxLevelsJ-1 (0 where unused)
};

struct GLTables {  // one (sensor, layer) pair
  std::vector<int> q0y, q0x;   // nc
  std::vector<double> wy, wx;  // nc
};

struct GradTables {  // one (sensor, layer) pair, derivative with respect to the layer height
  std::vector<int> qy, qx, tiey, tiex;        // nc
  std::vector<double> wy, wx, dty, dtx;       // nc
};

// DM fitting (Sec. 4.1, layers not at the DM altitudes): directions, DMs,
// the fitting pupil (corners of the active subapertures of an N x N grid).
struct FitHost {
  bool on = false;
  std::vector<fewha_dm_desc> dms;
  std::vector<double> dirs;   // x, y pairs (rad)
  int N = 0, iters = 10;
  double eps_rel = 1e-6;
  // derived
  std::vector<int> cmap;                    // (N+1)^2: >= 0 inside the fitting pupil
  std::vector<std::vector<GLTables>> tabL;  // [dir][layer] layers -> pupil corners
  std::vector<std::vector<GLTables>> tabD;  // [dir][dm]    DMs -> pupil corners
  std::vector<int> dm_off;                  // offsets of the DM grids in the command vector
  long n_act = 0;
  double eps = 0;                           // eps_rel * mean(diag(sum_k B_k^T M B_k))
};

// Fitting work of one fitted problem (one workgroup runs its CG vector work).
struct FitDev {
  int main, n_act, pad0, pad1;
  float eps, gain;
  float* x;        // fitted commands
  float* r;
  float* p;        // search direction (the source of the DM propagation)
  const float* adj;  // sum_k B_k^T M (B_k p or P_k phi)
  double* scal;    // rho
  int* numflag;    // the plan's breakdown flag (see ProbDev)
};

struct HostModel {
  double D = 0, obs = 0;
  std::vector<WfsHost> wfs;
  std::vector<LayerHost> layers;
  double L = 0;
  double alpha = 1, r0 = 0.15, L0 = 25, tau = 0;
  double alpha_eta = 0, na_fwhm = 11400, spot_fwhm = 4.85e-6;
  double gain = 1;
  bool closed = false;  // closed-loop control (Algorithm 1), F = I only
  int aug_keep = 0;     // augmented PCG: previous search directions kept (0 = plain PCG)
  bool have_pupil = false, have_wfs = false, have_layers = false;
  // derived
  double h[6] = {0}, g[6] = {0};
  std::vector<std::vector<GLTables>> tab;  // [g][l]
  std::vector<std::vector<GradTables>> gtab;  // [g][l]
  bool grad_ok = true;                     // every derivative stencil stays inside its layer
  std::string grad_msg;
  std::vector<double> Dprior;              // N_c
  std::vector<double> J;                   // N_c
  std::vector<int> layer_off;
  std::vector<int> slope_off;
  long n_c = 0, n_slopes = 0;
  FitHost fit;
  int tune_res = 0;  // resident transform side of the context's own plan (0 = default)
  int tune_pt_rows = 0;  // node rows per thread of the propagation adjoint (0 = default)
  int tune_split = 0;    // resident inverse levels: 0 or 1 = one workgroup per layer, 4 = quarters
  int tune_pt_split = 0; // 1: propagation-adjoint tiles of one band record, sensors split over the waves
  int tune_glob_fuse = 0; // 1: a layer's last two global inverse levels in one tile
  long n_act() const { return fit.on ? fit.n_act : n_c; }
  // [c | b | r | a_prev | a], then with augmentation the previous directions,
  // their images and a count (4 floats, keeping 16-byte alignment)
  long n_state() const { return 3L * n_c + 2L * n_act() + (aug_keep > 0 ? 2L * aug_keep * n_c + 4 : 0); }
};

// host set-up (setup.cpp); each returns FEWHA_OK or an error with a message
fewha_status build_model(HostModel& m, std::string& err);
void db3_filter(double h[6]);

}  // namespace fewha
