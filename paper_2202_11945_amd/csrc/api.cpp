// C ABI of libfewha: contexts (one configured problem), plans (device
// tables, work buffers and tile work lists of one or many problems), the
// launch sequences of every entry point, and HIP graph capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "fewha_internal.h"
#include "kernels.h"

using namespace fewha;

namespace {

constexpr int kRing = 8;          // pinned staging slots for per-call I/O tables
constexpr int kMaxIters = 256;    // PCG iterations per reconstruct call (graph-captured frames)
constexpr int kMaxSolveIters = 1 << 24;  // PCG iterations of one solve
constexpr int kSolveCheck = 16;   // iterations between two convergence checks of a solve
constexpr int kMaxSweeps = 32;    // refinement sweeps of one solve
static_assert(sizeof(GradIo) <= sizeof(IoDev), "per-call tables share the staging ring");

int ilog2i(int n) {
  int k = 0;
  while ((1 << k) < n) ++k;
  return k;
}
int cdiv(int a, int b) { return (a + b - 1) / b; }

struct Range {
  int off = 0, n = 0;
};

// Device plan of one or more finalized problems.
struct Plan {
  int device = -1;
  int nprob = 0;
  int res_max = kResMax;  // resident transform side (tuning)
  int pt_rows = 4;        // node rows per thread of the propagation adjoint (tuning)
  bool pt_wide = false;   // some (sensor, layer) pair has K > 3 corners per node (wide band records)
  bool pt_split = false;  // propagation-adjoint tiles of one band record, sensors split over the waves
  bool glob_fuse = false; // some inverse global tiles run a layer's last two levels (k_idwt_glob2)
  std::vector<const HostModel*> models;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  ProbDev* dP = nullptr;
  LayerDev* dL = nullptr;
  WfsDev* dW = nullptr;
  IoDev* dIO = nullptr;
  IoDev* dIOprof = nullptr;
  IoDev* dIO2 = nullptr;   // per-call table of a frame's true-residual restart (M c into q)
  Tile* dT = nullptr;
  std::vector<ProbDev> hP;
  std::vector<LayerDev> hL;
  std::vector<WfsDev> hW;
  std::vector<Tile> hT;
  Range idwt_res, fdwt_res, pg, gt, pt, upd;
  Range idwt_res4;          // the resident inverse levels in quarters (four tiles per layer)
  bool idwt_split = false;  // launch them instead of one workgroup per layer
  Range sin;  // slopes input: 2 x 2 groups of the propagation stage's subaperture tiles
  Range sin_frame, pg_pol;  // a frame's slope input: open-loop problems / closed-loop problems
  Range aug;                // augmented PCG: vector-update chunks of the problems with augmentation
  std::vector<Range> idwt_glob, fdwt_glob;
  Range fit_fwdL, fit_fwdD, fit_pt, fit_cg;  // DM fitting (empty when no problem fits)
  Range sinit, gprior, ghgt;                 // solve start, parameter-gradient reductions
  Range r64wfs;                              // FP64 residual: one tile per (problem, sensor)
  Range r64pt;                               // FP64 residual: 32x32 node tiles of the adjoint
  Range r64gt;                               // FP64 residual: 16x16 corner tiles of the sensor adjoint
  std::vector<Range> r64inv, r64fwd;         // FP64 residual: transform steps
  Resid64Tiles r64;
  Filter64 F64{};
  std::vector<float*> rbuf;                  // per problem: residual of a refined solve
  GradIo* dGIO = nullptr;
  const HatEnt* dHat = nullptr;              // hat tables of the propagation adjoint
  int nHat = 0;                              // entries of dHat
  const BandRec* dBand = nullptr;            // band records of the propagation adjoint
  const PtEnt* dPtE = nullptr;               // sensor lists of the propagation-adjoint tiles
  const int2* dGtr = nullptr;                // window rows of the Shack-Hartmann adjoint tiles
  const int2* dPgr = nullptr;                // tables of the propagation-stage tiles
  std::vector<float*> sstate;                // per problem: [x | unused | r] of a solve
  double* rho_host = nullptr;                // pinned readback: 2 n_dots doubles per problem
  std::vector<long> rho_off;
  int nprob_all = 0;                         // problems plus two fitting views per fitted problem
  FitDev* dF = nullptr;
  int max_fit_iters = 0;
  Filter F{};
  IoDev* pinned[kRing] = {nullptr};
  hipEvent_t ev[kRing] = {nullptr};
  bool ev_used[kRing] = {false};
  int ring = 0;
  std::map<int, hipGraphExec_t> graphs;
  std::map<int, hipGraph_t> graph_defs;
  hipStream_t cap_stream = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  std::vector<float*> prof_state;
  std::vector<long> n_state;
  std::vector<IoDev> last_io;
  bool ran = false;
  int* numflag = nullptr;                    // breakdown flag (host-mapped pinned memory)
  int* numflag_dev = nullptr;                // its device address
  // allocation-free frame: problem records whose work buffers live in the
  // library's static device scratch (see fewha_reconstruct_noalloc)
  // streamed frames (context plans): the host slopes arrive by sensor groups
  std::vector<int> sin_g;                    // problem 0: start of sensor g's tiles in the sin list (G + 1)
  float* dslopes = nullptr;                  // device copy of the streamed slopes
  hipStream_t copy_stream = nullptr;
  hipEvent_t copy_start = nullptr;
  std::vector<hipEvent_t> chunk_ev;
  ProbDev* dPna = nullptr;                   // in the arena, nprob_all records
  IoDev* na_io = nullptr;                    // per-call table at the start of the scratch
  size_t na_bytes = 0;                       // scratch the plan's frame needs
  // coarse-level correction of the converged solves, set up by the first
  // solve after a change of its side (0: Jacobi only)
  int coarse_side = kCoarseSide;
  bool coarse_ready = false;
  void* coarse_mem = nullptr;                // E^{-1}, indices, zc, slots, descriptors, tiles
  const CoarseDev* dC = nullptr;
  const Tile* dCT = nullptr;
  int n_coarse_tiles = 0;
  std::vector<int> coarse_m;                 // per problem: coarse unknowns (0: not corrected)
};

#define HIP_TRY(expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
      return FEWHA_EDEVICE;                                                    \
    }                                                                          \
  } while (0)

void destroy_plan(Plan* p) {
  if (!p) return;
  if (p->device >= 0) (void)hipSetDevice(p->device);
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& kv : p->graph_defs) (void)hipGraphDestroy(kv.second);
  for (int i = 0; i < kRing; ++i) {
    if (p->ev[i]) (void)hipEventDestroy(p->ev[i]);
    if (p->pinned[i]) (void)hipHostFree(p->pinned[i]);
  }
  for (float* s : p->prof_state)
    if (s) (void)hipFree(s);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->copy_stream) (void)hipStreamDestroy(p->copy_stream);
  if (p->copy_start) (void)hipEventDestroy(p->copy_start);
  for (hipEvent_t e : p->chunk_ev)
    if (e) (void)hipEventDestroy(e);
  if (p->dslopes) (void)hipFree(p->dslopes);
  if (p->t0) (void)hipEventDestroy(p->t0);
  if (p->t1) (void)hipEventDestroy(p->t1);
  if (p->rho_host) (void)hipHostFree(p->rho_host);
  if (p->numflag) (void)hipHostFree(p->numflag);
  if (p->coarse_mem) (void)hipFree(p->coarse_mem);
  if (p->arena) (void)hipFree(p->arena);
  delete p;
}

// Hat tables of one (sensor, layer) pair of the propagation adjoint: for every
// node row, then every node column, the corners whose bilinear cell touches
// the node (t = t0 + k rho within one node spacing, found in FP64) and their
// weights 1 - rho |k - c| with c = (p - t0) / rho, the transpose of the
// forward interpolation weights.
struct NodeHat {
  int lo;
  float w[kWideMaxK];
};
std::vector<NodeHat> node_hats(const GLPar& gp, int n, int axis) {
  const int K = gp.kmax;
  const double t0 = axis == 0 ? gp.t0y : gp.t0x;
  std::vector<NodeHat> out;
  for (int p = 0; p < n; ++p) {
    const double c = ((double)p - t0) * gp.inv_rho;
    const int lo = std::max((int)std::floor(c - gp.inv_rho) + 1, 0);
    const int hi = std::min((int)std::ceil(c + gp.inv_rho) - 1, gp.nc - 1);
    // no corner (outside the footprint, or between corners when rho > 2):
    // weights 0 on the valid corners at floor(c), so that lo never
    // decreases along the axis
    NodeHat e{std::max(0, std::min((int)std::floor(c), gp.nc - K)), {}};
    if (hi >= lo) {
      const int base = std::max(0, std::min(lo, gp.nc - K));
      e.lo = base;
      for (int k = 0; k < K; ++k) {
        const int corner = base + k;
        if (corner >= lo && corner <= hi)
          e.w[k] = (float)std::max(0.0, 1.0 - gp.rho * std::fabs((double)corner - c));
      }
    }
    out.push_back(e);
  }
  return out;
}

// Hat entries per node: one, two for a wide pair (K > 3).
int hat_per_node(int K) { return K > 3 ? 2 : 1; }

void append_hats(GLPar& gp, int n, std::vector<HatEnt>& out) {
  gp.hat_off = (int)out.size();
  const int per = hat_per_node(gp.kmax);
  for (int axis = 0; axis < 2; ++axis)
    for (const NodeHat& e : node_hats(gp, n, axis))
      for (int h = 0; h < per; ++h) out.push_back(HatEnt{e.lo, {e.w[3 * h], e.w[3 * h + 1], e.w[3 * h + 2]}});
}

// Propagation-adjoint tables of one (sensor, layer) pair: hat tables with K =
// 2 .. 6 corners per node and axis when the corner spacing is at least 1/3 of
// the node spacing, and one band record per kBandRows node rows, whose corner
// rows must fit pt_band(K, kBandRows) (K <= 3) or pt_band_wide(K); otherwise
// kmax = 0, the general gather.  Pairs of the same geometry (every problem of
// a batch of one system) share one copy of the tables.
struct HatTables {
  std::vector<HatEnt> hats;
  std::vector<BandRec> bands;
  std::map<std::tuple<double, double, double, int, int>, std::array<int, 3>> seen;  // -> kmax, hat_off, band_off
};

int kmax_of(double rho) {
  if (rho >= 1.0) return 2;
  if (rho >= 2.0 / 3.0) return 3;
  if (rho >= 0.5) return 4;
  if (rho >= 0.4) return 5;
  if (rho >= 1.0 / 3.0) return 6;
  return 0;
}

void set_hats(GLPar& gp, int n, HatTables& T) {
  gp.kmax = kmax_of(gp.rho);
  gp.hat_off = gp.band_off = -1;
  if (gp.kmax > 0 && gp.nc < gp.kmax) gp.kmax = 0;  // tiny sensor
  if (gp.kmax == 0) return;
  const auto key = std::make_tuple(gp.t0y, gp.t0x, gp.rho, gp.nc, n);
  const auto hit = T.seen.find(key);
  if (hit != T.seen.end()) {
    gp.kmax = hit->second[0];
    gp.hat_off = hit->second[1];
    gp.band_off = hit->second[2];
    return;
  }
  const int K = gp.kmax;
  const bool wide = K > 3;
  const int SB = wide ? pt_band_wide(K) : pt_band(K, kBandRows);
  const std::vector<NodeHat> rows = node_hats(gp, n, 0);
  std::vector<BandRec> recs;
  bool fits = true;
  for (int p = 0; p < n && fits; p += kBandRows) {
    const int last = std::min(p + kBandRows - 1, n - 1);
    const int ilo = rows[p].lo;
    if (rows[last].lo + K - ilo > SB) {
      fits = false;
      break;
    }
    const int cnt = std::min(kBandRows, n - p);  // node rows of the group inside the layer
    bool zero = true;
    for (int u = 0; u < cnt; ++u)
      for (int k = 0; k < K; ++k) zero = zero && rows[p + u].w[k] == 0.f;
    // step pattern (narrow pairs): every node row inside the layer, steps of
    // K - 2 or K - 1
    int pat = (cnt == kBandRows && !wide) ? 0 : -1;
    for (int u = 1; u < kBandRows && pat >= 0; ++u) {
      const int step = rows[p + u].lo - rows[p + u - 1].lo - (K - 2);
      if (step == 1)
        pat |= 1 << (u - 1);
      else if (step != 0)
        pat = -1;
    }
    // first band row: the group's first corner, or (dense records) moved up
    // so that the band stays inside the grid where it can
    const int base = pat >= 0 ? ilo : std::max(0, std::min(ilo, gp.nc - SB));
    BandRec r{};
    BandRecW rw{};
    r.so0 = rw.so0 = base * gp.nc * (int)sizeof(float);
    r.pat = rw.pat = zero ? kPatZero : (pat >= 0 ? pat : kPatDense);
    r.nrows = rw.nrows = std::min(SB, gp.nc - base);
    for (int u = 0; u < cnt && fits; ++u)
      for (int k = 0; k < K; ++k) {
        const int s = rows[p + u].lo + k - base;
        if (s < 0 || s >= r.nrows) {
          fits = false;
          break;
        }
        if (wide) {
          rw.w[u][s] = rows[p + u].w[k];
        } else {
          r.wk[u][k] = rows[p + u].w[k];
          r.w[u][s] = rows[p + u].w[k];
        }
      }
    if (wide) std::memcpy(&r, &rw, sizeof(r));
    recs.push_back(r);
  }
  if (!fits) {
    gp.kmax = 0;
  } else {
    append_hats(gp, n, T.hats);
    gp.band_off = (int)T.bands.size();
    T.bands.insert(T.bands.end(), recs.begin(), recs.end());
  }
  T.seen[key] = {gp.kmax, gp.hat_off, gp.band_off};
}

// Does (sensor, layer) pair gp add anything to the node tile of rows p0 ..
// p0 + ph - 1 and columns q0 .. q0 + qw - 1 of an n x n layer?  With hat
// tables: some row and some column of the tile have a nonzero hat (the
// gather is separable, so the tile's sum is zero otherwise; a sparse sensor,
// whose corners lie more than two node spacings apart, touches few node rows
// and columns inside its footprint).  Without (general gather): the tile
// meets the footprint, the corners t0 + k rho widened by two nodes.
bool pair_meets_tile(const GLPar& gp, const HatTables& T, int n, int p0, int ph, int q0, int qw) {
  if (gp.kmax == 0) {
    const double span = (gp.nc - 1) * gp.rho;
    auto meets = [&](double t0, int a, int ext) { return a + ext - 1 >= t0 - 2.0 && a <= t0 + span + 2.0; };
    return meets(gp.t0y, p0, ph) && meets(gp.t0x, q0, qw);
  }
  const int per = hat_per_node(gp.kmax);
  auto any = [&](int first, int a, int ext) {
    for (int p = a; p < std::min(a + ext, n); ++p)
      for (int h = 0; h < per; ++h) {
        const HatEnt& e = T.hats[(size_t)first + per * p + h];
        if (e.w[0] != 0.f || e.w[1] != 0.f || e.w[2] != 0.f) return true;
      }
    return false;
  };
  return any(gp.hat_off, p0, ph) && any(gp.hat_off + per * n, q0, qw);
}

// Longest first within each XCD's run of a launch's tiles: workgroup b runs
// on XCD b mod 8 and each XCD takes a contiguous run of the list in order
// (the device-side mapping), so sorting every run by descending sensor count
// (Tile::level of a propagation-adjoint tile) starts the longest workgroups
// first and shortens the tail.  The runs keep their tiles, so what an XCD's
// L2 holds does not change.
void sort_xcd_runs_by_count(std::vector<Tile>& v) {
  const int W = (int)v.size(), q = W / 8, r = W % 8;
  for (int x = 0; x < 8; ++x) {
    const int start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    const int len = q + (x < r ? 1 : 0);
    std::stable_sort(v.begin() + start, v.begin() + start + len,
                     [](const Tile& a, const Tile& b) { return a.level > b.level; });
  }
}

// Sensor lists of propagation-adjoint tiles, one copy per distinct list.
struct PtLists {
  std::vector<PtEnt> ents;
  std::map<std::vector<int>, int> seen;
  // tile (ty, tx) of a layer with n node rows and columns, pair parameters
  // gl[g * L + item] for the sensors g in `use`: returns {offset, count}
  std::pair<int, int> add(const std::vector<GLPar>& gl, int L, int item, const std::vector<int>& use, int n,
                          int ty, int tx, int recs_per_tile) {
    std::vector<int> key;
    if (use.size() > 63) return {-1, 0};  // a wave reads its tile's list (and the pad) from 64 lanes
    for (int g : use) {
      const GLPar& gp = gl[(size_t)g * L + item];
      PtEnt e{gp.v_off, gp.nc << 3 | gp.kmax, 0, 0};
      if (gp.kmax > 0) {
        const int per = hat_per_node(gp.kmax);
        e.hx = gp.hat_off + per * (n + tx * kPtW);
        e.band = gp.band_off + ty * recs_per_tile;  // kBandRows rows per record
      } else {
        e.nck = (g * L + item) << 3;
      }
      key.insert(key.end(), {e.v_off, e.nck, e.hx, e.band});
    }
    key.insert(key.end(), {0, 2, 0, 0});  // the pad entry
    auto it = seen.find(key);
    if (it != seen.end()) return {it->second, (int)use.size()};
    const int off = (int)ents.size();
    for (size_t i = 0; i < key.size(); i += 4) ents.push_back(PtEnt{key[i], key[i + 1], key[i + 2], key[i + 3]});
    seen[key] = off;
    return {off, (int)use.size()};
  }
};

// Byte-offset carving of the arena (256-byte aligned pieces).
struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    off = (off + 255) & ~size_t(255);
    size_t o = off;
    off += bytes;
    return o;
  }
};

fewha_status build_plan(Plan*& out, const std::vector<const HostModel*>& models, int device, int res,
                        int pt_rows, int split, int pt_split, int glob_fuse, std::string& err) {
  if (res != 32 && res != 64 && res != 128) {
    err = "tuning: the resident transform side must be 32, 64 or 128";
    return FEWHA_EINVAL;
  }
  if (pt_rows != 4 && pt_rows != 8) {
    err = "tuning: the propagation adjoint takes 4 or 8 node rows per thread";
    return FEWHA_EINVAL;
  }
  if (pt_split != 0 && pt_split != 1) {
    err = "tuning: pt_split must be 0 or 1";
    return FEWHA_EINVAL;
  }
  if (pt_split && pt_rows != 4) {
    err = "tuning: split propagation-adjoint tiles take 4 node rows per thread";
    return FEWHA_EINVAL;
  }
  if (glob_fuse != 0 && glob_fuse != 1) {
    err = "tuning: glob_fuse must be 0 or 1";
    return FEWHA_EINVAL;
  }
  // quarters need at least one resident level of output side >= 16 on every layer
  bool split_ok = true;
  for (const HostModel* m : models)
    for (const LayerHost& lh : m->layers) {
      const int R = std::min(lh.d.n, res);
      if (R < 16 || R < 2 * (lh.d.n >> lh.d.levels)) split_ok = false;
    }
  if (split == 4 && !split_ok) {
    err = "tuning: four workgroups per layer need every layer's resident side >= 16 and >= 2 (n >> levels)";
    return FEWHA_EINVAL;
  }
  // node rows of a propagation-adjoint tile, and its band records per wave
  const int kPtH = pt_split ? kBandRows : 4 * pt_rows;
  const int pt_recs = pt_split ? 1 : pt_rows;
  for (const HostModel* m : models)
    for (const LayerHost& lh : m->layers)
      if ((lh.d.n >> lh.d.levels) > res) {
        err = "tuning: a layer's coarsest block (n >> levels) exceeds the resident side " + std::to_string(res);
        return FEWHA_EINVAL;
      }
  std::unique_ptr<Plan> pl(new (std::nothrow) Plan());
  if (!pl) {
    err = "out of host memory";
    return FEWHA_ENOMEM;
  }
  Plan& P = *pl;
  P.device = device;
  P.res_max = res;
  P.pt_rows = pt_rows;
  P.pt_split = pt_split != 0;
  P.idwt_split = split == 4;
  P.nprob = (int)models.size();
  P.models = models;
  HIP_TRY(hipSetDevice(device));
  {
    const HostModel& m0 = *models[0];
    for (int i = 0; i < 6; ++i) {
      P.F.h[i] = (float)m0.h[i];
      P.F.g[i] = (float)m0.g[i];
      P.F64.h[i] = m0.h[i];
      P.F64.g[i] = m0.g[i];
    }
  }
  // ---- descriptors and tile lists ----
  struct ProbLayout {
    size_t phi, phiadj, tmpa, tmpb, sd, vadj, part, p0, p1, q, dots, jinv, itab, ftab, cmap, cinv, gl;
    size_t sstate, gphi, glam, gslots, gitab, gftab, amap, srow;
    size_t a64, b64, sd64, u64, rslots, cinv64, ftab64, rbuf, x64;
    size_t apdir, aqdir, aslots, afac;
  };
  std::vector<ProbLayout> lay(P.nprob);
  Carver cv;
  std::vector<Tile> t_sin, t_sinf, t_pgpol, t_aug, t_r64gt;
  std::vector<Tile> t_idwt_res, t_idwt_res4, t_fdwt_res, t_pg, t_gt, t_pt, t_upd, t_sinit, t_gprior, t_ghgt, t_r64wfs,
      t_r64pt;
  HatTables hats;  // hat tables and band records of every problem and fitting view, one set per plan
  PtLists ptl;     // sensor lists of the propagation-adjoint tiles
  std::vector<std::vector<Tile>> t_r64inv(kMaxLevelsJ), t_r64fwd(kMaxLevelsJ);
  std::vector<std::vector<double>> cinv64(P.nprob), ftab64(P.nprob);
  std::vector<std::vector<Tile>> t_idwt_glob, t_fdwt_glob;
  // host table images per problem (copied after allocation)
  std::vector<std::vector<int>> itab(P.nprob), cmap(P.nprob), gitab(P.nprob);
  std::vector<std::vector<int>> srow(P.nprob);  // row bases of the row-span slope layout
  std::vector<int2> gtrows;                     // Shack-Hartmann adjoint tiles' window rows (plan-wide)
  std::vector<int2> pgrows;                     // propagation-stage tiles' tables (plan-wide)
  static_assert(kGtS == 32, "a window row's 33 active flags: 32 bits and the base's low bit");
  std::vector<std::vector<float>> ftab(P.nprob), cinv(P.nprob), jinv(P.nprob), gftab(P.nprob);
  std::vector<std::vector<GLPar>> glp(P.nprob);
  for (int k = 0; k < P.nprob; ++k) {
    const HostModel& m = *models[k];
    ProbDev pd{};
    const int L = (int)m.layers.size(), G = (int)m.wfs.size();
    pd.L = L;
    pd.G = G;
    pd.layer0 = (int)P.hL.size();
    pd.wfs0 = (int)P.hW.size();
    pd.n_c = (int)m.n_c;
    pd.n_slopes = (int)m.n_slopes;
    pd.n_act = (int)m.n_act();
    pd.fitted = m.fit.on ? 1 : 0;
    pd.closed = m.closed ? 1 : 0;
    pd.aug_keep = m.aug_keep;
    pd.gain = (float)m.gain;
    int tmp_total = 0;
    for (int l = 0; l < L; ++l) {
      const LayerHost& lh = m.layers[l];
      LayerDev ld{};
      ld.n = lh.d.n;
      ld.log2n = ilog2i(ld.n);
      ld.levels = lh.d.levels;
      ld.res = std::min(ld.n, res);
      ld.off = m.layer_off[l];
      ld.n_glob_levels = ilog2i(ld.n / ld.res);
      ld.tmp_off = tmp_total;
      if (ld.n > ld.res) tmp_total += ld.n * ld.n / 4;
      ld.inv_delta = (float)(1.0 / lh.delta);
      for (int j = 0; j < kMaxLevelsJ; ++j) {
        ld.alpha_d[j] = (float)(m.alpha * lh.dtab[j]);
        ld.d64[j] = lh.dtab[j];
      }
      ld.cn2 = lh.d.cn2;
      ld.inv_delta64 = 1.0 / lh.delta;
      P.hL.push_back(ld);
    }
    int s_tot = 0, v_tot = 0, m_tot = 0, part_tot = 0, tab_tot = 0, gtab_tot = 0, sp_tot = 0;
    srow[k].clear();
    for (int g = 0; g < G; ++g) {
      const WfsHost& wh = m.wfs[g];
      WfsDev wd{};
      wd.N = wh.d.n_subap;
      wd.nc = wd.N + 1;
      // row-span slope layout: row i keeps its columns lo_i .. hi_i (first
      // and last active subaperture), rows packed in order; inactive
      // subapertures inside a span (a central obstruction) keep a slot
      wd.rb_off = (int)srow[k].size();
      int len = 0;
      for (int i = 0; i < wd.N; ++i) {
        int lo = wd.N, hi = -1;
        for (int j = 0; j < wd.N; ++j)
          if (wh.cmap[(size_t)i * wd.N + j] >= 0) {
            lo = std::min(lo, j);
            hi = j;
          }
        srow[k].push_back(hi >= lo ? len - lo : 0);
        if (hi >= lo) len += hi - lo + 1;
      }
      wd.sp_off = sp_tot;
      wd.sp_len = len;
      sp_tot += 2 * len;
      wd.lgs = wh.d.kind == FEWHA_LGS;
      wd.tt = wd.lgs && wh.d.tt_removal;
      wd.blocks = wd.lgs && m.alpha_eta > 0.0;
      wd.n_active = wh.n_active;
      wd.s_off = s_tot;
      s_tot += 2 * wd.N * wd.N;
      wd.v_off = v_tot;
      v_tot += wd.nc * wd.nc;
      wd.cs_off = m.slope_off[g];
      wd.m_off = m_tot;
      wd.cinv_off = 3 * m_tot;
      m_tot += wd.N * wd.N;
      wd.tiles_side = cdiv(wd.N, kTileS);
      wd.n_tiles_s = wd.tiles_side * wd.tiles_side;
      wd.part_off = part_tot;
      part_tot += 4 * wd.n_tiles_s;
      wd.tab_stride = 4 * wd.nc;
      wd.tab_off = tab_tot;
      tab_tot += L * wd.tab_stride;
      wd.gtab_off = gtab_tot;
      gtab_tot += L * 4 * wd.nc;
      wd.inv_sigma2 = (float)(1.0 / (wh.d.sigma * wh.d.sigma));
      wd.inv_nM = (float)(1.0 / wh.n_active);
      wd.inv_sigma2_d = 1.0 / (wh.d.sigma * wh.d.sigma);
      wd.inv_nM_d = 1.0 / wh.n_active;
      for (int v = 0; v < 4; ++v) wd.sum_cinv[v] = (float)wh.sum_cinv[v];
      P.hW.push_back(wd);
    }
    // table images
    itab[k].assign(tab_tot, 0);
    ftab[k].assign(tab_tot, 0.f);
    cmap[k].assign(m_tot, -1);
    cinv[k].assign(3 * (size_t)m_tot, 0.f);
    cinv64[k].assign(3 * (size_t)m_tot, 0.0);
    ftab64[k].assign(std::max(tab_tot, 1), 0.0);
    for (int g = 0; g < G; ++g) {
      const WfsDev& wd = P.hW[pd.wfs0 + g];
      const WfsHost& wh = m.wfs[g];
      for (int e = 0; e < wd.N * wd.N; ++e) cmap[k][wd.m_off + e] = wh.cmap[e];
      for (int e = 0; e < 3 * wd.N * wd.N; ++e) {
        cinv[k][wd.cinv_off + e] = (float)wh.cinv[e];
        cinv64[k][wd.cinv_off + e] = wh.cinv[e];
      }
      for (int l = 0; l < L; ++l) {
        const GLTables& t = m.tab[g][l];
        const int base = wd.tab_off + l * wd.tab_stride, nc = wd.nc;
        for (int j = 0; j < nc; ++j) {
          itab[k][base + j] = t.q0y[j];
          itab[k][base + nc + j] = t.q0x[j];
          ftab[k][base + 2 * nc + j] = (float)t.wy[j];
          ftab[k][base + 3 * nc + j] = (float)t.wx[j];
          ftab64[k][base + 2 * nc + j] = t.wy[j];
          ftab64[k][base + 3 * nc + j] = t.wx[j];
        }
      }
    }
    gitab[k].assign(std::max(gtab_tot, 1), 0);
    gftab[k].assign(std::max(gtab_tot, 1), 0.f);
    for (int g = 0; g < G; ++g) {
      const WfsDev& wd = P.hW[pd.wfs0 + g];
      for (int l = 0; l < L; ++l) {
        const GradTables& t = m.gtab[g][l];
        const int base = wd.gtab_off + l * 4 * wd.nc, nc = wd.nc;
        for (int j = 0; j < nc; ++j) {
          gitab[k][base + j] = t.qy[j];
          gitab[k][base + nc + j] = t.qx[j];
          gitab[k][base + 2 * nc + j] = t.tiey[j];
          gitab[k][base + 3 * nc + j] = t.tiex[j];
          gftab[k][base + j] = (float)t.wy[j];
          gftab[k][base + nc + j] = (float)t.wx[j];
          gftab[k][base + 2 * nc + j] = (float)t.dty[j];
          gftab[k][base + 3 * nc + j] = (float)t.dtx[j];
        }
      }
    }
    jinv[k].resize(m.n_c);
    for (long e = 0; e < m.n_c; ++e) jinv[k][e] = (float)(1.0 / m.J[e]);
    // propagation-adjoint parameters per (sensor, layer)
    glp[k].resize((size_t)G * L);
    for (int g = 0; g < G; ++g)
      for (int l = 0; l < L; ++l) {
        const WfsHost& wh = m.wfs[g];
        const LayerHost& lh = m.layers[l];
        const double scale = (wh.d.kind == FEWHA_LGS) ? 1.0 - lh.d.h / wh.d.H : 1.0;
        GLPar gp{};
        gp.t0y = (scale * (-0.5 * m.D) + lh.d.h * wh.d.theta_y + 0.5 * m.L) / lh.delta;
        gp.t0x = (scale * (-0.5 * m.D) + lh.d.h * wh.d.theta_x + 0.5 * m.L) / lh.delta;
        gp.rho = scale * (m.D / wh.d.n_subap) / lh.delta;
        gp.inv_rho = 1.0 / gp.rho;
        gp.nc = wh.d.n_subap + 1;
        gp.v_off = P.hW[pd.wfs0 + g].v_off;
        set_hats(gp, lh.d.n, hats);
        glp[k][(size_t)g * L + l] = gp;
      }
    // tiles
    int slot = 0;
    int maxng = 0;
    for (int l = 0; l < L; ++l) maxng = std::max(maxng, P.hL[pd.layer0 + l].n_glob_levels);
    if ((int)t_fdwt_glob.size() < maxng) {
      t_fdwt_glob.resize(maxng);
      t_idwt_glob.resize(maxng);
    }
    for (int s = 0; s < maxng; ++s)
      for (int l = 0; l < L; ++l) {
        const LayerDev& ld = P.hL[pd.layer0 + l];
        if (ld.n_glob_levels <= s) continue;
        const int mf = ld.n >> s;  // forward: input side
        const int tq = (mf / 2) / 16;
        // with glob_fuse a layer's first two global levels are one tile at
        // step 0 (its inner coarse block goes where step 1 would put it)
        const bool ffuse = glob_fuse && ld.n_glob_levels >= 2;
        if (!(ffuse && s == 1))
          for (int ty = 0; ty < tq; ++ty)
            for (int tx = 0; tx < tq; ++tx)
              t_fdwt_glob[s].push_back({k, l, ty, tx, slot++, ilog2i(mf), pd.layer0 + l, (ffuse && s == 0) ? 1 : 0});
        // inverse: output side; with glob_fuse a layer's last two global
        // levels are one tile of its full side at the inner level's step
        // (reading that step's scratch), and its last step has no tiles
        const int ng = ld.n_glob_levels;
        if (glob_fuse && ng >= 2 && s >= ng - 2) {
          if (s == ng - 1) continue;
          for (int ty = 0; ty < ld.n / 32; ++ty)
            for (int tx = 0; tx < ld.n / 32; ++tx)
              t_idwt_glob[s].push_back({k, l, ty, tx, 0, ilog2i(ld.n), pd.layer0 + l, 1});
          P.glob_fuse = true;
          continue;
        }
        const int mi = ld.res << (s + 1);
        const int ti = mi / 32;
        for (int ty = 0; ty < ti; ++ty)
          for (int tx = 0; tx < ti; ++tx) t_idwt_glob[s].push_back({k, l, ty, tx, 0, ilog2i(mi), pd.layer0 + l, 0});
      }
    for (int l = 0; l < L; ++l) {
      // transform tiles carry the global layer index (mask), so that the
      // layer and problem records load in parallel
      t_idwt_res.push_back({k, l, 0, 0, 0, 0, pd.layer0 + l, 0});
      for (int q = 0; q < 4; ++q) t_idwt_res4.push_back({k, l, 0, q, 0, 0, pd.layer0 + l, 0});
      t_fdwt_res.push_back({k, l, 0, 0, slot++, 0, pd.layer0 + l, 0});
    }
    pd.n_slots_fdwt = slot;
    const int nupd = cdiv(pd.n_c, kUpdChunk);
    for (int c = 0; c < nupd; ++c) {
      t_upd.push_back({k, 0, c, 0, c, 0, 0, 0});
      if (m.aug_keep > 0) t_aug.push_back({k, 0, c, 0, c, 0, 0, 0});
    }
    pd.n_slots_upd = nupd;
    pd.n_dots = std::max(pd.n_slots_fdwt, pd.n_slots_upd);
    for (int sl = 0; sl < pd.n_slots_fdwt; ++sl) t_sinit.push_back({k, 0, 0, 0, sl, 0, 0, 0});
    // parameter gradients: prior-term chunks per layer, height-term tiles per (layer, sensor)
    int gp = 0, gh = 0;
    for (int l = 0; l < L; ++l) {
      LayerDev& ld = P.hL[pd.layer0 + l];
      const int nch = cdiv(ld.n * ld.n, kGradChunk);
      ld.gp_off = gp;
      ld.gp_n = nch;
      for (int c2 = 0; c2 < nch; ++c2) t_gprior.push_back({k, l, c2, 0, gp + c2, 0, 0, 0});
      gp += nch;
      ld.gh_off = gh;
      for (int g = 0; g < G; ++g) {
        const int tc = cdiv(P.hW[pd.wfs0 + g].nc, kTileS);
        for (int ty = 0; ty < tc; ++ty)
          for (int tx = 0; tx < tc; ++tx) t_ghgt.push_back({k, g, ty, tx, gh++, l, 0, 0});
      }
      ld.gh_n = gh - ld.gh_off;
    }
    pd.n_gp = gp;
    pd.n_gh = gh;
    pd.alpha = m.alpha;
    // FP64 residual: transform steps per layer, one noise tile per sensor
    for (int l = 0; l < L; ++l) {
      const LayerDev& ld = P.hL[pd.layer0 + l];
      const int m0 = ld.n >> ld.levels;
      for (int st = 0; st < ld.levels; ++st) {
        const int mi = m0 << (st + 1), mf = ld.n >> st;
        for (int c2 = 0; c2 < cdiv(mi * mi, 1024); ++c2) t_r64inv[st].push_back({k, l, c2, 0, 0, ilog2i(mi), 0, 0});
        for (int c2 = 0; c2 < cdiv(mf * mf / 2, 1024); ++c2)
          t_r64fwd[st].push_back({k, l, c2, 0, 0, ilog2i(mf), 0, 0});
      }
    }
    for (int g = 0; g < G; ++g) t_r64wfs.push_back({k, g, 0, 0, 0, 0, 0, 0});
    for (int g = 0; g < G; ++g) {
      const WfsDev& wd = P.hW[pd.wfs0 + g];
      // propagation-stage tiles with their own tables (per layer the window's
      // 17 corner rows, then its 17 columns: cell index and fraction)
      for (int ty = 0; ty < wd.tiles_side; ++ty)
        for (int tx = 0; tx < wd.tiles_side; ++tx) {
          const int off = (int)pgrows.size();
          t_pg.push_back({k, g, ty, tx, pd.wfs0 + g, off, pd.layer0, 0});
          if (m.closed) t_pgpol.push_back({k, g, ty, tx, pd.wfs0 + g, off, pd.layer0, 0});
          for (int l = 0; l < L; ++l) {
            const GLTables& tb = m.tab[g][l];
            auto entry = [](int cell, double f) {
              const float ff = (float)f;
              int bits;
              std::memcpy(&bits, &ff, sizeof bits);
              return make_int2(cell, bits);
            };
            for (int c = 0; c <= kTileS; ++c) {
              const int ic = ty * kTileS + c;
              pgrows.push_back(ic < wd.nc ? entry(tb.q0y[ic], tb.wy[ic]) : make_int2(0, 0));
            }
            for (int c = 0; c <= kTileS; ++c) {
              const int jc = tx * kTileS + c;
              pgrows.push_back(jc < wd.nc ? entry(tb.q0x[jc], tb.wx[jc]) : make_int2(0, 0));
            }
          }
        }
      const int sg = cdiv(wd.tiles_side, 2);
      if (k == 0) P.sin_g.push_back((int)t_sin.size());
      for (int ty = 0; ty < sg; ++ty)
        for (int tx = 0; tx < sg; ++tx) {
          t_sin.push_back({k, g, ty, tx, pd.wfs0 + g, 0, pd.layer0, 0});
          if (!m.closed) t_sinf.push_back({k, g, ty, tx, pd.wfs0 + g, 0, pd.layer0, 0});
        }
      // Shack-Hartmann adjoint tiles: kGtS x kGtS corners over a window of
      // kGtS + 1 subaperture rows and columns; per window row the span base
      // and the active flags of the window's columns (tile.level: the first
      // row's entry)
      const int tc = cdiv(wd.nc, kGtS);
      const WfsHost& wh = m.wfs[g];
      for (int ty = 0; ty < tc; ++ty)
        for (int tx = 0; tx < tc; ++tx) {
          t_gt.push_back({k, g, ty, tx, pd.wfs0 + g, (int)gtrows.size(), pd.layer0, 0});
          for (int li = 0; li <= kGtS; ++li) {
            const int i = ty * kGtS - 1 + li;
            int base = 0, top = 0;
            unsigned bits = 0;
            if (i >= 0 && i < wd.N) {
              base = srow[k][wd.rb_off + i];
              for (int lj = 0; lj <= kGtS; ++lj) {
                const int j = tx * kGtS - 1 + lj;
                if (j < 0 || j >= wd.N || wh.cmap[(size_t)i * wd.N + j] < 0) continue;
                if (lj < 32)
                  bits |= 1u << lj;
                else
                  top = 1;
              }
            }
            gtrows.push_back(make_int2(base * 2 + top, (int)bits));
          }
        }
      const int tc16 = cdiv(wd.nc, kTileS);
      for (int ty = 0; ty < tc16; ++ty)
        for (int tx = 0; tx < tc16; ++tx) t_r64gt.push_back({k, g, ty, tx, pd.wfs0 + g, 0, pd.layer0, 0});
    }
    if (k == 0) P.sin_g.push_back((int)t_sin.size());
    // node tiles of the propagation adjoint (kPtH rows x kPtW columns) with the
    // sensors that add to them; 32x32 tiles for the FP64 residual's adjoint
    for (int l = 0; l < L; ++l) {
      const int n = P.hL[pd.layer0 + l].n;
      for (int ty = 0; ty < cdiv(n, kPtH); ++ty)
        for (int tx = 0; tx < cdiv(n, kPtW); ++tx) {
          std::vector<int> use;
          for (int g = 0; g < G; ++g)
            if (pair_meets_tile(glp[k][(size_t)g * L + l], hats, n, ty * kPtH, kPtH, tx * kPtW, kPtW))
              use.push_back(g);
          const auto li = ptl.add(glp[k], L, l, use, n, ty, tx, pt_recs);
          if (li.first < 0) {
            err = "more than 63 sensors meet one propagation-adjoint tile";
            return FEWHA_EINVAL;
          }
          t_pt.push_back({k, l, ty, tx, li.first, li.second, n, P.hL[pd.layer0 + l].off});
        }
      const int nt = cdiv(n, kTileN);
      for (int ty = 0; ty < nt; ++ty)
        for (int tx = 0; tx < nt; ++tx) t_r64pt.push_back({k, l, ty, tx, 0, 0, -1, 0});
    }
    // buffer layout
    ProbLayout& pl_ = lay[k];
    const size_t nc4 = sizeof(float) * (size_t)pd.n_c;
    pl_.phi = cv.take(nc4);
    pl_.phiadj = cv.take(nc4);
    pl_.tmpa = cv.take(sizeof(float) * std::max(tmp_total, 1));
    pl_.tmpb = cv.take(sizeof(float) * std::max(tmp_total, 1));
    pl_.sd = cv.take(sizeof(float) * std::max(sp_tot, 1));
    pl_.srow = cv.take(sizeof(int) * std::max<size_t>(srow[k].size(), 1));
    pl_.vadj = cv.take(sizeof(float) * v_tot);
    pl_.part = cv.take(sizeof(float) * part_tot);
    pl_.p0 = cv.take(nc4);
    pl_.p1 = cv.take(nc4);
    pl_.q = cv.take(nc4);
    pl_.dots = cv.take(sizeof(double) * (size_t)(2 * kDotRing) * pd.n_dots);
    pl_.jinv = cv.take(nc4);
    pl_.itab = cv.take(sizeof(int) * tab_tot);
    pl_.ftab = cv.take(sizeof(float) * tab_tot);
    pl_.cmap = cv.take(sizeof(int) * m_tot);
    pl_.amap = cv.take(std::max(m_tot, 1));
    pl_.cinv = cv.take(sizeof(float) * 3 * (size_t)m_tot);
    pl_.gl = cv.take(sizeof(GLPar) * (size_t)G * L);
    pl_.sstate = cv.take(sizeof(float) * 3 * (size_t)pd.n_c);
    pl_.gphi = cv.take(nc4);
    pl_.glam = cv.take(nc4);
    pl_.gslots = cv.take(sizeof(double) * (size_t)(pd.n_gp + 2 * pd.n_gh));
    pl_.gitab = cv.take(sizeof(int) * gitab[k].size());
    pl_.gftab = cv.take(sizeof(float) * gftab[k].size());
    pl_.a64 = cv.take(sizeof(double) * (size_t)pd.n_c);
    pl_.b64 = cv.take(sizeof(double) * (size_t)pd.n_c);
    pl_.sd64 = cv.take(sizeof(double) * s_tot);
    pl_.u64 = cv.take(sizeof(double) * v_tot);
    pl_.rslots = cv.take(sizeof(double) * 2 * (size_t)pd.n_slots_upd);
    pl_.cinv64 = cv.take(sizeof(double) * cinv64[k].size());
    pl_.ftab64 = cv.take(sizeof(double) * ftab64[k].size());
    pl_.rbuf = cv.take(nc4);
    pl_.x64 = cv.take(sizeof(double) * (size_t)pd.n_c);
    pl_.apdir = cv.take(nc4 * std::max(pd.aug_keep, 1));
    pl_.aqdir = cv.take(nc4 * std::max(pd.aug_keep, 1));
    pl_.aslots = cv.take(sizeof(double) * (size_t)kAugGroups * pd.n_slots_upd);
    pl_.afac = cv.take(sizeof(double) * kAugFac);
    P.hP.push_back(pd);
  }
  // ---- DM fitting views: (directions x layers) and (directions x DMs) ----
  struct FitLayout {
    int k, pL, pD;
    size_t u, x, r, p, adj, scal, itab, ftab, cmap, gl;
    std::vector<int> it;
    std::vector<float> ft;
    std::vector<GLPar> glp;
  };
  std::vector<FitLayout> fits;
  std::vector<Tile> t_ffL, t_ffD, t_fpt, t_fcg;
  std::vector<FitDev> hF;
  for (int k = 0; k < P.nprob; ++k) {
    const HostModel& m = *models[k];
    if (!m.fit.on) continue;
    const FitHost& f = m.fit;
    FitLayout fl;
    fl.k = k;
    const int K = (int)f.dirs.size() / 2, nc = f.N + 1, nd = (int)f.dms.size(), L = (int)m.layers.size();
    P.max_fit_iters = std::max(P.max_fit_iters, f.iters);
    // DM grids as layers of the second view
    const int dm_layer0 = (int)P.hL.size();
    for (int q = 0; q < nd; ++q) {
      LayerDev ld{};
      ld.n = f.dms[q].n_act;
      ld.res = ld.n;
      ld.off = f.dm_off[q];
      P.hL.push_back(ld);
    }
    // direction "sensors" of the two views; tables [view][dir][grid] with stride 4 nc
    int tab = 0;
    auto add_dirs = [&](int ngrid, const std::vector<std::vector<GLTables>>& tb) {
      const int w0 = (int)P.hW.size();
      for (int d = 0; d < K; ++d) {
        WfsDev wd{};
        wd.N = f.N;
        wd.nc = nc;
        wd.v_off = d * nc * nc;
        wd.m_off = 0;
        wd.tab_stride = 4 * nc;
        wd.tab_off = tab;
        for (int g2 = 0; g2 < ngrid; ++g2) {
          const GLTables& t = tb[d][g2];
          const int base = tab + g2 * 4 * nc;
          fl.it.resize(base + 4 * nc, 0);
          fl.ft.resize(base + 4 * nc, 0.f);
          for (int j = 0; j < nc; ++j) {
            fl.it[base + j] = t.q0y[j];
            fl.it[base + nc + j] = t.q0x[j];
            fl.ft[base + 2 * nc + j] = (float)t.wy[j];
            fl.ft[base + 3 * nc + j] = (float)t.wx[j];
          }
        }
        tab += ngrid * 4 * nc;
        P.hW.push_back(wd);
      }
      return w0;
    };
    const int wL = add_dirs(L, f.tabL);
    const int wD = add_dirs(nd, f.tabD);
    // adjoint-gather parameters of (direction, DM)
    for (int d = 0; d < K; ++d)
      for (int q = 0; q < nd; ++q) {
        const fewha_dm_desc& dm = f.dms[q];
        GLPar gp{};
        gp.t0x = (-0.5 * m.D + dm.h * f.dirs[2 * d]) / dm.pitch + 0.5 * (dm.n_act - 1);
        gp.t0y = (-0.5 * m.D + dm.h * f.dirs[2 * d + 1]) / dm.pitch + 0.5 * (dm.n_act - 1);
        gp.rho = (m.D / f.N) / dm.pitch;
        gp.inv_rho = 1.0 / gp.rho;
        gp.nc = nc;
        gp.v_off = d * nc * nc;
        set_hats(gp, dm.n_act, hats);
        fl.glp.push_back(gp);
      }
    ProbDev vL{}, vD{};
    vL.L = L;
    vL.G = K;
    vL.layer0 = P.hP[k].layer0;
    vL.wfs0 = wL;
    vD.L = nd;
    vD.G = K;
    vD.layer0 = dm_layer0;
    vD.wfs0 = wD;
    fl.pL = (int)P.hP.size();
    P.hP.push_back(vL);
    fl.pD = (int)P.hP.size();
    P.hP.push_back(vD);
    fl.u = cv.take(sizeof(float) * (size_t)K * nc * nc);
    fl.x = cv.take(sizeof(float) * f.n_act);
    fl.r = cv.take(sizeof(float) * f.n_act);
    fl.p = cv.take(sizeof(float) * f.n_act);
    fl.adj = cv.take(sizeof(float) * f.n_act);
    fl.scal = cv.take(sizeof(double) * 4);
    fl.itab = cv.take(sizeof(int) * fl.it.size());
    fl.ftab = cv.take(sizeof(float) * fl.ft.size());
    fl.cmap = cv.take(sizeof(int) * f.cmap.size());
    fl.gl = cv.take(sizeof(GLPar) * fl.glp.size());
    const int tc = cdiv(nc, kTileS);
    for (int d = 0; d < K; ++d)
      for (int ty = 0; ty < tc; ++ty)
        for (int tx = 0; tx < tc; ++tx) {
          t_ffL.push_back({fl.pL, d, ty, tx, 0, 0, 0, 0});
          t_ffD.push_back({fl.pD, d, ty, tx, 0, 0, 0, 0});
        }
    for (int q = 0; q < nd; ++q) {
      const int na = f.dms[q].n_act;
      for (int ty = 0; ty < cdiv(na, kPtH); ++ty)
        for (int tx = 0; tx < cdiv(na, kPtW); ++tx) {  // the directions that add to the tile
          std::vector<int> use;
          for (int d = 0; d < K; ++d)
            if (pair_meets_tile(fl.glp[(size_t)d * nd + q], hats, na, ty * kPtH, kPtH, tx * kPtW, kPtW))
              use.push_back(d);
          const auto li = ptl.add(fl.glp, nd, q, use, na, ty, tx, pt_recs);
          if (li.first < 0) {
            err = "more than 63 fitting directions";
            return FEWHA_EINVAL;
          }
          t_fpt.push_back({fl.pD, q, ty, tx, li.first, li.second, na, P.hL[dm_layer0 + q].off});
        }
    }
    t_fcg.push_back({(int)hF.size(), 0, 0, 0, 0, 0, 0, 0});
    FitDev fd{};
    fd.main = k;
    fd.n_act = (int)f.n_act;
    fd.eps = (float)f.eps;
    fd.gain = (float)m.gain;
    hF.push_back(fd);
    fits.push_back(std::move(fl));
  }
  P.nprob_all = (int)P.hP.size();

  // concatenated tile list
  auto add = [&](std::vector<Tile>& v) {
    Range r;
    r.off = (int)P.hT.size();
    r.n = (int)v.size();
    P.hT.insert(P.hT.end(), v.begin(), v.end());
    return r;
  };
  P.idwt_res = add(t_idwt_res);
  P.idwt_res4 = add(t_idwt_res4);
  P.fdwt_res = add(t_fdwt_res);
  P.pg = add(t_pg);
  P.sin = add(t_sin);
  P.sin_frame = add(t_sinf);
  P.pg_pol = add(t_pgpol);
  P.aug = add(t_aug);
  P.gt = add(t_gt);
  sort_xcd_runs_by_count(t_pt);
  P.pt = add(t_pt);
  P.upd = add(t_upd);
  for (auto& v : t_idwt_glob) P.idwt_glob.push_back(add(v));
  for (auto& v : t_fdwt_glob) P.fdwt_glob.push_back(add(v));
  P.fit_fwdL = add(t_ffL);
  P.fit_fwdD = add(t_ffD);
  sort_xcd_runs_by_count(t_fpt);
  P.fit_pt = add(t_fpt);
  P.fit_cg = add(t_fcg);
  P.sinit = add(t_sinit);
  P.gprior = add(t_gprior);
  P.ghgt = add(t_ghgt);
  P.r64wfs = add(t_r64wfs);
  P.r64pt = add(t_r64pt);
  P.r64gt = add(t_r64gt);
  for (int st = 0; st < kMaxLevelsJ; ++st) {
    P.r64inv.push_back(add(t_r64inv[st]));
    P.r64fwd.push_back(add(t_r64fwd[st]));
  }
  const size_t oP = cv.take(sizeof(ProbDev) * P.nprob_all);
  const size_t oL = cv.take(sizeof(LayerDev) * P.hL.size());
  const size_t oW = cv.take(sizeof(WfsDev) * P.hW.size());
  const size_t oIO = cv.take(sizeof(IoDev) * P.nprob_all);
  const size_t oIOp = cv.take(sizeof(IoDev) * P.nprob_all);
  const size_t oIO2 = cv.take(sizeof(IoDev) * P.nprob_all);
  const size_t oGIO = cv.take(sizeof(GradIo) * P.nprob_all);
  for (const auto& kv : hats.seen) P.pt_wide = P.pt_wide || kv.second[0] > 3;
  // at least 64 hat entries and 8 band records: the padded prefetch addresses
  hats.hats.resize(std::max<size_t>(hats.hats.size(), 64), HatEnt{0, {0.f, 0.f, 0.f}});
  hats.bands.resize(std::max<size_t>(hats.bands.size(), 8), BandRec{});
  const size_t oHat = cv.take(sizeof(HatEnt) * hats.hats.size());
  const size_t oBand = cv.take(sizeof(BandRec) * hats.bands.size());
  const size_t oPtE = cv.take(sizeof(PtEnt) * std::max<size_t>(ptl.ents.size(), 1));
  const size_t oGtr = cv.take(sizeof(int2) * std::max<size_t>(gtrows.size(), 1));
  const size_t oPgr = cv.take(sizeof(int2) * std::max<size_t>(pgrows.size(), 1));
  const size_t oF = cv.take(sizeof(FitDev) * std::max<size_t>(hF.size(), 1));
  const size_t oPna = cv.take(sizeof(ProbDev) * P.nprob_all);
  const size_t oT = cv.take(sizeof(Tile) * std::max<size_t>(P.hT.size(), 1));
  P.arena_bytes = cv.off;
  {
    hipError_t e = hipMalloc(&P.arena, P.arena_bytes);
    if (e != hipSuccess) {
      err = std::string("device allocation of ") + std::to_string(P.arena_bytes) + " bytes failed";
      return FEWHA_ENOMEM;
    }
  }
  HIP_TRY(hipMemset(P.arena, 0, P.arena_bytes));
  HIP_TRY(hipHostMalloc((void**)&P.numflag, sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
  *(volatile int*)P.numflag = 0;
  HIP_TRY(hipHostGetDevicePointer((void**)&P.numflag_dev, P.numflag, 0));
  for (ProbDev& pd : P.hP) pd.numflag = P.numflag_dev;
  for (FitDev& fd : hF) fd.numflag = P.numflag_dev;
  char* base = (char*)P.arena;
  for (int k = 0; k < P.nprob; ++k) {
    ProbDev& pd = P.hP[k];
    const ProbLayout& l = lay[k];
    pd.phi = (float*)(base + l.phi);
    pd.phiadj = (float*)(base + l.phiadj);
    pd.tmpa = (float*)(base + l.tmpa);
    pd.tmpb = (float*)(base + l.tmpb);
    pd.sd = (float*)(base + l.sd);
    pd.vadj = (float*)(base + l.vadj);
    pd.part = (float*)(base + l.part);
    pd.pbuf0 = (float*)(base + l.p0);
    pd.pbuf1 = (float*)(base + l.p1);
    pd.q = (float*)(base + l.q);
    pd.dots = (double*)(base + l.dots);
    pd.jinv = (const float*)(base + l.jinv);
    pd.itab = (const int*)(base + l.itab);
    pd.ftab = (const float*)(base + l.ftab);
    pd.cmap = (const int*)(base + l.cmap);
    pd.amap = (const unsigned char*)(base + l.amap);
    pd.srow = (const int*)(base + l.srow);
    pd.cinv = (const float*)(base + l.cinv);
    pd.gl = (const GLPar*)(base + l.gl);
    pd.gphi = (float*)(base + l.gphi);
    pd.glam = (float*)(base + l.glam);
    pd.gslots = (double*)(base + l.gslots);
    pd.gitab = (const int*)(base + l.gitab);
    pd.gftab = (const float*)(base + l.gftab);

    P.sstate.push_back((float*)(base + l.sstate));
    pd.a64 = (double*)(base + l.a64);
    pd.b64 = (double*)(base + l.b64);
    pd.sd64 = (double*)(base + l.sd64);
    pd.u64 = (double*)(base + l.u64);
    pd.rslots = (double*)(base + l.rslots);
    pd.cinv64 = (const double*)(base + l.cinv64);
    pd.ftab64 = (const double*)(base + l.ftab64);
    pd.rbuf = (float*)(base + l.rbuf);
    pd.x64 = (double*)(base + l.x64);
    pd.aug_pdir = (float*)(base + l.apdir);
    pd.aug_qdir = (float*)(base + l.aqdir);
    pd.aug_slots = (double*)(base + l.aslots);
    pd.aug_fac = (double*)(base + l.afac);
    P.rbuf.push_back(pd.rbuf);
    HIP_TRY(hipMemcpy(base + l.cinv64, cinv64[k].data(), sizeof(double) * cinv64[k].size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + l.ftab64, ftab64[k].data(), sizeof(double) * ftab64[k].size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + l.gitab, gitab[k].data(), sizeof(int) * gitab[k].size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + l.gftab, gftab[k].data(), sizeof(float) * gftab[k].size(), hipMemcpyHostToDevice));

    HIP_TRY(hipMemcpy(base + l.gl, glp[k].data(), sizeof(GLPar) * glp[k].size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + l.jinv, jinv[k].data(), sizeof(float) * jinv[k].size(), hipMemcpyHostToDevice));
    if (!itab[k].empty()) {
      HIP_TRY(hipMemcpy(base + l.itab, itab[k].data(), sizeof(int) * itab[k].size(), hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(base + l.ftab, ftab[k].data(), sizeof(float) * ftab[k].size(), hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(base + l.cmap, cmap[k].data(), sizeof(int) * cmap[k].size(), hipMemcpyHostToDevice));
    {
      std::vector<unsigned char> act(cmap[k].size());
      for (size_t e = 0; e < act.size(); ++e) act[e] = cmap[k][e] >= 0 ? 1 : 0;
      if (!act.empty()) HIP_TRY(hipMemcpy(base + l.amap, act.data(), act.size(), hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(base + l.cinv, cinv[k].data(), sizeof(float) * cinv[k].size(), hipMemcpyHostToDevice));
    if (!srow[k].empty())
      HIP_TRY(hipMemcpy(base + l.srow, srow[k].data(), sizeof(int) * srow[k].size(), hipMemcpyHostToDevice));
  }
  for (size_t i = 0; i < fits.size(); ++i) {
    const FitLayout& fl = fits[i];
    const ProbDev& main = P.hP[fl.k];
    ProbDev& vL = P.hP[fl.pL];
    ProbDev& vD = P.hP[fl.pD];
    float* u = (float*)(base + fl.u);
    vL.phi = main.phi;  // layers of the reconstruction
    vL.vadj = u;
    vL.itab = vD.itab = (const int*)(base + fl.itab);
    vL.ftab = vD.ftab = (const float*)(base + fl.ftab);
    vL.cmap = vD.cmap = (const int*)(base + fl.cmap);
    vD.phi = (float*)(base + fl.p);
    vD.phiadj = (float*)(base + fl.adj);
    vD.vadj = u;
    vD.gl = (const GLPar*)(base + fl.gl);

    FitDev& fd = hF[i];
    fd.x = (float*)(base + fl.x);
    fd.r = (float*)(base + fl.r);
    fd.p = vD.phi;
    fd.adj = vD.phiadj;
    fd.scal = (double*)(base + fl.scal);
    const FitHost& f = models[fl.k]->fit;
    HIP_TRY(hipMemcpy(base + fl.itab, fl.it.data(), sizeof(int) * fl.it.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + fl.ftab, fl.ft.data(), sizeof(float) * fl.ft.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + fl.cmap, f.cmap.data(), sizeof(int) * f.cmap.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + fl.gl, fl.glp.data(), sizeof(GLPar) * fl.glp.size(), hipMemcpyHostToDevice));
  }
  P.dF = (FitDev*)(base + oF);
  P.dPna = (ProbDev*)(base + oPna);
  if (!hF.empty()) HIP_TRY(hipMemcpy(P.dF, hF.data(), sizeof(FitDev) * hF.size(), hipMemcpyHostToDevice));
  P.dP = (ProbDev*)(base + oP);
  P.dL = (LayerDev*)(base + oL);
  P.dW = (WfsDev*)(base + oW);
  P.dIO = (IoDev*)(base + oIO);
  P.dIOprof = (IoDev*)(base + oIOp);
  P.dIO2 = (IoDev*)(base + oIO2);
  P.dGIO = (GradIo*)(base + oGIO);
  P.dHat = (const HatEnt*)(base + oHat);
  P.nHat = (int)hats.hats.size();
  P.dBand = (const BandRec*)(base + oBand);
  if (!hats.hats.empty())
    HIP_TRY(hipMemcpy(base + oHat, hats.hats.data(), sizeof(HatEnt) * hats.hats.size(), hipMemcpyHostToDevice));
  if (!hats.bands.empty())
    HIP_TRY(hipMemcpy(base + oBand, hats.bands.data(), sizeof(BandRec) * hats.bands.size(), hipMemcpyHostToDevice));
  P.dPgr = (const int2*)(base + oPgr);
  if (!pgrows.empty())
    HIP_TRY(hipMemcpy(base + oPgr, pgrows.data(), sizeof(int2) * pgrows.size(), hipMemcpyHostToDevice));
  P.dGtr = (const int2*)(base + oGtr);
  if (!gtrows.empty())
    HIP_TRY(hipMemcpy(base + oGtr, gtrows.data(), sizeof(int2) * gtrows.size(), hipMemcpyHostToDevice));
  P.dPtE = (const PtEnt*)(base + oPtE);
  if (!ptl.ents.empty())
    HIP_TRY(hipMemcpy(base + oPtE, ptl.ents.data(), sizeof(PtEnt) * ptl.ents.size(), hipMemcpyHostToDevice));
  P.dT = (Tile*)(base + oT);
  // work lists of the FP64 residual chain (device addresses: after P.dT is set)
  {
    Resid64Tiles& rt = P.r64;
    rt.upd = P.dT + P.upd.off;
    rt.upd_n = P.upd.n;
    for (int st = 0; st < kMaxLevelsJ; ++st) {
      rt.inv[st] = P.dT + P.r64inv[st].off;
      rt.inv_n[st] = P.r64inv[st].n;
      rt.fwd[st] = P.dT + P.r64fwd[st].off;
      rt.fwd_n[st] = P.r64fwd[st].n;
      if (rt.inv_n[st] > 0) rt.n_steps = st + 1;
    }
    rt.pg = P.dT + P.pg.off;
    rt.pg_n = P.pg.n;
    rt.wfs = P.dT + P.r64wfs.off;
    rt.wfs_n = P.r64wfs.n;
    rt.gt = P.dT + P.r64gt.off;  // the FP64 sensor adjoint's own 16 x 16 corner tiles
    rt.gt_n = P.r64gt.n;
    rt.pt = P.dT + P.r64pt.off;
    rt.pt_n = P.r64pt.n;
  }
  HIP_TRY(hipMemcpy(P.dP, P.hP.data(), sizeof(ProbDev) * P.nprob_all, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(P.dL, P.hL.data(), sizeof(LayerDev) * P.hL.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(P.dW, P.hW.data(), sizeof(WfsDev) * P.hW.size(), hipMemcpyHostToDevice));
  if (!P.hT.empty()) HIP_TRY(hipMemcpy(P.dT, P.hT.data(), sizeof(Tile) * P.hT.size(), hipMemcpyHostToDevice));
  for (int i = 0; i < kRing; ++i) {
    HIP_TRY(hipHostMalloc((void**)&P.pinned[i], sizeof(IoDev) * P.nprob_all, hipHostMallocDefault));
    HIP_TRY(hipEventCreateWithFlags(&P.ev[i], hipEventDisableTiming));
  }
  {
    long tot = 0;
    for (int k = 0; k < P.nprob; ++k) {
      P.rho_off.push_back(tot);
      tot += 2 * P.hP[k].n_dots;  // a dot group, or the residual pairs (2 per update slot)
    }
    HIP_TRY(hipHostMalloc((void**)&P.rho_host, sizeof(double) * std::max(tot, 1L), hipHostMallocDefault));
  }
  HIP_TRY(hipStreamCreateWithFlags(&P.cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipEventCreate(&P.t0));
  HIP_TRY(hipEventCreate(&P.t1));
  P.n_state.resize(P.nprob);
  for (int k = 0; k < P.nprob; ++k) P.n_state[k] = models[k]->n_state();
  out = pl.release();
  return FEWHA_OK;
}

// ---- the allocation-free frame ----
// The work buffers of fewha_reconstruct_noalloc live in this array, one copy
// per device, for the life of the process.  Host code never uses its name
// as an address: each device's copy is looked up once (noalloc_scratch) and
// that address is what kernels and copies receive.
constexpr size_t kNoAllocBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of `scratch` on `device` (current), looked up once per device.
fewha_status noalloc_scratch(int device, unsigned char** out, std::string& err) {
  static std::mutex mu;
  static std::map<int, unsigned char*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it == addr.end()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return FEWHA_EDEVICE;
    }
    it = addr.emplace(device, (unsigned char*)ptr).first;
  }
  *out = it->second;
  return FEWHA_OK;
}

// Problem records of plan P whose frame work buffers (layers, adjoint,
// coarse-block scratch, slope buffer, corner grids, tip/tilt partials,
// search directions, M p, inner-product slots) are carved from the static
// scratch after a 256-byte per-call table; the tables stay in the arena.
// Every buffer is written before it is read within a frame, so the scratch
// needs no clearing.  Called at set-up with the plan's device current.
fewha_status setup_noalloc(Plan& P, std::string& err) {
  unsigned char* base = nullptr;
  fewha_status s = noalloc_scratch(P.device, &base, err);
  if (s != FEWHA_OK) return s;
  std::vector<ProbDev> v(P.hP);
  size_t off = 256;  // the per-call IoDev table
  static_assert(sizeof(IoDev) <= 256, "one per-call table in the scratch head");
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return base + o;
  };
  for (int k = 0; k < P.nprob; ++k) {
    ProbDev& pd = v[k];
    const size_t nc4 = sizeof(float) * (size_t)pd.n_c;
    size_t tmp = 4, sd = 4, vadj = 4, part = 4;
    for (int l = 0; l < pd.L; ++l) {
      const LayerDev& ld = P.hL[pd.layer0 + l];
      if (ld.n > ld.res) tmp = std::max(tmp, sizeof(float) * (size_t)(ld.tmp_off + ld.n * ld.n / 4));
    }
    for (int g = 0; g < pd.G; ++g) {
      const WfsDev& wd = P.hW[pd.wfs0 + g];
      sd = std::max(sd, sizeof(float) * (size_t)(wd.sp_off + 2 * wd.sp_len));
      vadj = std::max(vadj, sizeof(float) * (size_t)(wd.v_off + wd.nc * wd.nc));
      part = std::max(part, sizeof(float) * (size_t)(wd.part_off + 4 * wd.n_tiles_s));
    }
    pd.phi = (float*)take(nc4);
    pd.phiadj = (float*)take(nc4);
    pd.tmpa = (float*)take(tmp);
    pd.tmpb = (float*)take(tmp);
    pd.sd = (float*)take(sd);
    pd.vadj = (float*)take(vadj);
    pd.part = (float*)take(part);
    pd.pbuf0 = (float*)take(nc4);
    pd.pbuf1 = (float*)take(nc4);
    pd.q = (float*)take(nc4);
    pd.dots = (double*)take(sizeof(double) * (size_t)(2 * kDotRing) * pd.n_dots);
  }
  if (sizeof(IoDev) * (size_t)P.nprob_all > 256) {
    err = "allocation-free frame: per-call table larger than the scratch head";
    return FEWHA_EINVAL;
  }
  P.na_bytes = off;
  P.na_io = (IoDev*)base;
  HIP_TRY(hipMemcpy(P.dPna, v.data(), sizeof(ProbDev) * v.size(), hipMemcpyHostToDevice));
  return FEWHA_OK;
}

// Streamed frames of a context plan: the device slope buffer, a copy stream
// and one event per sensor group (at most kMaxChunks groups).
constexpr int kMaxChunks = 64;
fewha_status setup_streamed(Plan& P, long n_slopes, int G, std::string& err) {
  HIP_TRY(hipMalloc(&P.dslopes, sizeof(float) * std::max(n_slopes, 1L)));
  HIP_TRY(hipStreamCreateWithFlags(&P.copy_stream, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&P.copy_start, hipEventDisableTiming));
  P.chunk_ev.assign(std::min(G, kMaxChunks), nullptr);
  for (hipEvent_t& e : P.chunk_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return FEWHA_OK;
}

// Stage a per-call table (nprob entries, zero-padded to nprob_all) and copy
// it to the device, stream ordered.  The pinned slot is reused only after the
// copy that read it has completed.
template <typename T>
fewha_status upload_table(Plan& P, const std::vector<T>& v, hipStream_t s, T* dst, std::string& err) {
  const int slot = P.ring;
  P.ring = (P.ring + 1) % kRing;
  if (P.ev_used[slot]) HIP_TRY(hipEventSynchronize(P.ev[slot]));
  std::memset(P.pinned[slot], 0, sizeof(T) * P.nprob_all);
  std::memcpy(P.pinned[slot], v.data(), sizeof(T) * P.nprob);
  HIP_TRY(hipMemcpyAsync(dst, P.pinned[slot], sizeof(T) * P.nprob_all, hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(P.ev[slot], s));
  P.ev_used[slot] = true;
  return FEWHA_OK;
}
fewha_status upload_io(Plan& P, const std::vector<IoDev>& io, hipStream_t s, IoDev* dst, std::string& err) {
  return upload_table(P, io, s, dst, err);
}

// The breakdown flag of plan P, read and cleared: FEWHA_ENUMERIC when a PCG
// step of earlier work on the plan (finished by now) found p^T M p <= 0 with
// a nonzero residual or a non-finite inner product.  Work still running is
// seen by a later call.
fewha_status take_numeric(Plan& P, std::string& err) {
  volatile int* f = P.numflag;
  const int v = f ? *f : 0;
  if (v == 0) return FEWHA_OK;
  *f = 0;
  err = "numerical breakdown in earlier work: PCG met p^T M p <= 0 with a nonzero residual, or a non-finite "
        "inner product, in problem " + std::to_string(v - 1) + " (its results are not valid)";
  return FEWHA_ENUMERIC;
}

// The true-residual restart's table: in = each problem's state (c first), out = its q.
fewha_status upload_refresh_io(Plan& P, const std::vector<IoDev>& io, hipStream_t s, std::string& err) {
  std::vector<IoDev> t(P.nprob);
  for (int k = 0; k < P.nprob; ++k) {
    t[k].in = io[k].state;
    t[k].out = P.hP[k].q;
  }
  return upload_io(P, t, s, P.dIO2, err);
}

LaunchArgs args(const Plan& P, hipStream_t s, const IoDev* io) {
  LaunchArgs a;
  a.P = P.dP;
  a.L = P.dL;
  a.W = P.dW;
  a.IO = io;
  a.F = P.F;
  a.stream = s;
  a.res_max = P.res_max;
  a.pt_rows = P.pt_rows;
  a.pt_wide = P.pt_wide ? 1 : 0;
  a.pt_split = P.pt_split ? 1 : 0;
  a.glob_fuse = P.glob_fuse ? 1 : 0;
  a.hats = P.dHat;
  a.n_hats = P.nHat;
  a.bands = P.dBand;
  a.pents = P.dPtE;
  a.gtrows = P.dGtr;
  a.pgrows = P.dPgr;
  return a;
}

const Tile* T(const Plan& P, const Range& r) { return P.dT + r.off; }

void enq_idwt(const Plan& P, const LaunchArgs& a, int src, int out, int iter) {
  if (P.idwt_split)
    launch_idwt_res4(a, T(P, P.idwt_res4), P.idwt_res4.n, src, out, iter);
  else
    launch_idwt_res(a, T(P, P.idwt_res), P.idwt_res.n, src, out, iter);
  for (size_t s = 0; s < P.idwt_glob.size(); ++s)
    launch_idwt_glob(a, T(P, P.idwt_glob[s]), P.idwt_glob[s].n, src, out, iter, (int)s);
}
void enq_fdwt(const Plan& P, const LaunchArgs& a, int epi, int iter) {
  for (size_t s = 0; s < P.fdwt_glob.size(); ++s)
    launch_fdwt_glob(a, T(P, P.fdwt_glob[s]), P.fdwt_glob[s].n, epi, iter, (int)s);
  launch_fdwt_res(a, T(P, P.fdwt_res), P.fdwt_res.n, epi, iter);
}
// A^T C_hat^{-1} (slopes in the work buffer) -> phiadj
void enq_adjoint(const Plan& P, const LaunchArgs& a, int gt_mode, int pt_mode) {
  launch_gammaT(a, T(P, P.gt), P.gt.n, gt_mode);
  launch_pT(a, T(P, P.pt), P.pt.n, pt_mode);
}
void enq_apply_M_core(const Plan& P, const LaunchArgs& a) {
  launch_pgamma(a, T(P, P.pg), P.pg.n, PG_DENSE);
  enq_adjoint(P, a, GT_WEIGHTED, PT_PHIADJ);
}

// One frame after its slopes are in the slope buffer with their tip/tilt
// partials; refresh: restart from the true residual b' - M c (q = M c from
// enq_refresh_mc) instead of Algorithm 1's recurrence (b' - b) + r.
void enq_frame_body(const Plan& P, const LaunchArgs& a, int iters, bool refresh);

// q = M c of every problem (the state's c): the operator chain on the second
// per-call table (in = state, out = q), before the frame's slopes take the
// slope buffer.
void enq_refresh_mc(const Plan& P, const LaunchArgs& a) {
  LaunchArgs b = a;
  b.IO = P.dIO2;
  enq_idwt(P, b, SRC_IN, OUT_PHI, 0);
  enq_apply_M_core(P, b);
  enq_fdwt(P, b, EPI_APPLYM, 0);
}

void enq_reconstruct(const Plan& P, const LaunchArgs& a, int iters, bool refresh = false) {
  if (refresh) enq_refresh_mc(P, a);
  launch_slopes_in(a, T(P, P.sin_frame), P.sin_frame.n);  // open loop: the measured slopes
  launch_pgamma(a, T(P, P.pg_pol), P.pg_pol.n, PG_POL_IN);  // closed loop: s + Gamma P a^(i-1)
  enq_frame_body(P, a, iters, refresh);
}

void enq_frame_body(const Plan& P, const LaunchArgs& a, int iters, bool refresh) {
  enq_adjoint(P, a, GT_WEIGHTED, PT_PHIADJ);
  enq_fdwt(P, a, refresh ? EPI_RHSQ : EPI_RHS, 0);
  // augmented PCG (Sec. 3.3): start projected against the previous frame's directions
  launch_aug_gram(a, T(P, P.aug), P.aug.n);
  launch_aug_init(a, T(P, P.aug), P.aug.n);
  for (int k = 0; k < iters; ++k) {
    launch_aug_p(a, T(P, P.aug), P.aug.n, k);  // p_k of the problems with augmentation
    enq_idwt(P, a, k == 0 ? SRC_PUPD0 : SRC_PUPD, OUT_PHI, k);
    enq_apply_M_core(P, a);
    enq_fdwt(P, a, EPI_PCG, k);
    // x updates in pairs of steps (bitwise the sequential ones): even steps
    // leave theirs to the next, odd steps take both; a last even step its own
    const int xm = (k & 1) ? UPD_X_PAIR : (k + 1 < iters ? UPD_X_DEFER : UPD_X_ONE);
    launch_update(a, T(P, P.upd), P.upd.n, k, nullptr, xm);
  }
  launch_aug_store(a, T(P, P.aug), P.aug.n, iters);  // the next frame's W and A W
  enq_idwt(P, a, SRC_STATE_C, OUT_FIT, 0);
  if (P.fit_cg.n > 0) {  // DM fitting: CG on (sum_k B_k^T M B_k + eps I) a = sum_k B_k^T M P_k phi
    launch_fit_fwd(a, T(P, P.fit_fwdL), P.fit_fwdL.n);
    launch_pT(a, T(P, P.fit_pt), P.fit_pt.n, PT_PHIADJ);
    launch_fit_cg(a, P.dF, P.fit_cg.n, FIT_INIT);
    for (int k = 0; k < P.max_fit_iters; ++k) {
      launch_fit_fwd(a, T(P, P.fit_fwdD), P.fit_fwdD.n);
      launch_pT(a, T(P, P.fit_pt), P.fit_pt.n, PT_PHIADJ);
      launch_fit_cg(a, P.dF, P.fit_cg.n, FIT_ITER);
    }
    launch_fit_cg(a, P.dF, P.fit_cg.n, FIT_FINAL);
  }
}

// Fixed-order sum of dot group `grp` of every problem, read back to the host.
fewha_status read_rho(Plan& P, hipStream_t st, int grp, int count_k, std::vector<double>& out, std::string& err) {
  for (int k = 0; k < P.nprob; ++k) {
    const ProbDev& pd = P.hP[k];
    HIP_TRY(hipMemcpyAsync(P.rho_host + P.rho_off[k], pd.dots + (long)grp * pd.n_dots, sizeof(double) * pd.n_dots,
                           hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  out.assign(P.nprob, 0.0);
  for (int k = 0; k < P.nprob; ++k) {
    const ProbDev& pd = P.hP[k];
    const int n = count_k == 0 ? pd.n_slots_fdwt : pd.n_slots_upd;
    double a = 0.0;
    for (int i = 0; i < n; ++i) a += P.rho_host[P.rho_off[k] + i];
    out[k] = a;
  }
  return FEWHA_OK;
}

// ---- coarse-level correction of the converged solves ----

// Coarse unknowns of problem k: the top-left s x s block of every layer's
// coefficients (s = min(side, n_l)), the side halved until the problem has
// at most kCoarseMax of them.
std::vector<int> coarse_indices(const Plan& P, int k, int side) {
  const ProbDev& pd = P.hP[k];
  for (int s = side; s >= 1; s /= 2) {
    std::vector<int> idx;
    for (int l = 0; l < pd.L; ++l) {
      const LayerDev& ly = P.hL[pd.layer0 + l];
      const int sl = std::min(s, ly.n);
      for (int i = 0; i < sl; ++i)
        for (int j = 0; j < sl; ++j) idx.push_back(ly.off + i * ly.n + j);
    }
    if ((int)idx.size() <= kCoarseMax) return idx;
  }
  return {};
}

// E^{-1} in FP32 from the symmetric part of E (FP64 Cholesky L L^T, then
// L^{-T} L^{-1}); false when E is not numerically positive definite.
bool spd_inverse(const std::vector<float>& E, int m, std::vector<float>& out) {
  std::vector<double> A((size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) A[(size_t)i * m + j] = 0.5 * ((double)E[(size_t)i * m + j] + (double)E[(size_t)j * m + i]);
  for (int j = 0; j < m; ++j) {
    double d = A[(size_t)j * m + j];
    for (int k = 0; k < j; ++k) d -= A[(size_t)j * m + k] * A[(size_t)j * m + k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    d = std::sqrt(d);
    A[(size_t)j * m + j] = d;
#pragma omp parallel for schedule(static)
    for (int i = j + 1; i < m; ++i) {
      double v = A[(size_t)i * m + j];
      for (int k = 0; k < j; ++k) v -= A[(size_t)i * m + k] * A[(size_t)j * m + k];
      A[(size_t)i * m + j] = v / d;
    }
  }
  // row c of Lt holds column c of L^{-1} (entries c .. m - 1)
  std::vector<double> Lt((size_t)m * m, 0.0);
#pragma omp parallel for schedule(dynamic, 8)
  for (int c = 0; c < m; ++c) {
    double* x = &Lt[(size_t)c * m];
    for (int i = c; i < m; ++i) {
      double v = i == c ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) v -= A[(size_t)i * m + k] * x[k];
      x[i] = v / A[(size_t)i * m + i];
    }
  }
  out.assign((size_t)m * m, 0.f);
#pragma omp parallel for schedule(dynamic, 8)
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) {
      double v = 0.0;
      for (int k = i; k < m; ++k) v += Lt[(size_t)i * m + k] * Lt[(size_t)j * m + k];
      out[(size_t)i * m + j] = out[(size_t)j * m + i] = (float)v;
    }
  return true;
}

// Builds the coarse-level correction of every problem: E = Z^T M Z column by
// column (M applied by the plan's own kernels to unit vectors; the instances
// of one system in a batch probe different columns in the same launch), E^{-1}
// on the host, and the device records of the solve kernels.  A system whose
// E is not positive definite is left uncorrected (m = 0: plain Jacobi).
fewha_status setup_coarse(Plan& P, hipStream_t st, std::string& err) {
  if (P.coarse_ready) return FEWHA_OK;
  if (P.coarse_mem) {
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipFree(P.coarse_mem));
    P.coarse_mem = nullptr;
  }
  P.dC = nullptr;
  P.dCT = nullptr;
  P.n_coarse_tiles = 0;
  P.coarse_m.assign(P.nprob, 0);
  if (P.coarse_side <= 0) {
    P.coarse_ready = true;
    return FEWHA_OK;
  }
  const int np = P.nprob;
  // systems: problems built from one configured context share M
  std::vector<int> sys(np), rank(np);
  std::vector<int> first, count;
  for (int k = 0; k < np; ++k) {
    int s = -1;
    for (size_t q = 0; q < first.size(); ++q)
      if (P.models[first[q]] == P.models[k]) s = (int)q;
    if (s < 0) {
      s = (int)first.size();
      first.push_back(k);
      count.push_back(0);
    }
    sys[k] = s;
    rank[k] = count[s]++;
  }
  const int ns = (int)first.size();
  std::vector<std::vector<int>> idx(ns);
  for (int s = 0; s < ns; ++s) idx[s] = coarse_indices(P, first[s], P.coarse_side);
  // temporary set-up memory: E per system, a unit vector and M e_j per problem, probe records
  size_t tb = 0;
  auto grab = [&](size_t& at, size_t bytes) {
    at = tb;
    tb += (bytes + 255) & ~size_t(255);
  };
  std::vector<size_t> oE(ns), oIdxT(ns), oIn(np), oOut(np);
  for (int s = 0; s < ns; ++s) {
    grab(oE[s], sizeof(float) * idx[s].size() * idx[s].size());
    grab(oIdxT[s], sizeof(int) * std::max<size_t>(idx[s].size(), 1));
  }
  for (int k = 0; k < np; ++k) {
    grab(oIn[k], sizeof(float) * P.hP[k].n_c);
    grab(oOut[k], sizeof(float) * P.hP[k].n_c);
  }
  size_t oQ;
  grab(oQ, sizeof(CoarseProbe) * np);
  char* tmp = nullptr;
  HIP_TRY(hipMalloc((void**)&tmp, tb));
  auto release = [&]() { (void)hipFree(tmp); };
  std::vector<CoarseProbe> hq(np);
  std::vector<IoDev> io(np);
  int rounds = 0;
  hipError_t e = hipSuccess;
  for (int s = 0; s < ns && e == hipSuccess; ++s)
    e = hipMemcpyAsync(tmp + oIdxT[s], idx[s].data(), sizeof(int) * idx[s].size(), hipMemcpyHostToDevice, st);
  for (int k = 0; k < np && e == hipSuccess; ++k) {
    const int s = sys[k], m = (int)idx[s].size();
    hq[k] = CoarseProbe{(float*)(tmp + oIn[k]), (const float*)(tmp + oOut[k]), (const int*)(tmp + oIdxT[s]),
                        (float*)(tmp + oE[s]), m, rank[k], count[s], 0};
    rounds = std::max(rounds, cdiv(m, count[s]));
    io[k] = IoDev{};
    io[k].in = hq[k].in;
    io[k].out = (float*)(tmp + oOut[k]);
    e = hipMemsetAsync(tmp + oIn[k], 0, sizeof(float) * P.hP[k].n_c, st);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(tmp + oQ, hq.data(), sizeof(CoarseProbe) * np, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) {
    release();
    err = std::string("coarse set-up: ") + hipGetErrorString(e);
    return FEWHA_EDEVICE;
  }
  fewha_status fs = upload_io(P, io, st, P.dIO, err);
  if (fs != FEWHA_OK) {
    release();
    return fs;
  }
  const LaunchArgs a = args(P, st, P.dIO);
  const CoarseProbe* dQ = (const CoarseProbe*)(tmp + oQ);
  for (int t = 0; t < rounds; ++t) {
    launch_coarse_probe(dQ, np, t, false, st);
    enq_idwt(P, a, SRC_IN, OUT_PHI, 0);
    enq_apply_M_core(P, a);
    enq_fdwt(P, a, EPI_APPLYM, 0);
    launch_coarse_probe(dQ, np, t, true, st);
  }
  e = hipGetLastError();
  std::vector<std::vector<float>> Einv(ns);
  for (int s = 0; s < ns && e == hipSuccess; ++s) {
    const int m = (int)idx[s].size();
    std::vector<float> E((size_t)m * m);
    e = hipMemcpyAsync(E.data(), tmp + oE[s], sizeof(float) * E.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && !spd_inverse(E, m, Einv[s])) {
      Einv[s].clear();
      idx[s].clear();
    }
  }
  release();
  if (e != hipSuccess) {
    err = std::string("coarse set-up: ") + hipGetErrorString(e);
    return FEWHA_EDEVICE;
  }
  // persistent memory: per system E^{-1} and indices; per problem zc and slots; records, tiles
  tb = 0;
  std::vector<size_t> oEi(ns), oIdx(ns), oZ(np), oS(np);
  std::vector<Tile> tiles;
  std::vector<CoarseDev> hc(np);
  for (int s = 0; s < ns; ++s) {
    grab(oEi[s], sizeof(float) * std::max<size_t>(Einv[s].size(), 1));
    grab(oIdx[s], sizeof(int) * std::max<size_t>(idx[s].size(), 1));
  }
  for (int k = 0; k < np; ++k) {
    const int m = (int)idx[sys[k]].size(), nb = cdiv(m, kCoarseRows);
    grab(oZ[k], sizeof(float) * P.hP[k].n_c);
    grab(oS[k], sizeof(double) * kDotRing * std::max(nb, 1));
    for (int b = 0; b < nb; ++b) tiles.push_back(Tile{k, 0, b, 0, b, 0, 0, 0});
    P.coarse_m[k] = m;
  }
  size_t oC, oT;
  grab(oC, sizeof(CoarseDev) * np);
  grab(oT, sizeof(Tile) * std::max<size_t>(tiles.size(), 1));
  char* mem = nullptr;
  HIP_TRY(hipMalloc((void**)&mem, tb));
  P.coarse_mem = mem;
  for (int k = 0; k < np; ++k) {
    const int s = sys[k], m = (int)idx[s].size();
    hc[k] = CoarseDev{(const float*)(mem + oEi[s]), (const int*)(mem + oIdx[s]), (float*)(mem + oZ[k]),
                      (double*)(mem + oS[k]), m, cdiv(m, kCoarseRows), {0, 0}};
    HIP_TRY(hipMemsetAsync(mem + oZ[k], 0, sizeof(float) * P.hP[k].n_c, st));
    HIP_TRY(hipMemsetAsync(mem + oS[k], 0, sizeof(double) * kDotRing * std::max(hc[k].n_slots, 1), st));
  }
  for (int s = 0; s < ns; ++s)
    if (!idx[s].empty()) {
      HIP_TRY(hipMemcpyAsync(mem + oEi[s], Einv[s].data(), sizeof(float) * Einv[s].size(), hipMemcpyHostToDevice, st));
      HIP_TRY(hipMemcpyAsync(mem + oIdx[s], idx[s].data(), sizeof(int) * idx[s].size(), hipMemcpyHostToDevice, st));
    }
  HIP_TRY(hipMemcpyAsync(mem + oC, hc.data(), sizeof(CoarseDev) * np, hipMemcpyHostToDevice, st));
  if (!tiles.empty())
    HIP_TRY(hipMemcpyAsync(mem + oT, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));  // the host vectors above go out of scope
  P.dC = (const CoarseDev*)(mem + oC);
  P.dCT = (const Tile*)(mem + oT);
  P.n_coarse_tiles = (int)tiles.size();
  P.coarse_ready = true;
  return FEWHA_OK;
}

// Correction solve M d = r (r in P.rbuf) by the FP32 Jacobi-preconditioned CG
// of Algorithm 1 from d = 0: the same kernels as a frame, one launch per
// stage and iteration over all problems; every kSolveCheck iterations the
// host reads rho_k and stops once sqrt(rho_k / rho_0) <= tol for every
// problem.  d is left in the x part of P.sstate.  With the coarse-level
// correction set up (setup_coarse), z = J^{-1} r + Z E^{-1} Z^T r: p_k is
// formed by k_coarse_p and rho_k includes (Z^T r)^T E^{-1} Z^T r; the
// convergence test keeps the Jacobi-weighted residual r^T J^{-1} r.
fewha_status pcg_core(Plan& P, hipStream_t st, int max_iters, double tol, int& iters, std::string& err) {
  std::vector<IoDev> io(P.nprob);
  for (int k = 0; k < P.nprob; ++k) {
    io[k].in = P.rbuf[k];
    io[k].state = P.sstate[k];
  }
  fewha_status s = upload_io(P, io, st, P.dIO, err);
  if (s != FEWHA_OK) return s;
  const LaunchArgs a = args(P, st, P.dIO);
  const CoarseDev* C = P.n_coarse_tiles > 0 ? P.dC : nullptr;
  launch_solve_init(a, T(P, P.sinit), P.sinit.n);
  if (C) launch_coarse(a, C, P.dCT, P.n_coarse_tiles, 0);
  std::vector<double> rho0, rho;
  if ((s = read_rho(P, st, 0, 0, rho0, err)) != FEWHA_OK) return s;
  auto worst = [&](const std::vector<double>& r) {
    double w = 0.0;
    for (int k = 0; k < P.nprob; ++k)
      if (rho0[k] > 0.0) w = std::max(w, std::sqrt(std::max(r[k], 0.0) / rho0[k]));
    return w;
  };
  double rel = worst(rho0);
  int k = 0;
  while (k < max_iters && rel > tol) {
    const int kend = std::min(max_iters, k + kSolveCheck);
    for (; k < kend; ++k) {
      if (C) launch_coarse_p(a, C, T(P, P.upd), P.upd.n, k);  // p_k with the coarse correction
      enq_idwt(P, a, C ? SRC_PJ : (k == 0 ? SRC_PUPD0 : SRC_PUPD), OUT_PHI, k);
      enq_apply_M_core(P, a);
      enq_fdwt(P, a, EPI_PCG, k);
      launch_update(a, T(P, P.upd), P.upd.n, k, C);
      if (C) launch_coarse(a, C, P.dCT, P.n_coarse_tiles, k + 1);
    }
    HIP_TRY(hipGetLastError());
    if ((s = read_rho(P, st, 2 * (k & (kDotRing - 1)), k, rho, err)) != FEWHA_OK) return s;
    rel = worst(rho);
  }
  iters = k;
  return FEWHA_OK;
}

// M x = b' with b' = b + W^{-T} A^T C_hat^{-1} s + W^{-T} g (each term optional)
// to a relative residual ||b' - M x|| / ||b'|| <= rtol by mixed-precision
// iterative refinement: x = 0; repeat { r = b' - M x in FP64; stop if small;
// M d = r by the FP32 PCG; x += d }, the iterate kept in FP64 and rounded to
// float once at the end.  The FP32 PCG alone stalls where the rounding of the
// FP32 operator dominates, and a right-hand side rounded to float moves the
// solution by M^{-1} times its rounding; forming b' inside the FP64 residual
// avoids both.  ||b'|| is the residual norm of the first sweep (x = 0).
fewha_status run_solve(Plan& P, hipStream_t st, const std::vector<const float*>& b,
                       const std::vector<const float*>& sl, const std::vector<const float*>& g,
                       const std::vector<float*>& x, int max_iters, double rtol, int* iters_done, double* rel_res,
                       std::string& err) {
  if (max_iters < 0 || max_iters > kMaxSolveIters || !(rtol >= 0.0)) {
    err = "solve: need 0 <= max_iters <= 2^24 and rtol >= 0";
    return FEWHA_EINVAL;
  }
  for (int k = 0; k < P.nprob; ++k)
    if (!x[k]) {
      err = "solve: null x (problem " + std::to_string(k) + ")";
      return FEWHA_EINVAL;
    }
  for (int k = 0; k < P.nprob; ++k)
    if (P.hP[k].aug_keep > 0) {
      err = "solve: not available with augmentation (the augmented PCG keeps a frame's directions); "
            "use a context without it";
      return FEWHA_ESTATE;
    }
  HIP_TRY(hipSetDevice(P.device));
  fewha_status s;
  if ((s = setup_coarse(P, st, err)) != FEWHA_OK) return s;
  std::vector<IoDev> io(P.nprob);
  auto stage = [&](auto fill) -> fewha_status {
    for (int k = 0; k < P.nprob; ++k) {
      io[k] = IoDev{};
      fill(k, io[k]);
    }
    return upload_io(P, io, st, P.dIO, err);
  };
  const LaunchArgs a = args(P, st, P.dIO);
  if ((s = stage([&](int k, IoDev& d) { d.state = x[k]; })) != FEWHA_OK) return s;
  launch64_iterate(a, T(P, P.upd), P.upd.n, 0);
  int total = 0;
  double rel = 0.0, prev = HUGE_VAL;
  std::vector<double> bnorm(P.nprob, 0.0);
  for (int sweep = 0;; ++sweep) {
    if ((s = stage([&](int k, IoDev& d) {
           d.in = b[k];
           d.rs = sl[k];
           d.rg = g[k];
           d.out = P.rbuf[k];
         })) != FEWHA_OK)
      return s;
    launch64_resid_chain(a, P.r64, P.F64);
    HIP_TRY(hipGetLastError());
    for (int k = 0; k < P.nprob; ++k) {
      const ProbDev& pd = P.hP[k];
      HIP_TRY(hipMemcpyAsync(P.rho_host + P.rho_off[k], pd.rslots, sizeof(double) * 2 * pd.n_slots_upd,
                             hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    rel = 0.0;
    for (int k = 0; k < P.nprob; ++k) {
      double rr = 0.0;
      for (int i = 0; i < P.hP[k].n_slots_upd; ++i) rr += P.rho_host[P.rho_off[k] + 2 * i];
      if (sweep == 0) bnorm[k] = std::sqrt(rr);
      if (bnorm[k] > 0.0) rel = std::max(rel, std::sqrt(rr) / bnorm[k]);
    }
    // stop: converged, out of iterations, or a sweep that no longer helps
    if (rel <= rtol || total >= max_iters || sweep >= kMaxSweeps || rel > 0.5 * prev) break;
    prev = rel;
    const double inner = std::max(1e-4, std::min(0.1, 0.3 * rtol / rel));
    int it = 0;
    if ((s = pcg_core(P, st, max_iters - total, inner, it, err)) != FEWHA_OK) return s;
    total += it;
    if ((s = stage([&](int k, IoDev& d) { d.in = P.sstate[k]; })) != FEWHA_OK) return s;
    launch64_iterate(a, T(P, P.upd), P.upd.n, 1);
  }
  if ((s = stage([&](int k, IoDev& d) { d.state = x[k]; })) != FEWHA_OK) return s;
  launch64_iterate(a, T(P, P.upd), P.upd.n, 2);
  HIP_TRY(hipGetLastError());
  if (iters_done) *iters_done = total;
  if (rel_res) *rel_res = rel;
  return FEWHA_OK;
}

// phi = W^{-1} c = delta^{-1} W^T c per layer (inverse transform to a caller buffer).
fewha_status run_winv(Plan& P, hipStream_t st, const std::vector<const float*>& in, const std::vector<float*>& out,
                      std::string& err) {
  std::vector<IoDev> io(P.nprob);
  for (int k = 0; k < P.nprob; ++k) {
    if (!in[k] || !out[k]) {
      err = "apply_Winv: null pointer";
      return FEWHA_EINVAL;
    }
    io[k].in = in[k];
    io[k].out = out[k];
  }
  HIP_TRY(hipSetDevice(P.device));
  fewha_status s = upload_io(P, io, st, P.dIO, err);
  if (s != FEWHA_OK) return s;
  enq_idwt(P, args(P, st, P.dIO), SRC_IN, OUT_USER, 0);
  HIP_TRY(hipGetLastError());
  return FEWHA_OK;
}

// c = W^{-T} phi = delta^{-1} W phi per layer (forward transform of a caller buffer).
fewha_status run_winvT(Plan& P, hipStream_t st, const std::vector<const float*>& in, const std::vector<float*>& out,
                       std::string& err) {
  std::vector<IoDev> io(P.nprob);
  HIP_TRY(hipSetDevice(P.device));
  for (int k = 0; k < P.nprob; ++k) {
    if (!in[k] || !out[k]) {
      err = "apply_WinvT: null pointer";
      return FEWHA_EINVAL;
    }
    HIP_TRY(hipMemcpyAsync(P.hP[k].phiadj, in[k], sizeof(float) * P.hP[k].n_c, hipMemcpyDeviceToDevice, st));
    io[k].out = out[k];
  }
  fewha_status s = upload_io(P, io, st, P.dIO, err);
  if (s != FEWHA_OK) return s;
  enq_fdwt(P, args(P, st, P.dIO), EPI_PLAIN, 0);
  HIP_TRY(hipGetLastError());
  return FEWHA_OK;
}

// Gradients of a loss of the layers phi = W^{-1} c*, c* = M^{-1} b, with respect to
// alpha, the Cn2 weights and the layer heights, given the adjoint solution
// lambda = M^{-1} W^{-T} dL/dphi:
//   g_alpha   = -lambda^T D c
//   g_gamma_l = alpha lambda_l^T D_l c_l / gamma_l           (D_l scales as 1/gamma_l)
//   g_h_l     = <dA_l W^{-1} lambda, C_hat^{-1} (s - A phi)> - <C_hat^{-1} A W^{-1} lambda, dA_l phi>
// with dA_l = d A / d h_l.  The loss's own dependence on h is the caller's.
fewha_status run_param_grads(Plan& P, hipStream_t st, const std::vector<const float*>& slopes,
                             const std::vector<const float*>& c, const std::vector<const float*>& lam,
                             const std::vector<double*>& out, std::string& err) {
  for (int k = 0; k < P.nprob; ++k) {
    if (!slopes[k] || !c[k] || !lam[k] || !out[k]) {
      err = "param_grads: null pointer (problem " + std::to_string(k) + ")";
      return FEWHA_EINVAL;
    }
    if (!P.models[k]->grad_ok) {
      err = "param_grads: " + P.models[k]->grad_msg;
      return FEWHA_EGEOM;
    }
  }
  HIP_TRY(hipSetDevice(P.device));
  const int n = P.nprob;
  std::vector<IoDev> io(n);
  fewha_status s;
  const LaunchArgs a = args(P, st, P.dIO);
  auto stage = [&](auto fill) -> fewha_status {
    for (int k = 0; k < n; ++k) {
      io[k] = IoDev{};
      fill(k, io[k]);
    }
    return upload_io(P, io, st, P.dIO, err);
  };
  // W^{-1} c and W^{-1} lambda
  if ((s = stage([&](int k, IoDev& d) { d.in = c[k]; d.out = P.hP[k].gphi; })) != FEWHA_OK) return s;
  enq_idwt(P, a, SRC_IN, OUT_USER, 0);
  if ((s = stage([&](int k, IoDev& d) { d.in = lam[k]; d.out = P.hP[k].glam; })) != FEWHA_OK) return s;
  enq_idwt(P, a, SRC_IN, OUT_USER, 0);
  // term 0: Gamma^T C_hat^{-1} (s - A phi) against dA W^{-1} lambda
  if ((s = stage([&](int k, IoDev& d) { d.in = slopes[k]; })) != FEWHA_OK) return s;
  launch_slopes_in(a, T(P, P.sin), P.sin.n);
  if ((s = stage([&](int k, IoDev& d) { d.in = P.hP[k].gphi; })) != FEWHA_OK) return s;
  launch_pgamma(a, T(P, P.pg), P.pg.n, PG_RESID_IN);
  launch_gammaT(a, T(P, P.gt), P.gt.n, GT_WEIGHTED);
  launch_grad_height(a, T(P, P.ghgt), P.ghgt.n, 0);
  // term 1: Gamma^T C_hat^{-1} A W^{-1} lambda against dA phi
  if ((s = stage([&](int k, IoDev& d) { d.in = P.hP[k].glam; })) != FEWHA_OK) return s;
  launch_pgamma(a, T(P, P.pg), P.pg.n, PG_DENSE_IN);
  launch_gammaT(a, T(P, P.gt), P.gt.n, GT_WEIGHTED);
  launch_grad_height(a, T(P, P.ghgt), P.ghgt.n, 1);
  // prior terms and the fixed-order reductions
  std::vector<GradIo> g(n);
  for (int k = 0; k < n; ++k) g[k] = GradIo{c[k], lam[k], out[k]};
  if ((s = upload_table(P, g, st, P.dGIO, err)) != FEWHA_OK) return s;
  launch_grad_prior(a, P.dGIO, T(P, P.gprior), P.gprior.n);
  launch_grad_final(a, P.dGIO, n);
  HIP_TRY(hipGetLastError());
  return FEWHA_OK;
}

}  // namespace

// ------------------------------------------------------------ C ABI

struct fewha_ctx {
  int device = -1;
  hipStream_t stream = nullptr;
  bool finalized = false;
  long frames = 0;        // frames reconstructed so far (the restart schedule's clock)
  int refresh_every = 0;  // restart from the true residual every this many frames (0 = never)
  int coarse_side = kCoarseSide;  // coarse-level correction of the converged solves (0 = Jacobi only)
  std::string err;
  HostModel m;
  Plan* plan = nullptr;
};

struct fewha_batch {
  std::vector<fewha_ctx*> ctxs;
  Plan* plan = nullptr;
  hipStream_t stream = nullptr;
  std::string err;
  long frames = 0;        // as fewha_ctx, for every problem of the batch
  int refresh_every = 0;
  // frame path in parts (tuning streams > 1): contiguous slices of the
  // problem list, each with its own plan and stream; fork / join events
  std::vector<Plan*> parts;
  std::vector<int> part_first;
  std::vector<hipStream_t> part_stream;
  std::vector<hipEvent_t> part_done;
  hipEvent_t fork = nullptr;
};

static void destroy_batch_parts(fewha_batch* b) {
  for (Plan*& q : b->parts) destroy_plan(q);
  for (hipStream_t s : b->part_stream)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->part_done)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  b->parts.clear();
  b->part_stream.clear();
  b->part_done.clear();
  b->fork = nullptr;
}

#define CHECK_CTX(c)                 \
  do {                               \
    if (!(c)) return FEWHA_EINVAL;   \
  } while (0)

static fewha_status fail(fewha_ctx* c, fewha_status s, const std::string& msg) {
  c->err = msg;
  return s;
}

extern "C" {

fewha_status fewha_create(fewha_ctx** out, int device) {
  if (!out) return FEWHA_EINVAL;
  *out = nullptr;
  fewha_ctx* c = new (std::nothrow) fewha_ctx();
  if (!c) return FEWHA_ENOMEM;
  c->device = device;
  if (device >= 0) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device >= n || hipSetDevice(device) != hipSuccess) {
      delete c;
      return FEWHA_EDEVICE;
    }
  }
  *out = c;
  return FEWHA_OK;
}

fewha_status fewha_set_stream(fewha_ctx* c, void* s) {
  CHECK_CTX(c);
  c->stream = (hipStream_t)s;
  return FEWHA_OK;
}

fewha_status fewha_set_pupil(fewha_ctx* c, double D, double obs) {
  CHECK_CTX(c);
  if (c->finalized) return fail(c, FEWHA_ESTATE, "set_pupil after finalize");
  if (!(D > 0.0) || !(obs >= 0.0 && obs < 1.0)) return fail(c, FEWHA_EINVAL, "set_pupil: need D > 0, 0 <= obstruction < 1");
  c->m.D = D;
  c->m.obs = obs;
  c->m.have_pupil = true;
  return FEWHA_OK;
}

fewha_status fewha_set_wfs(fewha_ctx* c, int G, const fewha_wfs_desc* w) {
  CHECK_CTX(c);
  if (c->finalized) return fail(c, FEWHA_ESTATE, "set_wfs after finalize");
  if (G < 1 || G > 1024 || !w) return fail(c, FEWHA_EINVAL, "set_wfs: need 1 <= G <= 1024 and a descriptor array");
  std::vector<WfsHost> v(G);
  for (int g = 0; g < G; ++g) {
    const fewha_wfs_desc& d = w[g];
    if ((d.kind != FEWHA_NGS && d.kind != FEWHA_LGS) || d.n_subap < 1 || d.n_subap > 4096 || !(d.sigma > 0.0) ||
        (d.kind == FEWHA_LGS && !(d.H > 0.0)))
      return fail(c, FEWHA_EINVAL, "set_wfs: sensor " + std::to_string(g) + " has an invalid descriptor");
    v[g].d = d;
    v[g].d.mask = nullptr;
    if (d.mask) v[g].mask.assign(d.mask, d.mask + (size_t)d.n_subap * d.n_subap);
    for (auto& b : v[g].mask) b = b ? 1 : 0;
  }
  c->m.wfs = std::move(v);
  c->m.have_wfs = true;
  return FEWHA_OK;
}

fewha_status fewha_set_layers(fewha_ctx* c, int L, const fewha_layer_desc* l, double side) {
  CHECK_CTX(c);
  if (c->finalized) return fail(c, FEWHA_ESTATE, "set_layers after finalize");
  if (L < 1 || L > 64 || !l || !(side > 0.0)) return fail(c, FEWHA_EINVAL, "set_layers: need 1 <= L <= 64, side > 0");
  c->m.layers.assign(L, LayerHost());
  for (int i = 0; i < L; ++i) c->m.layers[i].d = l[i];
  c->m.L = side;
  c->m.have_layers = true;
  return FEWHA_OK;
}

fewha_status fewha_set_prior(fewha_ctx* c, double alpha, double r0, double L0, double tau) {
  CHECK_CTX(c);
  if (c->finalized) return fail(c, FEWHA_ESTATE, "set_prior after finalize");
  if (!(alpha > 0.0) || !(r0 > 0.0) || !(L0 > 0.0) || !(tau >= 0.0))
    return fail(c, FEWHA_EINVAL, "set_prior: need alpha, r0, L0 > 0 and tau >= 0");
  c->m.alpha = alpha;
  c->m.r0 = r0;
  c->m.L0 = L0;
  c->m.tau = tau;
  return FEWHA_OK;
}

fewha_status fewha_set_noise(fewha_ctx* c, double alpha_eta, double na_fwhm, double spot_fwhm) {
  CHECK_CTX(c);
  if (c->finalized) return fail(c, FEWHA_ESTATE, "set_noise after finalize");
  if (!(alpha_eta >= 0.0) || !(na_fwhm >= 0.0) || !(spot_fwhm > 0.0))
    return fail(c, FEWHA_EINVAL, "set_noise: need alpha_eta >= 0, na_fwhm >= 0, spot_fwhm > 0");
  c->m.alpha_eta = alpha_eta;
  c->m.na_fwhm = na_fwhm;
  c->m.spot_fwhm = spot_fwhm;
  return FEWHA_OK;
}

fewha_status fewha_set_control(fewha_ctx* c, double gain) {
  CHECK_CTX(c);
  if (c->finalized) return fail(c, FEWHA_ESTATE, "set_control after finalize");
  if (!(gain >= 0.0 && gain <= 1.0)) return fail(c, FEWHA_EINVAL, "set_control: gain must lie in [0, 1]");
  c->m.gain = gain;
  return FEWHA_OK;
}

fewha_status fewha_set_loop(fewha_ctx* c, int closed) {
  CHECK_CTX(c);
  if (c->finalized) return fail(c, FEWHA_ESTATE, "set_loop after finalize");
  if (closed != 0 && closed != 1) return fail(c, FEWHA_EINVAL, "set_loop: closed must be 0 or 1");
  c->m.closed = closed == 1;
  return FEWHA_OK;
}

fewha_status fewha_set_augmentation(fewha_ctx* c, int keep) {
  CHECK_CTX(c);
  if (c->finalized) return fail(c, FEWHA_ESTATE, "set_augmentation after finalize");
  if (keep < 0 || keep > kAugMax)
    return fail(c, FEWHA_EINVAL, "set_augmentation: keep must lie in [0, " + std::to_string(kAugMax) + "]");
  c->m.aug_keep = keep;
  return FEWHA_OK;
}

fewha_status fewha_set_photons(fewha_ctx* c, int G, const double* n_photons) {
  CHECK_CTX(c);
  if (c->finalized) return fail(c, FEWHA_ESTATE, "set_photons after finalize");
  if (!c->m.have_wfs) return fail(c, FEWHA_ESTATE, "set_photons: call fewha_set_wfs first");
  if (G != (int)c->m.wfs.size() || !n_photons)
    return fail(c, FEWHA_EINVAL, "set_photons: need one photon count per sensor");
  for (int g = 0; g < G; ++g)
    if (!(n_photons[g] > 0.0) || !std::isfinite(n_photons[g]))
      return fail(c, FEWHA_EINVAL, "set_photons: sensor " + std::to_string(g) + " needs a positive photon count");
  for (int g = 0; g < G; ++g) c->m.wfs[g].d.sigma = 1.0 / std::sqrt(n_photons[g]);
  return FEWHA_OK;
}

fewha_status fewha_set_fitting(fewha_ctx* c, int n_dm, const fewha_dm_desc* dms, int n_dirs, const double* dirs_xy,
                               int n_fit, int fit_iters, double eps_rel) {
  CHECK_CTX(c);
  if (c->finalized) return fail(c, FEWHA_ESTATE, "set_fitting after finalize");
  if (n_dm < 1 || n_dm > 16 || !dms || n_dirs < 1 || n_dirs > 256 || !dirs_xy || n_fit < 1 || n_fit > 4096 ||
      fit_iters < 0 || fit_iters > 256 || !(eps_rel >= 0.0))
    return fail(c, FEWHA_EINVAL, "set_fitting: invalid argument");
  for (int q = 0; q < n_dm; ++q)
    if (dms[q].n_act < 2 || dms[q].n_act > 4096 || !(dms[q].pitch > 0.0))
      return fail(c, FEWHA_EINVAL, "set_fitting: DM " + std::to_string(q) + " has an invalid descriptor");
  FitHost& f = c->m.fit;
  f.on = true;
  f.dms.assign(dms, dms + n_dm);
  f.dirs.assign(dirs_xy, dirs_xy + 2 * n_dirs);
  f.N = n_fit;
  f.iters = fit_iters;
  f.eps_rel = eps_rel;
  return FEWHA_OK;
}

fewha_status fewha_set_tuning(fewha_ctx* c, const fewha_tuning* t) {
  CHECK_CTX(c);
  if (c->finalized) return fail(c, FEWHA_ESTATE, "set_tuning after finalize");
  if (!t) return fail(c, FEWHA_EINVAL, "set_tuning: null tuning");
  for (int i = 0; i < 2; ++i)
    if (t->reserved[i]) return fail(c, FEWHA_EINVAL, "set_tuning: reserved fields must be zero");
  if (t->glob_fuse != 0 && t->glob_fuse != 1) return fail(c, FEWHA_EINVAL, "set_tuning: glob_fuse must be 0 or 1");
  if (t->pt_split != 0 && t->pt_split != 1) return fail(c, FEWHA_EINVAL, "set_tuning: pt_split must be 0 or 1");
  if (t->pt_split && t->pt_rows == 8)
    return fail(c, FEWHA_EINVAL, "set_tuning: pt_split needs pt_rows 0 or 4");
  if (t->res_split != 0 && t->res_split != 1 && t->res_split != 4)
    return fail(c, FEWHA_EINVAL, "set_tuning: res_split must be 0, 1 or 4");
  if (t->streams != 0 && t->streams != 1)
    return fail(c, FEWHA_EINVAL, "set_tuning: a context runs one stream (streams 0 or 1)");
  if (t->dwt_resident != 0 && t->dwt_resident != 32 && t->dwt_resident != 64 && t->dwt_resident != 128)
    return fail(c, FEWHA_EINVAL, "set_tuning: dwt_resident must be 0, 32, 64 or 128");
  if (t->pt_rows != 0 && t->pt_rows != 4 && t->pt_rows != 8)
    return fail(c, FEWHA_EINVAL, "set_tuning: pt_rows must be 0, 4 or 8");
  c->m.tune_res = t->dwt_resident;
  c->m.tune_pt_rows = t->pt_rows;
  c->m.tune_split = t->res_split;
  c->m.tune_pt_split = t->pt_split;
  c->m.tune_glob_fuse = t->glob_fuse;
  return FEWHA_OK;
}

fewha_status fewha_finalize(fewha_ctx* c) {
  CHECK_CTX(c);
  if (c->finalized) return fail(c, FEWHA_ESTATE, "finalize called twice");
  if (c->m.closed && c->m.fit.on)
    return fail(c, FEWHA_EINVAL, "closed loop needs F = I (the layers at the DM altitudes): no fitting step");
  fewha_status s = build_model(c->m, c->err);
  if (s != FEWHA_OK) return s;
  if (c->device >= 0) {
    std::vector<const HostModel*> ms{&c->m};
    s = build_plan(c->plan, ms, c->device, c->m.tune_res > 0 ? c->m.tune_res : kResMax,
                   c->m.tune_pt_rows > 0 ? c->m.tune_pt_rows : 4, c->m.tune_split, c->m.tune_pt_split,
                   c->m.tune_glob_fuse, c->err);
    if (s != FEWHA_OK) return s;
    c->plan->coarse_side = c->coarse_side;
    if ((s = setup_noalloc(*c->plan, c->err)) != FEWHA_OK ||
        (s = setup_streamed(*c->plan, c->m.n_slopes, (int)c->m.wfs.size(), c->err)) != FEWHA_OK) {
      destroy_plan(c->plan);
      c->plan = nullptr;
      return s;
    }
  }
  c->finalized = true;
  return FEWHA_OK;
}

fewha_status fewha_sizes(const fewha_ctx* c, long* n_coeff, long* n_slopes, long* n_layer_pts, long* n_act,
                         long* n_state) {
  if (!c) return FEWHA_EINVAL;
  if (!c->finalized) return FEWHA_ESTATE;
  if (n_coeff) *n_coeff = c->m.n_c;
  if (n_slopes) *n_slopes = c->m.n_slopes;
  if (n_layer_pts) *n_layer_pts = c->m.n_c;
  if (n_act) *n_act = c->m.n_act();
  if (n_state) *n_state = c->m.n_state();
  return FEWHA_OK;
}

fewha_status fewha_get_table(const fewha_ctx* c, int which, double* out, long n) {
  if (!c || !out) return FEWHA_EINVAL;
  if (!c->finalized) return FEWHA_ESTATE;
  std::vector<double> v;
  switch (which) {
    case FEWHA_TABLE_FILTER:
      v.assign(c->m.h, c->m.h + 6);
      break;
    case FEWHA_TABLE_PRIOR:
      v = c->m.Dprior;
      break;
    case FEWHA_TABLE_PRECOND:
      v = c->m.J;
      break;
    case FEWHA_TABLE_MASK:
      for (const WfsHost& w : c->m.wfs)
        for (uint8_t b : w.mask) v.push_back(b);
      break;
    default:
      return FEWHA_EINVAL;
  }
  if (n < (long)v.size()) return FEWHA_EINVAL;
  std::copy(v.begin(), v.end(), out);
  return FEWHA_OK;
}

// Frame f (0-based) restarts from the true residual when f > 0 and f is a
// multiple of the refresh period.
static bool refresh_due(long frames, int every) { return every > 0 && frames > 0 && frames % every == 0; }

static fewha_status ready(fewha_ctx* c) {
  if (!c) return FEWHA_EINVAL;
  if (!c->finalized) return fail(c, FEWHA_ESTATE, "context not finalized");
  if (c->device < 0 || !c->plan) return fail(c, FEWHA_ESTATE, "host-only context: no device");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, FEWHA_EDEVICE, "hipSetDevice failed");
  return take_numeric(*c->plan, c->err);
}

static fewha_status finish(fewha_ctx* c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, FEWHA_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return FEWHA_OK;
}

fewha_status fewha_apply_A(fewha_ctx* c, const float* layers, float* slopes) {
  fewha_status s = ready(c);
  if (s != FEWHA_OK) return s;
  if (!layers || !slopes) return fail(c, FEWHA_EINVAL, "apply_A: null pointer");
  Plan& P = *c->plan;
  std::vector<IoDev> io(1);
  io[0].in = layers;
  io[0].out = slopes;
  if ((s = upload_io(P, io, c->stream, P.dIO, c->err)) != FEWHA_OK) return s;
  LaunchArgs a = args(P, c->stream, P.dIO);
  launch_pgamma(a, T(P, P.pg), P.pg.n, PG_COMPACT);
  return finish(c);
}

fewha_status fewha_apply_AT(fewha_ctx* c, const float* slopes, float* layers) {
  fewha_status s = ready(c);
  if (s != FEWHA_OK) return s;
  if (!layers || !slopes) return fail(c, FEWHA_EINVAL, "apply_AT: null pointer");
  Plan& P = *c->plan;
  std::vector<IoDev> io(1);
  io[0].in = slopes;
  io[0].out = layers;
  if ((s = upload_io(P, io, c->stream, P.dIO, c->err)) != FEWHA_OK) return s;
  LaunchArgs a = args(P, c->stream, P.dIO);
  launch_slopes_in(a, T(P, P.sin), P.sin.n);
  enq_adjoint(P, a, GT_PLAIN, PT_USER);
  return finish(c);
}

fewha_status fewha_apply_M(fewha_ctx* c, const float* x, float* Mx) {
  fewha_status s = ready(c);
  if (s != FEWHA_OK) return s;
  if (!x || !Mx) return fail(c, FEWHA_EINVAL, "apply_M: null pointer");
  Plan& P = *c->plan;
  std::vector<IoDev> io(1);
  io[0].in = x;
  io[0].out = Mx;
  if ((s = upload_io(P, io, c->stream, P.dIO, c->err)) != FEWHA_OK) return s;
  LaunchArgs a = args(P, c->stream, P.dIO);
  enq_idwt(P, a, SRC_IN, OUT_PHI, 0);
  enq_apply_M_core(P, a);
  enq_fdwt(P, a, EPI_APPLYM, 0);
  return finish(c);
}

fewha_status fewha_rhs(fewha_ctx* c, const float* slopes, float* b) {
  fewha_status s = ready(c);
  if (s != FEWHA_OK) return s;
  if (!slopes || !b) return fail(c, FEWHA_EINVAL, "rhs: null pointer");
  Plan& P = *c->plan;
  std::vector<IoDev> io(1);
  io[0].in = slopes;
  io[0].out = b;
  if ((s = upload_io(P, io, c->stream, P.dIO, c->err)) != FEWHA_OK) return s;
  LaunchArgs a = args(P, c->stream, P.dIO);
  launch_slopes_in(a, T(P, P.sin), P.sin.n);
  enq_adjoint(P, a, GT_WEIGHTED, PT_PHIADJ);
  enq_fdwt(P, a, EPI_PLAIN, 0);
  return finish(c);
}

fewha_status fewha_reconstruct(fewha_ctx* c, const float* slopes, float* state, float* layers_out, float* dm_out,
                               int iters) {
  fewha_status s = ready(c);
  if (s != FEWHA_OK) return s;
  if (!slopes || !state) return fail(c, FEWHA_EINVAL, "reconstruct: null slopes or state");
  if (iters < 0 || iters > kMaxIters) return fail(c, FEWHA_EINVAL, "reconstruct: iters must lie in [0, 256]");
  if (((uintptr_t)state & 15) != 0) return fail(c, FEWHA_EINVAL, "reconstruct: state must be 16-byte aligned");
  Plan& P = *c->plan;
  std::vector<IoDev> io(1);
  io[0].in = slopes;
  io[0].state = state;
  io[0].layers_out = layers_out;
  io[0].dm_out = dm_out;
  if ((s = upload_io(P, io, c->stream, P.dIO, c->err)) != FEWHA_OK) return s;
  const bool refresh = refresh_due(c->frames, c->refresh_every);
  if (refresh && (s = upload_refresh_io(P, io, c->stream, c->err)) != FEWHA_OK) return s;
  LaunchArgs a = args(P, c->stream, P.dIO);
  enq_reconstruct(P, a, iters, refresh);
  ++c->frames;
  return finish(c);
}

fewha_status fewha_set_refresh(fewha_ctx* c, int every) {
  CHECK_CTX(c);
  if (every < 0) return fail(c, FEWHA_EINVAL, "set_refresh: every must be >= 0");
  c->refresh_every = every;
  return FEWHA_OK;
}

static bool coarse_side_ok(int side) { return side == 0 || (side >= 1 && side <= 64 && (side & (side - 1)) == 0); }

fewha_status fewha_set_solve_coarse(fewha_ctx* c, int side) {
  CHECK_CTX(c);
  if (!coarse_side_ok(side))
    return fail(c, FEWHA_EINVAL, "set_solve_coarse: side must be 0 or a power of two up to 64");
  c->coarse_side = side;
  if (c->plan && c->plan->coarse_side != side) {
    c->plan->coarse_side = side;
    c->plan->coarse_ready = false;
  }
  return FEWHA_OK;
}

fewha_status fewha_set_frame_count(fewha_ctx* c, long frames) {
  CHECK_CTX(c);
  if (frames < 0) return fail(c, FEWHA_EINVAL, "set_frame_count: frames must be >= 0");
  c->frames = frames;
  return FEWHA_OK;
}

fewha_status fewha_reconstruct_noalloc(fewha_ctx* c, const float* slopes, float* state, float* layers_out,
                                       float* dm_out, int iters) {
  fewha_status s = ready(c);
  if (s != FEWHA_OK) return s;
  if (!slopes || !state) return fail(c, FEWHA_EINVAL, "reconstruct_noalloc: null slopes or state");
  if (iters < 0 || iters > kMaxIters) return fail(c, FEWHA_EINVAL, "reconstruct_noalloc: iters must lie in [0, 256]");
  if (((uintptr_t)state & 15) != 0) return fail(c, FEWHA_EINVAL, "reconstruct_noalloc: state must be 16-byte aligned");
  Plan& P = *c->plan;
  if (c->m.fit.on || c->m.aug_keep > 0 || c->refresh_every > 0)
    return fail(c, FEWHA_EINVAL,
                "reconstruct_noalloc: not available with the DM fitting step, augmentation or residual refresh");
  if (P.na_bytes > kNoAllocBytes)
    return fail(c, FEWHA_EINVAL, "reconstruct_noalloc: the frame needs " + std::to_string(P.na_bytes) +
                                     " bytes of scratch; the static scratch holds " + std::to_string(kNoAllocBytes));
  // the per-call table through a pinned slot of the ring (no host or device allocation)
  const int slot = P.ring;
  P.ring = (P.ring + 1) % kRing;
  if (P.ev_used[slot] && hipEventSynchronize(P.ev[slot]) != hipSuccess)
    return fail(c, FEWHA_EDEVICE, "reconstruct_noalloc: staging event failed");
  IoDev* io = P.pinned[slot];
  std::memset(io, 0, sizeof(IoDev) * P.nprob_all);
  io[0].in = slopes;
  io[0].state = state;
  io[0].layers_out = layers_out;
  io[0].dm_out = dm_out;
  if (hipMemcpyAsync(P.na_io, io, sizeof(IoDev) * P.nprob_all, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipEventRecord(P.ev[slot], c->stream) != hipSuccess)
    return fail(c, FEWHA_EDEVICE, "reconstruct_noalloc: staging copy failed");
  P.ev_used[slot] = true;
  LaunchArgs a = args(P, c->stream, P.na_io);
  a.P = P.dPna;
  enq_reconstruct(P, a, iters);
  ++c->frames;
  return finish(c);
}

fewha_status fewha_reconstruct_streamed(fewha_ctx* c, const float* host_slopes, float* state, float* layers_out,
                                        float* dm_out, int iters, int chunks) {
  fewha_status s = ready(c);
  if (s != FEWHA_OK) return s;
  if (!host_slopes || !state) return fail(c, FEWHA_EINVAL, "reconstruct_streamed: null slopes or state");
  if (iters < 0 || iters > kMaxIters) return fail(c, FEWHA_EINVAL, "reconstruct_streamed: iters must lie in [0, 256]");
  if (((uintptr_t)state & 15) != 0) return fail(c, FEWHA_EINVAL, "reconstruct_streamed: state must be 16-byte aligned");
  Plan& P = *c->plan;
  const HostModel& m = c->m;
  const int G = (int)m.wfs.size();
  if (chunks < 1 || chunks > (int)P.chunk_ev.size())
    return fail(c, FEWHA_EINVAL, "reconstruct_streamed: chunks must lie in [1, min(sensors, 64)]");
  std::string& err = c->err;
  const hipStream_t st = c->stream;
  // the copies wait for earlier work on the stream (the previous frame reads the buffer)
  HIP_TRY(hipEventRecord(P.copy_start, st));
  HIP_TRY(hipStreamWaitEvent(P.copy_stream, P.copy_start, 0));
  auto soff = [&](int g) { return g < G ? (long)m.slope_off[g] : m.n_slopes; };
  for (int q = 0; q < chunks; ++q) {
    const int g0 = (int)((long)G * q / chunks), g1 = (int)((long)G * (q + 1) / chunks);
    const long o = soff(g0), n = soff(g1) - o;
    if (n > 0)
      HIP_TRY(hipMemcpyAsync(P.dslopes + o, host_slopes + o, sizeof(float) * n, hipMemcpyHostToDevice, P.copy_stream));
    HIP_TRY(hipEventRecord(P.chunk_ev[q], P.copy_stream));
  }
  std::vector<IoDev> io(1);
  io[0].in = P.dslopes;
  io[0].state = state;
  io[0].layers_out = layers_out;
  io[0].dm_out = dm_out;
  if ((s = upload_io(P, io, st, P.dIO, err)) != FEWHA_OK) return s;
  const bool refresh = refresh_due(c->frames, c->refresh_every);
  if (refresh && (s = upload_refresh_io(P, io, st, err)) != FEWHA_OK) return s;
  const LaunchArgs a = args(P, st, P.dIO);
  if (refresh) enq_refresh_mc(P, a);
  // closed loop: the mirrors' part of the pseudo-open-loop slopes while the measurement arrives
  if (m.closed) launch_pgamma(a, T(P, P.pg), P.pg.n, PG_APREV);
  for (int q = 0; q < chunks; ++q) {
    const int g0 = (int)((long)G * q / chunks), g1 = (int)((long)G * (q + 1) / chunks);
    HIP_TRY(hipStreamWaitEvent(st, P.chunk_ev[q], 0));
    launch_slopes_in(a, T(P, P.sin) + P.sin_g[g0], P.sin_g[g1] - P.sin_g[g0], m.closed ? 1 : 0);
  }
  enq_frame_body(P, a, iters, refresh);
  ++c->frames;
  return finish(c);
}

fewha_status fewha_solve(fewha_ctx* c, const float* rhs, float* x, int max_iters, double rtol, int* iters_done,
                         double* rel_res) {
  fewha_status s = ready(c);
  if (s != FEWHA_OK) return s;
  if (!rhs) return fail(c, FEWHA_EINVAL, "solve: null rhs");
  return run_solve(*c->plan, c->stream, {rhs}, {nullptr}, {nullptr}, {x}, max_iters, rtol, iters_done, rel_res,
                   c->err);
}

fewha_status fewha_solve_map(fewha_ctx* c, const float* slopes, const float* g_layers, float* x, int max_iters,
                             double rtol, int* iters_done, double* rel_res) {
  fewha_status s = ready(c);
  if (s != FEWHA_OK) return s;
  return run_solve(*c->plan, c->stream, {nullptr}, {slopes}, {g_layers}, {x}, max_iters, rtol, iters_done, rel_res,
                   c->err);
}

fewha_status fewha_apply_Winv(fewha_ctx* c, const float* coef, float* layers) {
  fewha_status s = ready(c);
  if (s != FEWHA_OK) return s;
  return run_winv(*c->plan, c->stream, {coef}, {layers}, c->err);
}

fewha_status fewha_apply_WinvT(fewha_ctx* c, const float* layers, float* coef) {
  fewha_status s = ready(c);
  if (s != FEWHA_OK) return s;
  return run_winvT(*c->plan, c->stream, {layers}, {coef}, c->err);
}

fewha_status fewha_param_grads(fewha_ctx* c, const float* slopes, const float* coef, const float* lam,
                               double* grads) {
  fewha_status s = ready(c);
  if (s != FEWHA_OK) return s;
  return run_param_grads(*c->plan, c->stream, {slopes}, {coef}, {lam}, {grads}, c->err);
}

// ---- batches ----

static fewha_status bfail(fewha_batch* b, fewha_status s, const std::string& m) {
  b->err = m;
  return s;
}

// Breakdown flags of the batch plan and of its stream parts.
static fewha_status bready(fewha_batch* b) {
  fewha_status s = take_numeric(*b->plan, b->err);
  for (Plan* q : b->parts)
    if (s == FEWHA_OK) s = take_numeric(*q, b->err);
  return s;
}

fewha_status fewha_batch_create(fewha_batch** out, fewha_ctx* const* ctxs, int n) {
  return fewha_batch_create_tuned(out, ctxs, n, nullptr);
}

fewha_status fewha_batch_create_tuned(fewha_batch** out, fewha_ctx* const* ctxs, int n, const fewha_tuning* t) {
  if (!out || !ctxs || n < 1) return FEWHA_EINVAL;
  if (t && (t->dwt_resident < 0 || t->pt_rows < 0 || t->streams < 0 || t->streams > 4 || t->streams > n ||
            (t->res_split != 0 && t->res_split != 1 && t->res_split != 4) || (t->pt_split != 0 && t->pt_split != 1) ||
            (t->pt_split && t->pt_rows == 8) || (t->glob_fuse != 0 && t->glob_fuse != 1) || t->reserved[0] ||
            t->reserved[1]))
    return FEWHA_EINVAL;
  *out = nullptr;
  int dev = -1;
  std::vector<const HostModel*> ms;
  for (int k = 0; k < n; ++k) {
    if (!ctxs[k] || !ctxs[k]->finalized || ctxs[k]->device < 0) return FEWHA_ESTATE;
    if (dev >= 0 && ctxs[k]->device != dev) return FEWHA_EINVAL;
    dev = ctxs[k]->device;
    ms.push_back(&ctxs[k]->m);
  }
  fewha_batch* b = new (std::nothrow) fewha_batch();
  if (!b) return FEWHA_ENOMEM;
  b->ctxs.assign(ctxs, ctxs + n);
  const int res = (t && t->dwt_resident > 0) ? t->dwt_resident : kResMax;
  const int rows = (t && t->pt_rows > 0) ? t->pt_rows : 4;
  const int split = t ? t->res_split : 0;
  const int pt_split = t ? t->pt_split : 0;
  const int glob_fuse = t ? t->glob_fuse : 0;
  fewha_status s = build_plan(b->plan, ms, dev, res, rows, split, pt_split, glob_fuse, b->err);
  if (s != FEWHA_OK) {
    delete b;
    return s;
  }
  const int parts = (t && t->streams > 1) ? t->streams : 1;
  if (parts > 1) {
    auto undo = [&](fewha_status st) {
      destroy_batch_parts(b);
      destroy_plan(b->plan);
      delete b;
      return st;
    };
    b->parts.assign(parts, nullptr);
    b->part_stream.assign(parts, nullptr);
    b->part_done.assign(parts, nullptr);
    if (hipSetDevice(dev) != hipSuccess || hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
      return undo(FEWHA_EDEVICE);
    for (int q = 0; q < parts; ++q) {
      const int k0 = (int)((long)n * q / parts), k1 = (int)((long)n * (q + 1) / parts);
      b->part_first.push_back(k0);
      std::vector<const HostModel*> mq(ms.begin() + k0, ms.begin() + k1);
      if ((s = build_plan(b->parts[q], mq, dev, res, rows, split, pt_split, glob_fuse, b->err)) != FEWHA_OK)
        return undo(s);
      if (hipStreamCreateWithFlags(&b->part_stream[q], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&b->part_done[q], hipEventDisableTiming) != hipSuccess)
        return undo(FEWHA_EDEVICE);
    }
  }
  *out = b;
  return FEWHA_OK;
}

fewha_status fewha_batch_set_stream(fewha_batch* b, void* s) {
  if (!b) return FEWHA_EINVAL;
  b->stream = (hipStream_t)s;
  return FEWHA_OK;
}

// One frame of every problem of plan P on stream st: the I/O table, then the
// captured graph of `iters` iterations (captured on first use) or the plain
// launches.
static fewha_status run_frame(Plan& P, hipStream_t st, const std::vector<IoDev>& io, int iters, int use_graph,
                              bool refresh, std::string& err) {
  fewha_status s = upload_io(P, io, st, P.dIO, err);
  if (s != FEWHA_OK) return s;
  if (refresh && (s = upload_refresh_io(P, io, st, err)) != FEWHA_OK) return s;
  P.last_io = io;
  P.ran = true;
  if (!use_graph) {
    enq_reconstruct(P, args(P, st, P.dIO), iters, refresh);
    return FEWHA_OK;
  }
  const int key = 2 * iters + (refresh ? 1 : 0);  // one graph per iteration count and restart kind
  auto it = P.graphs.find(key);
  if (it == P.graphs.end()) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    HIP_TRY(hipStreamBeginCapture(P.cap_stream, hipStreamCaptureModeThreadLocal));
    enq_reconstruct(P, args(P, P.cap_stream, P.dIO), iters, refresh);
    HIP_TRY(hipStreamEndCapture(P.cap_stream, &g));
    HIP_TRY(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    P.graph_defs[key] = g;
    it = P.graphs.emplace(key, ge).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, st));
  return FEWHA_OK;
}

fewha_status fewha_batch_reconstruct(fewha_batch* b, const float* const* slopes, float* const* state,
                                     float* const* layers_out, float* const* dm_out, int iters, int use_graph) {
  if (!b) return FEWHA_EINVAL;
  if (fewha_status s0 = bready(b); s0 != FEWHA_OK) return s0;
  if (!slopes || !state) return bfail(b, FEWHA_EINVAL, "batch_reconstruct: null slopes or state array");
  if (iters < 0 || iters > kMaxIters) return bfail(b, FEWHA_EINVAL, "batch_reconstruct: iters must lie in [0, 256]");
  Plan& P = *b->plan;
  std::string& err = b->err;
  std::vector<IoDev> io(P.nprob);
  for (int k = 0; k < P.nprob; ++k) {
    if (!slopes[k] || !state[k]) return bfail(b, FEWHA_EINVAL, "batch_reconstruct: null pointer for problem " + std::to_string(k));
    if (((uintptr_t)state[k] & 15) != 0)
      return bfail(b, FEWHA_EINVAL, "batch_reconstruct: state must be 16-byte aligned (problem " + std::to_string(k) + ")");
    io[k].in = slopes[k];
    io[k].state = state[k];
    io[k].layers_out = layers_out ? layers_out[k] : nullptr;
    io[k].dm_out = dm_out ? dm_out[k] : nullptr;
  }
  HIP_TRY(hipSetDevice(P.device));
  fewha_status s;
  const bool refresh = refresh_due(b->frames, b->refresh_every);
  if (b->parts.empty()) {
    if ((s = run_frame(P, b->stream, io, iters, use_graph, refresh, err)) != FEWHA_OK) return s;
  } else {
    // fork: every part waits for the work queued before this call
    HIP_TRY(hipEventRecord(b->fork, b->stream));
    for (size_t q = 0; q < b->parts.size(); ++q) {
      Plan& Q = *b->parts[q];
      const std::vector<IoDev> ioq(io.begin() + b->part_first[q], io.begin() + b->part_first[q] + Q.nprob);
      HIP_TRY(hipStreamWaitEvent(b->part_stream[q], b->fork, 0));
      if ((s = run_frame(Q, b->part_stream[q], ioq, iters, use_graph, refresh, err)) != FEWHA_OK) return s;
      HIP_TRY(hipEventRecord(b->part_done[q], b->part_stream[q]));
    }
    // join: work queued after this call waits for every part
    for (size_t q = 0; q < b->parts.size(); ++q) HIP_TRY(hipStreamWaitEvent(b->stream, b->part_done[q], 0));
    P.last_io = io;  // stage timing runs the whole batch's plan on these buffers
    P.ran = true;
  }
  ++b->frames;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bfail(b, FEWHA_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return FEWHA_OK;
}

fewha_status fewha_batch_set_refresh(fewha_batch* b, int every) {
  if (!b || every < 0) return FEWHA_EINVAL;
  b->refresh_every = every;
  return FEWHA_OK;
}

fewha_status fewha_batch_set_solve_coarse(fewha_batch* b, int side) {
  if (!b || !b->plan) return FEWHA_EINVAL;
  if (!coarse_side_ok(side)) {
    b->err = "batch_set_solve_coarse: side must be 0 or a power of two up to 64";
    return FEWHA_EINVAL;
  }
  if (b->plan->coarse_side != side) {
    b->plan->coarse_side = side;
    b->plan->coarse_ready = false;
  }
  return FEWHA_OK;
}

fewha_status fewha_batch_set_frame_count(fewha_batch* b, long frames) {
  if (!b || frames < 0) return FEWHA_EINVAL;
  b->frames = frames;
  return FEWHA_OK;
}

fewha_status fewha_batch_solve(fewha_batch* b, const float* const* rhs, float* const* x, int max_iters, double rtol,
                               int* iters_done, double* rel_res) {
  if (!b) return FEWHA_EINVAL;
  if (fewha_status s0 = bready(b); s0 != FEWHA_OK) return s0;
  if (!rhs || !x) return bfail(b, FEWHA_EINVAL, "batch_solve: null pointer array");
  const int n = b->plan->nprob;
  std::vector<const float*> vr(rhs, rhs + n), none(n, nullptr);
  std::vector<float*> vx(x, x + n);
  for (int k = 0; k < n; ++k)
    if (!vr[k]) return bfail(b, FEWHA_EINVAL, "batch_solve: null rhs");
  return run_solve(*b->plan, b->stream, vr, none, none, vx, max_iters, rtol, iters_done, rel_res, b->err);
}

fewha_status fewha_batch_solve_map(fewha_batch* b, const float* const* slopes, const float* const* g_layers,
                                   float* const* x, int max_iters, double rtol, int* iters_done, double* rel_res) {
  if (!b) return FEWHA_EINVAL;
  if (fewha_status s0 = bready(b); s0 != FEWHA_OK) return s0;
  if (!x) return bfail(b, FEWHA_EINVAL, "batch_solve_map: null x array");
  const int n = b->plan->nprob;
  std::vector<const float*> vs(n, nullptr), vg(n, nullptr), none(n, nullptr);
  if (slopes) vs.assign(slopes, slopes + n);
  if (g_layers) vg.assign(g_layers, g_layers + n);
  std::vector<float*> vx(x, x + n);
  return run_solve(*b->plan, b->stream, none, vs, vg, vx, max_iters, rtol, iters_done, rel_res, b->err);
}

fewha_status fewha_batch_apply_Winv(fewha_batch* b, const float* const* coef, float* const* layers) {
  if (!b) return FEWHA_EINVAL;
  if (fewha_status s0 = bready(b); s0 != FEWHA_OK) return s0;
  if (!coef || !layers) return bfail(b, FEWHA_EINVAL, "batch_apply_Winv: null pointer array");
  const int n = b->plan->nprob;
  std::vector<const float*> vi(coef, coef + n);
  std::vector<float*> vo(layers, layers + n);
  return run_winv(*b->plan, b->stream, vi, vo, b->err);
}

fewha_status fewha_batch_apply_WinvT(fewha_batch* b, const float* const* layers, float* const* coef) {
  if (!b) return FEWHA_EINVAL;
  if (fewha_status s0 = bready(b); s0 != FEWHA_OK) return s0;
  if (!coef || !layers) return bfail(b, FEWHA_EINVAL, "batch_apply_WinvT: null pointer array");
  const int n = b->plan->nprob;
  std::vector<const float*> vi(layers, layers + n);
  std::vector<float*> vo(coef, coef + n);
  return run_winvT(*b->plan, b->stream, vi, vo, b->err);
}

fewha_status fewha_batch_param_grads(fewha_batch* b, const float* const* slopes, const float* const* coef,
                                     const float* const* lam, double* const* grads) {
  if (!b) return FEWHA_EINVAL;
  if (fewha_status s0 = bready(b); s0 != FEWHA_OK) return s0;
  if (!slopes || !coef || !lam || !grads) return bfail(b, FEWHA_EINVAL, "batch_param_grads: null pointer array");
  const int n = b->plan->nprob;
  std::vector<const float*> vs(slopes, slopes + n), vc(coef, coef + n), vl(lam, lam + n);
  std::vector<double*> vg(grads, grads + n);
  return run_param_grads(*b->plan, b->stream, vs, vc, vl, vg, b->err);
}

fewha_status fewha_batch_time_stage(fewha_batch* b, int stage, int reps, double* avg_us, long* workgroups) {
  if (!b || !avg_us) return FEWHA_EINVAL;
  if (stage < 0 || stage >= FEWHA_STAGE_COUNT || reps < 1) return bfail(b, FEWHA_EINVAL, "time_stage: bad stage or reps");
  Plan& P = *b->plan;
  if (!P.ran) return bfail(b, FEWHA_ESTATE, "time_stage: run batch_reconstruct first");
  std::string& err = b->err;
  HIP_TRY(hipSetDevice(P.device));
  // private copies of the states so that timing never changes caller data
  if (P.prof_state.empty()) {
    P.prof_state.assign(P.nprob, nullptr);
    for (int k = 0; k < P.nprob; ++k) HIP_TRY(hipMalloc(&P.prof_state[k], sizeof(float) * P.n_state[k]));
  }
  std::vector<IoDev> io = P.last_io;
  for (int k = 0; k < P.nprob; ++k) {
    HIP_TRY(hipMemcpyAsync(P.prof_state[k], io[k].state, sizeof(float) * P.n_state[k], hipMemcpyDeviceToDevice,
                           b->stream));
    io[k].state = P.prof_state[k];
    io[k].layers_out = nullptr;
    io[k].dm_out = nullptr;
  }
  fewha_status s = upload_io(P, io, b->stream, P.dIOprof, err);
  if (s != FEWHA_OK) return s;
  LaunchArgs a = args(P, b->stream, P.dIOprof);
  const int it = 1;  // an inner iteration: fused p update with beta
  long wg = 0;
  auto run = [&]() {
    switch (stage) {
      case FEWHA_STAGE_IDWT_RES:
        if (P.idwt_split) {
          launch_idwt_res4(a, T(P, P.idwt_res4), P.idwt_res4.n, SRC_PUPD, OUT_PHI, it);
          wg = P.idwt_res4.n;
        } else {
          launch_idwt_res(a, T(P, P.idwt_res), P.idwt_res.n, SRC_PUPD, OUT_PHI, it);
          wg = P.idwt_res.n;
        }
        break;
      case FEWHA_STAGE_IDWT_GLOB:
        wg = 0;
        for (size_t st = 0; st < P.idwt_glob.size(); ++st) {
          launch_idwt_glob(a, T(P, P.idwt_glob[st]), P.idwt_glob[st].n, SRC_PUPD, OUT_PHI, it, (int)st);
          wg += P.idwt_glob[st].n;
        }
        break;
      case FEWHA_STAGE_P_GAMMA:
        launch_pgamma(a, T(P, P.pg), P.pg.n, PG_DENSE);
        wg = P.pg.n;
        break;
      case FEWHA_STAGE_GAMMA_T:
        launch_gammaT(a, T(P, P.gt), P.gt.n, GT_WEIGHTED);
        wg = P.gt.n;
        break;
      case FEWHA_STAGE_P_T:
        launch_pT(a, T(P, P.pt), P.pt.n, PT_PHIADJ);
        wg = P.pt.n;
        break;
      case FEWHA_STAGE_FDWT_GLOB:
        wg = 0;
        for (size_t st = 0; st < P.fdwt_glob.size(); ++st) {
          launch_fdwt_glob(a, T(P, P.fdwt_glob[st]), P.fdwt_glob[st].n, EPI_PCG, it, (int)st);
          wg += P.fdwt_glob[st].n;
        }
        break;
      case FEWHA_STAGE_FDWT_RES:
        launch_fdwt_res(a, T(P, P.fdwt_res), P.fdwt_res.n, EPI_PCG, it);
        wg = P.fdwt_res.n;
        break;
      case FEWHA_STAGE_UPDATE:
        launch_update(a, T(P, P.upd), P.upd.n, it);
        wg = P.upd.n;
        break;
    }
  };
  run();  // warm
  HIP_TRY(hipEventRecord(P.t0, b->stream));
  for (int r = 0; r < reps; ++r) run();
  HIP_TRY(hipEventRecord(P.t1, b->stream));
  HIP_TRY(hipEventSynchronize(P.t1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, P.t0, P.t1));
  *avg_us = 1000.0 * ms / reps;
  if (workgroups) *workgroups = wg;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bfail(b, FEWHA_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return FEWHA_OK;
}

void fewha_batch_destroy(fewha_batch* b) {
  if (!b) return;
  destroy_batch_parts(b);
  destroy_plan(b->plan);
  delete b;
}

const char* fewha_last_error(const fewha_ctx* c) { return c ? c->err.c_str() : "null context"; }
const char* fewha_batch_last_error(const fewha_batch* b) { return b ? b->err.c_str() : "null batch"; }

void fewha_destroy(fewha_ctx* c) {
  if (!c) return;
  destroy_plan(c->plan);
  delete c;
}

}  // extern "C"
