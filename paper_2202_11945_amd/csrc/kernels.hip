// gfx950 kernels of the FEWHA hot path.  Every kernel walks a work list of
// tiles spanning all problems of a plan, so one launch serves one stage of a
// whole batch.  Bulk arithmetic is FP32; PCG inner products are accumulated
// in FP64 per workgroup and summed across workgroups in a fixed order
// (deterministic: no atomics anywhere).
//
// Memory-level parallelism: the transform and vector kernels gather the
// loads of several elements before their dependent stores (fetch / finish
// pairs), so a thread keeps several global loads in flight.
#include "kernels.h"

namespace fewha {

// ---------------------------------------------------------------- helpers

// Global-address-space view of a device pointer held in a struct (loads
// through it compile to global, not flat, memory instructions).
typedef const float __attribute__((address_space(1)))* gptr_f;
// 16-byte global loads and stores (clang vector type; HIP's float4 has no
// assignment from a global-space reference).
typedef float v4f __attribute__((ext_vector_type(4)));
typedef const v4f __attribute__((address_space(1)))* gptr_f4;
typedef v4f __attribute__((address_space(1)))* gptr_w4;
// Stores and FP64 accesses likewise.  A flat access also counts against the
// LDS / scalar-load wait counter, so a later LDS wait or barrier would wait
// for it to reach memory.
typedef float __attribute__((address_space(1)))* gptr_w;
typedef const double __attribute__((address_space(1)))* gptr_d;
typedef double __attribute__((address_space(1)))* gptr_wd;

// Wave sums by DPP moves inside the vector ALU (no LDS crossbar round
// trips): pair and quad swaps, the half-row and row mirrors give every lane
// its 16-lane row sum; row_bcast:15 and row_bcast:31 then carry rows 0-2
// into row 3, and lane 63's total is returned to every lane.  Every lane of
// the wave must be active (the moves read the source lanes whatever the
// exec mask).  Fixed order: ((R3 + R2) + (R1 + R0)) of the row sums.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140, kDppBcast15 = 0x142,
              kDppBcast31 = 0x143;
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<kDppXor1, 0xF>(v);
  v += dpp_f<kDppXor2, 0xF>(v);
  v += dpp_f<kDppHalfMirror, 0xF>(v);
  v += dpp_f<kDppMirror, 0xF>(v);
  v += dpp_f<kDppBcast15, 0xA>(v);
  v += dpp_f<kDppBcast31, 0xC>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<kDppXor1, 0xF>(v);
  v += dpp_d<kDppXor2, 0xF>(v);
  v += dpp_d<kDppHalfMirror, 0xF>(v);
  v += dpp_d<kDppMirror, 0xF>(v);
  v += dpp_d<kDppBcast15, 0xA>(v);
  v += dpp_d<kDppBcast31, 0xC>(v);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Block sum; result valid in thread 0.  `sh` holds one slot per wave.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh, int nthreads) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (nthreads >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;
}

// Sums of slot groups by one wave in a fixed order: lane l adds slots l,
// l + 64, l + 128, ... in turn, then a fixed shuffle tree; the result,
// identical in every workgroup that sums the same slots, is in every lane.
// Two phases, so that a kernel can put the slot loads in flight before its
// own loads and reduce them while those are in flight: slots_issue requests
// the first H slots of every lane of every group (up to 64 H per group)
// together; slots_reduce adds them (and, for longer groups, the rest in a
// loop).
template <int G, int H>
struct SlotLoads {
  double v[G][H];
};
template <int G, int H>
__device__ __forceinline__ void slots_issue(const double* const (&s)[G], const int (&n)[G], SlotLoads<G, H>& L) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int g = 0; g < G; ++g) {
#pragma unroll
    for (int u = 0; u < H; ++u) L.v[g][u] = 0.0;
    if (n[g] > 0) {  // wave-uniform; a group of no slots may have no storage
#pragma unroll
      for (int u = 0; u < H; ++u) L.v[g][u] = ((gptr_d)s[g])[min(lane + 64 * u, n[g] - 1)];
    }
  }
}
template <int G, int H>
__device__ __forceinline__ void slots_reduce(const double* const (&s)[G], const int (&n)[G], const SlotLoads<G, H>& L,
                                             double (&out)[G]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < H; ++u) {
      // an opaque copy: without it the compiler folds the first addition
      // into slots_issue's branch, right behind its load, and waits there
      // for the slot before the kernel's own loads are requested
      double x = L.v[g][u];
      asm volatile("" : "+v"(x));
      if (lane + 64 * u < n[g]) a += x;
    }
    for (int i = lane + 64 * H; i < n[g]; i += 64) a += ((gptr_d)s[g])[i];
    out[g] = wave_sum(a);
  }
}
template <int G, int H = 4>
__device__ __forceinline__ void wave_sum_slots_n(const double* const (&s)[G], const int (&n)[G], double (&out)[G]) {
  SlotLoads<G, H> L;
  slots_issue<G, H>(s, n, L);
  slots_reduce<G, H>(s, n, L, out);
}
__device__ __forceinline__ double wave_sum_slots(const double* s, int n) {
  const double* const ss[1] = {s};
  const int nn[1] = {n};
  double o[1];
  wave_sum_slots_n<1>(ss, nn, o);
  return o[0];
}

// XCD-aware work distribution.  Workgroups are dispatched round-robin over
// the 8 XCDs (workgroup b runs on XCD b mod 8) and every XCD has its own L2.
// Tile lists are ordered by problem, item and tile, so giving each XCD a
// contiguous run of tiles keeps the data that neighbouring tiles share (a
// problem's layers, corner grids, halos) in one L2 instead of eight.  A
// bijection of [0, W): XCD x takes tiles [start_x, start_x + count_x).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int b, int W) {
  const int x = b % kXcds, i = b / kXcds;
  const int q = W / kXcds, r = W % kXcds;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}
__device__ __forceinline__ const Tile& my_tile(const Tile* tiles) {
  return tiles[xcd_tile((int)blockIdx.x, (int)gridDim.x)];
}

__device__ __forceinline__ const double* dot_group(const ProbDev& pr, int g) {
  return pr.dots + (long)g * pr.n_dots;
}
__device__ __forceinline__ int rho_count(const ProbDev& pr, int k) {
  return k == 0 ? pr.n_slots_fdwt : pr.n_slots_upd;
}
// Dot groups of iteration k in a ring of kDotRing iterations: rho_k = r_k^T J^{-1} r_k
// and pi_k = p_k^T M p_k (each step reads only the current and previous iteration).
__device__ __forceinline__ int rho_grp(int k) { return 2 * (k & (kDotRing - 1)); }
__device__ __forceinline__ int pi_grp(int k) { return 2 * (k & (kDotRing - 1)) + 1; }

// Search direction p_j and its image M p_j of iteration j: the augmented
// PCG keeps its first aug_keep of each (the next frame's W and A W); later
// ones, and those of the plain PCG, alternate between two buffers.
__device__ __forceinline__ float* p_loc(const ProbDev& pr, int j) {
  return pr.aug_keep > j ? pr.aug_pdir + (long)j * pr.n_c : ((j & 1) ? pr.pbuf1 : pr.pbuf0);
}
__device__ __forceinline__ float* q_loc(const ProbDev& pr, int j) {
  return pr.aug_keep > j ? pr.aug_qdir + (long)j * pr.n_c : pr.q;
}
// rho_k = r_k^T J^{-1} r_k, summed by a wave in a fixed order; a problem with
// augmentation forms rho_0 of its projected residual in slots of its own.
__device__ __forceinline__ const double* rho_slots(const ProbDev& pr, int k, int& n) {
  if (k == 0 && pr.aug_keep > 0) {
    n = pr.n_slots_upd;
    return pr.aug_slots + (long)kAugRho0 * pr.n_slots_upd;
  }
  n = rho_count(pr, k);
  return dot_group(pr, rho_grp(k));
}
// rho_k and rho_{k-1} with their loads in flight together
__device__ __forceinline__ void rho_sum2(const ProbDev& pr, int k, double& rk, double& rkm) {
  int n0, n1;
  const double* const s[2] = {rho_slots(pr, k, n0), rho_slots(pr, k - 1, n1)};
  const int n[2] = {n0, n1};
  double o[2];
  wave_sum_slots_n<2>(s, n, o);
  rk = o[0];
  rkm = o[1];
}

// Search-direction source of the inverse transform (fused p update).
struct PSrc {
  const float* __restrict__ src;  // plain source (SRC_IN / SRC_STATE_C)
  const float* __restrict__ r;
  const float* __restrict__ jinv;
  const float* __restrict__ pold;
  float* __restrict__ pnew;
  float beta;
  int mode;
};

__device__ __forceinline__ PSrc make_psrc(const ProbDev& pr, const IoDev& io, int mode, int iter, float beta) {
  PSrc s;
  if (pr.aug_keep > 0 && (mode == SRC_PUPD0 || mode == SRC_PUPD)) mode = SRC_PJ;  // p_j formed by k_aug_p
  s.mode = mode;
  s.src = (mode == SRC_IN) ? io.in : (mode == SRC_PJ) ? p_loc(pr, iter) : io.state;  // state starts with c
  s.r = io.state + 2L * pr.n_c;
  s.jinv = pr.jinv;
  s.pnew = p_loc(pr, iter);
  s.pold = p_loc(pr, iter - 1);
  s.beta = beta;
  return s;
}

struct CoefLoad {
  float a, b, c;
};
__device__ __forceinline__ CoefLoad coef_fetch(const PSrc& s, int e) {
  CoefLoad v{0.f, 0.f, 0.f};
  if (s.mode == SRC_IN || s.mode == SRC_STATE_C || s.mode == SRC_PJ) {
    v.a = ((gptr_f)s.src)[e];
  } else {
    v.a = ((gptr_f)s.r)[e];
    v.b = ((gptr_f)s.jinv)[e];
    if (s.mode == SRC_PUPD) v.c = ((gptr_f)s.pold)[e];
  }
  return v;
}
// p = J^{-1} r (first iteration) or p = J^{-1} r + beta p_old; written once by its owner
__device__ __forceinline__ float coef_finish(const PSrc& s, int e, const CoefLoad& v, bool owner) {
  if (s.mode == SRC_IN || s.mode == SRC_STATE_C || s.mode == SRC_PJ) return v.a;
  const float z = v.a * v.b;
  const float p = (s.mode == SRC_PUPD0) ? z : fmaf(s.beta, v.c, z);
  if (owner) ((gptr_w)s.pnew)[e] = p;
  return p;
}

// Coefficient loads without branches: every path issues the same loads in
// the same order, so the compiler's wait for the loads a kernel needs first
// leaves the later ones in flight (with a load under a condition, or a mode
// branch around it, it waits for all of them).  In a plain source mode all
// three pointers are the source; without p_old the third is r again (the
// repeated loads hit the same cache lines).
struct CoefPtrs {
  gptr_f a, b, c;
};
__device__ __forceinline__ CoefPtrs coef_ptrs(const PSrc& s) {
  const bool plain = s.mode == SRC_IN || s.mode == SRC_STATE_C || s.mode == SRC_PJ;
  const gptr_f a = (gptr_f)(plain ? s.src : s.r);
  return CoefPtrs{a, plain ? a : (gptr_f)s.jinv, s.mode == SRC_PUPD ? (gptr_f)s.pold : a};
}
__device__ __forceinline__ CoefLoad coef_load(const CoefPtrs& p, int e) { return CoefLoad{p.a[e], p.b[e], p.c[e]}; }

// beta_k = rho_k / rho_{k-1} in two phases (see slots_issue): beta_issue
// before a kernel's coefficient loads, beta_reduce once they are in flight;
// every wave sums the slots itself in the same fixed order (no barrier, the
// same value in every wave).
template <int H>
struct BetaLoads {
  const double* s[2];
  int n[2];
  SlotLoads<2, H> L;
};
template <int H>
__device__ __forceinline__ void beta_issue(const ProbDev& pr, int mode, int iter, BetaLoads<H>& b) {
  if (mode != SRC_PUPD) return;
  b.s[0] = rho_slots(pr, iter, b.n[0]);
  b.s[1] = rho_slots(pr, iter - 1, b.n[1]);
  slots_issue<2, H>(b.s, b.n, b.L);
}
template <int H>
__device__ __forceinline__ float beta_reduce(int mode, const BetaLoads<H>& b) {
  if (mode != SRC_PUPD) return 0.f;
  double o[2];
  slots_reduce<2, H>(b.s, b.n, b.L, o);
  return (float)((o[1] != 0.0) ? o[0] / o[1] : 0.0);
}

// Final output of the inverse transform: phi = delta^{-1} W^T c, optionally
// with the open-loop control update of Algorithm 1 (F = I).
struct OutLoad {
  float a, ap;
};
// The output's destinations and constants, read from the problem once per
// kernel (a store through them could alias the problem record).
struct OutDst {
  gptr_w phi;
  gptr_w out;
  gptr_w layers_out;
  gptr_w aprev;  // F = I control update: previous and new commands in the state
  gptr_w a;
  gptr_w dm_out;
  float gain;
  int mode;  // out_mode, with OUT_FIT split by pr.fitted
};
enum { OUTD_PHI, OUTD_USER, OUTD_FITTED, OUTD_CONTROL, OUTD_CLOSED };
__device__ __forceinline__ OutDst out_dst(const ProbDev& pr, const IoDev& io, int out_mode) {
  OutDst d;
  d.phi = (gptr_w)pr.phi;
  d.out = (gptr_w)io.out;
  d.layers_out = (gptr_w)io.layers_out;
  d.aprev = (gptr_w)(io.state + 3L * pr.n_c);
  d.a = d.aprev + pr.n_act;
  d.dm_out = (gptr_w)io.dm_out;
  d.gain = pr.gain;
  d.mode = out_mode == OUT_PHI    ? OUTD_PHI
           : out_mode == OUT_USER ? OUTD_USER
           : pr.fitted            ? OUTD_FITTED
           : pr.closed            ? OUTD_CLOSED
                                  : OUTD_CONTROL;
  return d;
}
__device__ __forceinline__ OutLoad out_fetch(const OutDst& d, int e) {
  OutLoad o{0.f, 0.f};
  if (d.mode == OUTD_CONTROL || d.mode == OUTD_CLOSED) o.a = ((gptr_f)d.a)[e];
  if (d.mode == OUTD_CLOSED) o.ap = ((gptr_f)d.aprev)[e];
  return o;
}
__device__ __forceinline__ void out_finish(const OutDst& d, int e, float v, const OutLoad& o) {
  if (d.mode == OUTD_PHI) {
    d.phi[e] = v;
  } else if (d.mode == OUTD_USER) {
    d.out[e] = v;
  } else if (d.mode == OUTD_FITTED) {  // OUT_FIT, DM commands from the fitting step that follows
    d.phi[e] = v;
    if (d.layers_out) d.layers_out[e] = v;
  } else {  // OUT_FIT, F = I: open-loop or closed-loop control of Algorithm 1
    if (d.layers_out) d.layers_out[e] = v;
    const float nw = d.mode == OUTD_CLOSED ? o.a + d.gain * (v - o.ap) : (1.0f - d.gain) * o.a + d.gain * v;
    d.aprev[e] = o.a;
    d.a[e] = nw;
    if (d.dm_out) d.dm_out[e] = nw;
  }
}

// Forward-transform epilogue at layer position e (level index j):
// v = delta^{-1} (W x)_e, then
//   EPI_APPLYM: out = v + alpha D x            (M x)
//   EPI_PCG   : q = v + alpha D p, += p q      (M p and pi)
//   EPI_RHS   : b' = v, r0 = (b' - b) + r      (warm restart), += r0 J^{-1} r0
//   EPI_RHSQ  : b' = v, r0 = b' - q            (restart from the true residual, q = M c), += r0 J^{-1} r0
//   EPI_PLAIN : out = v                        (right-hand side only)
struct EpiLoad {
  float x0, x1, x2;
};
__device__ __forceinline__ EpiLoad epi_fetch(const ProbDev& pr, const IoDev& io, int epi, int iter, int e) {
  EpiLoad l{0.f, 0.f, 0.f};
  if (epi == EPI_APPLYM) {
    l.x0 = ((gptr_f)io.in)[e];
  } else if (epi == EPI_PCG) {
    l.x0 = ((gptr_f)p_loc(pr, iter))[e];
  } else if (epi == EPI_RHS) {
    l.x0 = ((gptr_f)io.state)[pr.n_c + e];
    l.x1 = ((gptr_f)io.state)[2L * pr.n_c + e];
    l.x2 = ((gptr_f)pr.jinv)[e];
  } else if (epi == EPI_RHSQ) {
    l.x0 = ((gptr_f)pr.q)[e];
    l.x2 = ((gptr_f)pr.jinv)[e];
  }
  return l;
}
// The epilogue's destinations, read from the problem once per kernel (a
// store through them could alias the problem record, so reading them at
// every output would reload them after every store); ad = alpha D of the
// output's level, likewise passed in.
struct EpiDst {
  gptr_w q;    // EPI_PCG
  gptr_w out;  // EPI_APPLYM, EPI_PLAIN
  gptr_w b;    // EPI_RHS: b' and r0 in the state
  gptr_w r;
};
__device__ __forceinline__ EpiDst epi_dst(const ProbDev& pr, const IoDev& io, int iter) {
  return EpiDst{(gptr_w)q_loc(pr, iter), (gptr_w)io.out, (gptr_w)(io.state + pr.n_c),
                (gptr_w)(io.state + 2L * pr.n_c)};
}
__device__ __forceinline__ void epi_finish(const EpiDst& dst, int epi, int e, float ad, float v, const EpiLoad& l,
                                           double& acc) {
  if (epi == EPI_APPLYM) {
    dst.out[e] = v + ad * l.x0;
  } else if (epi == EPI_PCG) {
    const float qe = v + ad * l.x0;
    dst.q[e] = qe;
    acc += (double)l.x0 * (double)qe;
  } else if (epi == EPI_RHS || epi == EPI_RHSQ) {
    const float r0 = epi == EPI_RHS ? (v - l.x0) + l.x1 : v - l.x0;
    dst.b[e] = v;
    dst.r[e] = r0;
    acc += (double)r0 * (double)r0 * (double)l.x2;
  } else {
    dst.out[e] = v;
  }
}

__device__ __forceinline__ int dot_group_of(int epi, int iter) { return epi == EPI_PCG ? pi_grp(iter) : 0; }

constexpr int kU = 4;  // elements per thread with loads in flight together
constexpr int kUG = 6; // ... for the 36 x 36 windows of the global transform levels (one round at 256 threads)

// ------------------------------------------------ inverse DWT, resident part
// One line of a synthesis pass: outputs 2 K0 .. 2 (K0 + NP) - 1 of a line
// whose coarse half sits at src[k S] (k < half) and detail half at
// src[(half + k) S], written to dst[0 ..]; periodic:
//   x_t = sum_{i = t mod 2} h_i a[(t-i)/2] + g_i d[(t-i)/2]   (indices mod half)
// Consecutive output pairs share four of their six taps, so the NP + 2 taps
// of each half are read once into registers.  Only the taps K0 - 2 and
// K0 - 1 can wrap (K0 + NP <= half; with half = 1 or 2 they wrap more than
// once, hence the mask); the others are read at fixed offsets from the line
// position (the stride S is a compile-time constant).
template <int NP, int S>
__device__ __forceinline__ void syn_line(const float* src, int half, int K0, const Filter& F, float* dst) {
  float a[NP + 2], d[NP + 2];
  const int i0 = (K0 - 2) & (half - 1), i1 = (K0 - 1) & (half - 1);
  a[0] = src[i0 * S];
  d[0] = src[(half + i0) * S];
  a[1] = src[i1 * S];
  d[1] = src[(half + i1) * S];
  const float* b = src + K0 * S;
  const float* bd = b + half * S;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    a[i + 2] = b[i * S];
    d[i + 2] = bd[i * S];
  }
#pragma unroll
  for (int p = 0; p < NP; ++p) {  // a[p + 2] = a[k0], a[p + 1] = a[k0 - 1], a[p] = a[k0 - 2]
    dst[2 * p] = F.h[0] * a[p + 2] + F.h[2] * a[p + 1] + F.h[4] * a[p] + F.g[0] * d[p + 2] + F.g[2] * d[p + 1] +
                 F.g[4] * d[p];
    dst[2 * p + 1] = F.h[1] * a[p + 2] + F.h[3] * a[p + 1] + F.h[5] * a[p] + F.g[1] * d[p + 2] +
                     F.g[3] * d[p + 1] + F.g[5] * d[p];
  }
}

// A synthesis pass over m lines of side m: line l (one per lane position)
// reads src + l (stride S along the line) and writes dst + l S.  Each thread
// takes np consecutive output pairs of one line (np = m^2 / 2 / threads,
// at least 1), so neighbouring lanes touch neighbouring LDS words.
template <int S>
__device__ __forceinline__ void syn_pass(const float* src, float* dst, int m, const Filter& F) {
  const int half = m >> 1, nt = blockDim.x;
  const int np = max(1, m * half / nt), nch = half / np, lm = __builtin_ctz(m);
  for (int task = threadIdx.x; task < m * nch; task += nt) {
    const int l = task & (m - 1), K0 = (task >> lm) * np;
    for (int p0 = 0; p0 < np; p0 += 8) {
      const int k = K0 + p0, c = min(np - p0, 8);
      float* o = dst + l * S + 2 * k;
      if (c == 8)
        syn_line<8, S>(src + l, half, k, F, o);
      else if (c == 4)
        syn_line<4, S>(src + l, half, k, F, o);
      else if (c == 2)
        syn_line<2, S>(src + l, half, k, F, o);
      else
        syn_line<1, S>(src + l, half, k, F, o);
    }
  }
}

// The last synthesis pass (rows) written straight to global memory:
// g[l gs + t] = scale x_t for line l, each thread its run of 2 np outputs
// (float4 stores when `vec`: g, gs and the runs 16-byte aligned).
template <int S>
__device__ __forceinline__ void syn_pass_out(const float* src, int m, const Filter& F, float* g, int gs,
                                             float scale, bool vec) {
  const int half = m >> 1, nt = blockDim.x;
  const int np = max(1, m * half / nt), nch = half / np, lm = __builtin_ctz(m);
  typedef v4f __attribute__((address_space(1)))* gw4;
  typedef float __attribute__((address_space(1)))* gw1;
  for (int task = threadIdx.x; task < m * nch; task += nt) {
    const int l = task & (m - 1), K0 = (task >> lm) * np;
    for (int p0 = 0; p0 < np; p0 += 8) {
      const int k = K0 + p0, c = min(np - p0, 8);
      float o[16];
      if (c == 8)
        syn_line<8, S>(src + l, half, k, F, o);
      else if (c == 4)
        syn_line<4, S>(src + l, half, k, F, o);
      else if (c == 2)
        syn_line<2, S>(src + l, half, k, F, o);
      else
        syn_line<1, S>(src + l, half, k, F, o);
      float* dst = g + (long)l * gs + 2 * k;
      if (vec && c >= 2) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (4 * i < 2 * c)
            ((gw4)dst)[i] = v4f{o[4 * i] * scale, o[4 * i + 1] * scale, o[4 * i + 2] * scale, o[4 * i + 3] * scale};
      } else {
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (i < 2 * c) ((gw1)dst)[i] = o[i] * scale;
      }
    }
  }
}

// The same passes for a level side M known at compile time: NP output
// pairs per task (one task per thread at 1024 threads), so a thread's taps
// are read in one straight sequence (with the run length chosen at run time
// the compiler waited for the first LDS reads before issuing the rest).
template <int S, int M>
__device__ __forceinline__ void syn_pass_m(const float* src, float* dst, const Filter& F) {
  constexpr int half = M / 2, np = M * half / 1024 > 1 ? M * half / 1024 : 1, nch = half / np;
  constexpr int lm = __builtin_ctz(M);
  static_assert(np <= 8, "at most 8 output pairs per task");
  for (int task = threadIdx.x; task < M * nch; task += blockDim.x) {
    const int l = task & (M - 1), K0 = (task >> lm) * np;
    syn_line<np, S>(src + l, half, K0, F, dst + l * S + 2 * K0);
  }
}
template <int S, int M>
__device__ __forceinline__ void syn_pass_out_m(const float* src, const Filter& F, float* g, int gs, float scale,
                                               bool vec) {
  constexpr int half = M / 2, np = M * half / 1024 > 1 ? M * half / 1024 : 1, nch = half / np;
  constexpr int lm = __builtin_ctz(M);
  static_assert(np <= 8, "at most 8 output pairs per task");
  typedef v4f __attribute__((address_space(1)))* gw4;
  typedef float __attribute__((address_space(1)))* gw1;
  for (int task = threadIdx.x; task < M * nch; task += blockDim.x) {
    const int l = task & (M - 1), K0 = (task >> lm) * np;
    float o[2 * np];
    syn_line<np, S>(src + l, half, K0, F, o);
    float* dst = g + (long)l * gs + 2 * K0;
    if (np >= 2 && vec) {
#pragma unroll
      for (int i = 0; i < np / 2; ++i)
        ((gw4)dst)[i] = v4f{o[4 * i] * scale, o[4 * i + 1] * scale, o[4 * i + 2] * scale, o[4 * i + 3] * scale};
    } else {
#pragma unroll
      for (int i = 0; i < 2 * np; ++i) ((gw1)dst)[i] = o[i] * scale;
    }
  }
}
// f(std::integral_constant<int, M>) for M = M0, 2 M0, ..., MMAX in turn.
template <int M, int MMAX, class Fn>
__device__ __forceinline__ void for_sides(Fn&& f) {
  f(std::integral_constant<int, M>{});
  if constexpr (M < MMAX) for_sides<2 * M, MMAX>(f);
}

// One workgroup per (problem, layer): all synthesis levels whose output side
// is at most the layer's resident side R (<= RMAX, the LDS capacity of the
// instantiation) run in LDS.  Columns then rows, periodic, Mallat layout.
// The LDS rows have the odd stride S = RMAX + 1 and the column pass writes its
// result transposed (Bt[c][t] = x[t][c]), so both passes walk their lines
// with lanes on consecutive words and strided writes free of bank conflicts.
// Every global load of the block is issued in one round, before the inner
// products of beta are reduced.
template <int RMAX>
__global__ __launch_bounds__(1024) void k_idwt_res(const ProbDev* P, const LayerDev* LD, const IoDev* IO,
                                                   const Tile* tiles, Filter F, int src_mode, int out_mode,
                                                   int iter) {
  __shared__ float A[RMAX * (RMAX + 1)];
  __shared__ float B[RMAX * (RMAX + 1)];
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[t.mask];  // the global layer index, carried by the tile
  const IoDev& io = IO[t.prob];
  PSrc ps = make_psrc(pr, io, src_mode, iter, 0.f);
  const int n = ly.n, R = ly.res, lr = __builtin_ctz(R);
  constexpr int S = RMAX + 1;
  const int m0 = n >> ly.levels;
  const int off = ly.off;
  const int nt = blockDim.x;
  // every resident coefficient (the R x R top-left block of the Mallat layout:
  // the coarse block and the detail quadrants of all resident levels), kUL
  // per thread at 1024 threads per workgroup (the launch shape)
  constexpr int kUL = RMAX * RMAX / 1024 > 0 ? RMAX * RMAX / 1024 : 1;
  BetaLoads<2> bl;
  beta_issue<2>(pr, ps.mode, iter, bl);
  // loads without branches (indices past the block clamped), so that beta's
  // inner products are summed while the block's loads are in flight
  const CoefPtrs cp = coef_ptrs(ps);
  CoefLoad v[kUL];
#pragma unroll
  for (int u = 0; u < kUL; ++u) {
    const int e = min((int)threadIdx.x + u * nt, R * R - 1);
    v[u] = coef_load(cp, off + (e >> lr) * n + (e & (R - 1)));
  }
  ps.beta = beta_reduce<2>(ps.mode, bl);
#pragma unroll
  for (int u = 0; u < kUL; ++u) {
    const int e = threadIdx.x + u * nt;
    if (e < R * R) A[(e >> lr) * S + (e & (R - 1))] = coef_finish(ps, off + (e >> lr) * n + (e & (R - 1)), v[u], true);
  }
  for (int e = threadIdx.x + kUL * nt; e < R * R; e += nt) {  // workgroups under 1024 threads only
    const int g = off + (e >> lr) * n + (e & (R - 1));
    A[(e >> lr) * S + (e & (R - 1))] = coef_finish(ps, g, coef_fetch(ps, g), true);
  }
  __syncthreads();
  // the last rows pass stores the output itself (layers, caller buffer, or
  // the coarse block of the first global level); the control update of a
  // frame's final transform keeps the separate output phase
  const bool plain_out = n != R || out_mode == OUT_PHI || out_mode == OUT_USER;
  const bool direct = plain_out && 2 * m0 <= R;
  float* gout = n != R ? pr.tmpa + ly.tmp_off : ((out_mode == OUT_PHI ? pr.phi : io.out) + off);
  const int gs = n != R ? R : n;
  const bool vec = (((uintptr_t)gout) & 15) == 0;
  const float oscale = n != R ? 1.f : ly.inv_delta;
  for_sides<2, RMAX>([&](auto side) {  // the levels of output side M = 2 m0 .. R
    constexpr int M = decltype(side)::value;
    if (M < 2 * m0 || M > R) return;
    syn_pass_m<S, M>(A, B, F);  // columns (along y): A[t][c] -> B[c][t]
    __syncthreads();
    if (M == R && direct) {
      syn_pass_out_m<S, M>(B, F, gout, gs, oscale, vec);
    } else {
      syn_pass_m<S, M>(B, A, F);  // rows (along x): B[c][r] = row r of the level -> A[r][c]
      __syncthreads();
    }
  });
  if (direct) return;
  if (n == R) {
    const OutDst od = out_dst(pr, io, out_mode);
    for (int e0 = threadIdx.x; e0 < R * R; e0 += kU * nt) {
      OutLoad o[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * nt;
        if (e < R * R) o[u] = out_fetch(od, off + e);  // n == R: row-major e
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * nt;
        if (e < R * R) out_finish(od, off + e, A[(e >> lr) * S + (e & (R - 1))] * ly.inv_delta, o[u]);
      }
    }
  } else {
    const gptr_w dst = (gptr_w)(pr.tmpa + ly.tmp_off);
    for (int e = threadIdx.x; e < R * R; e += nt) dst[e] = A[(e >> lr) * S + (e & (R - 1))];
  }
}

// A run of NP synthesis output pairs from a window that holds its halo (no
// wrap): pair p takes coarse taps a[base + p + 2], a[base + p + 1],
// a[base + p] and the same detail taps (rows of stride S from a_src, d_src);
// outputs 2p and 2p + 1 go to dst[2p ds], dst[(2p + 1) ds].  The same products
// and order as the per-output form.
template <int NP>
__device__ __forceinline__ void syn_run(const float* a_src, const float* d_src, int S, int base, const Filter& F,
                                        float* dst, int ds) {
  float a[NP + 2], d[NP + 2];
#pragma unroll
  for (int i = 0; i < NP + 2; ++i) {
    a[i] = a_src[(base + i) * S];
    d[i] = d_src[(base + i) * S];
  }
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    dst[(2 * p) * ds] = F.h[0] * a[p + 2] + F.h[2] * a[p + 1] + F.h[4] * a[p] + F.g[0] * d[p + 2] +
                        F.g[2] * d[p + 1] + F.g[4] * d[p];
    dst[(2 * p + 1) * ds] = F.h[1] * a[p + 2] + F.h[3] * a[p + 1] + F.h[5] * a[p] + F.g[1] * d[p + 2] +
                            F.g[3] * d[p + 1] + F.g[5] * d[p];
  }
}

// ------------------------------------- inverse DWT, resident part in quarters
// The same levels as k_idwt_res over four workgroups per (problem, layer),
// so that a batch launch fills the chip: every workgroup synthesizes the
// levels below the top one (output side R/2 and less) itself in LDS, then
// the top level (output side R) for one quadrant of the output, R/2 x R/2,
// from a window of the top level's four bands (the lower levels' result and
// the three detail quadrants, 2 coefficients of halo before each direction,
// periodic).  A coefficient of the lower block is owned (its search
// direction stored) by quarter 0, a top-level detail coefficient by the
// quarter whose output it falls under.  Needs R >= 2 (n >> levels): at
// least one resident level.
template <int RMAX>
__global__ __launch_bounds__(512) void k_idwt_res4(const ProbDev* P, const LayerDev* LD, const IoDev* IO,
                                                   const Tile* tiles, Filter F, int src_mode, int out_mode,
                                                   int iter) {
  constexpr int HMAX = RMAX / 2;           // side of the lower block
  constexpr int S = HMAX + 1;              // LDS stride of the lower levels
  constexpr int QHM = HMAX / 2 + 2;        // band window side
  constexpr int WS = 2 * QHM + 1;          // window / column-pass stride
  constexpr int YN = HMAX * WS > HMAX * S ? HMAX * WS : HMAX * S;
  __shared__ float X[HMAX * S];            // lower levels (ping), then the lower block's result
  __shared__ float Y[YN];                  // lower levels (pong), then the column pass
  __shared__ float Wn[2 * QHM * WS];       // the top level's window of four bands
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[t.mask];
  const IoDev& io = IO[t.prob];
  PSrc ps = make_psrc(pr, io, src_mode, iter, 0.f);
  const int n = ly.n, R = ly.res, h = R >> 1, lh = __builtin_ctz(h), off = ly.off;
  const int m0 = n >> ly.levels;
  const int qy = t.tx >> 1, qx = t.tx & 1;  // output quadrant
  const int qh = (h >> 1) + 2;              // window side of each band
  const int nt = blockDim.x;
  const bool lower_owner = t.tx == 0;
  // one round of loads, all in flight together: the lower block (h x h, the
  // Mallat layout's top-left: coarse block and the detail quadrants of every
  // level below the top), then the three detail windows of the top level
  // under this quadrant (qh^2 each); element e of a thread is threadIdx.x + u nt
  constexpr int kUL = (HMAX * HMAX + 3 * QHM * QHM + 511) / 512;
  const int nlow = h * h, nwin = qh * qh, ntot = nlow + 3 * nwin;
  const float rq = 1.0f / (float)qh, rw = 1.0f / (float)nwin;
  CoefLoad v[kUL];
  int pos[kUL], dst[kUL];
  unsigned owned = 0;  // bit u: this thread's window entry u is a coefficient of its own quadrant
  BetaLoads<2> bl;
  beta_issue<2>(pr, ps.mode, iter, bl);
#pragma unroll
  for (int u = 0; u < kUL; ++u) {
    const int e = threadIdx.x + u * nt;
    pos[u] = -1;
    dst[u] = 0;
    if (e < nlow) {
      pos[u] = off + (e >> lh) * n + (e & (h - 1));
      dst[u] = (e >> lh) * S + (e & (h - 1));
    } else if (e < ntot) {
      const int w = e - nlow;
      int b = (int)((float)w * rw), i = w - b * nwin;  // band b: (0, 1), (1, 0), (1, 1)
      if (i >= nwin) { ++b; i -= nwin; }
      if (i < 0) { --b; i += nwin; }
      int iy = (int)((float)i * rq), ix = i - iy * qh;
      if (ix >= qh) { ++iy; ix -= qh; }
      if (ix < 0) { --iy; ix += qh; }
      const int by = (b + 1) >> 1, bx = (b + 1) & 1;
      pos[u] = off + (by * h + ((qy * (h >> 1) - 2 + iy) & (h - 1))) * n + bx * h +
               ((qx * (h >> 1) - 2 + ix) & (h - 1));
      dst[u] = (by * qh + iy) * WS + bx * qh + ix;
      if (iy >= 2 && ix >= 2) owned |= 1u << u;
    }
    if (pos[u] >= 0) v[u] = coef_fetch(ps, pos[u]);
  }
  ps.beta = beta_reduce<2>(ps.mode, bl);  // every lane of every wave is here
#pragma unroll
  for (int u = 0; u < kUL; ++u) {
    if (pos[u] < 0) continue;
    if ((int)threadIdx.x + u * nt < nlow)
      X[dst[u]] = coef_finish(ps, pos[u], v[u], lower_owner);
    else
      Wn[dst[u]] = coef_finish(ps, pos[u], v[u], (owned >> u) & 1u);
  }
  __syncthreads();
  for (int m = 2 * m0; m <= h; m <<= 1) {
    syn_pass<S>(X, Y, m, F);  // columns: X[t][c] -> Y[c][t]
    __syncthreads();
    syn_pass<S>(Y, X, m, F);  // rows: Y[c][r] -> X[r][c]
    __syncthreads();
  }
  // the coarse band of the top level's window from the lower block's result
  for (int e = threadIdx.x; e < nwin; e += nt) {
    const int iy = e / qh, ix = e - iy * qh;
    Wn[iy * WS + ix] = X[((qy * (h >> 1) - 2 + iy) & (h - 1)) * S + ((qx * (h >> 1) - 2 + ix) & (h - 1))];
  }
  __syncthreads();
  // columns: one window column and a run of 4 output pairs per task
  constexpr int kRun = 4;
  const int wcols = 2 * qh;
  for (int task = threadIdx.x; task < wcols * (h / 2 / kRun); task += nt) {
    const int lx = task % wcols, t0p = (task / wcols) * kRun;
    syn_run<kRun>(Wn + lx, Wn + qh * WS + lx, WS, t0p, F, Y + 2 * t0p * WS + lx, WS);
  }
  __syncthreads();
  // rows, straight to the output quadrant (the layer, or the coarse block of
  // the first global level)
  const bool final_level = (n == R);
  const OutDst od = out_dst(pr, io, out_mode);
  const gptr_w nxt = (gptr_w)(pr.tmpa + ly.tmp_off);  // stride R
  const int r0 = qy * h, c0 = qx * h;
  for (int e0 = threadIdx.x; e0 < h * h; e0 += kU * nt) {
    OutLoad o[kU];
    if (final_level) {
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * nt;
        if (e < h * h) o[u] = out_fetch(od, off + (r0 + (e >> lh)) * n + c0 + (e & (h - 1)));
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + u * nt;
      if (e >= h * h) break;
      const int lt = e >> lh, ls = e & (h - 1);
      const int par = ls & 1, k = ((ls - par) >> 1) + 2;
      const float* Br = Y + lt * WS;
      const float acc = F.h[par] * Br[k] + F.h[par + 2] * Br[k - 1] + F.h[par + 4] * Br[k - 2] +
                        F.g[par] * Br[qh + k] + F.g[par + 2] * Br[qh + k - 1] + F.g[par + 4] * Br[qh + k - 2];
      const int row = r0 + lt, col = c0 + ls;
      if (final_level)
        out_finish(od, off + row * n + col, acc * ly.inv_delta, o[u]);
      else
        nxt[row * R + col] = acc;
    }
  }
}

// ----------------------------------------------- inverse DWT, one global level
// (Both global-level kernels are held to 64 VGPRs, 8 waves per SIMD: a batch
// launch of 2048 tiles then runs in a single round of workgroups.)
// Output tile 32x32 of the level with side m = 2^t.level (> the resident side).  The
// coarse block comes from scratch, the three detail quadrants from the
// coefficient source; 2 halo coefficients per direction (6 taps, 3 per phase).
constexpr int kGT = 32;           // output tile side
constexpr int kGH = kGT / 2 + 2;  // coefficients per band and direction (18)
constexpr int kGW = 2 * kGH;      // 36

// The two synthesis passes of a global level's output tile from its window
// of four bands in A (coarse block at band (0, 0)): columns into B, then rows
// to the output (the layers, or the next level's coarse block in scratch).
struct GlobOut {
  int n, off, m, t0, s0;
  float inv_delta;
  gptr_w nxt;  // the next level's coarse block in scratch (stride m)
};
__device__ __forceinline__ void idwt_glob_passes(const ProbDev& pr, const IoDev& io, const Filter& F, int out_mode,
                                                 const GlobOut& g, float* A, float* B);

// One output tile of one global level: the window's bands from scratch (the
// coarse block) and the coefficient source (with the fused p update), then
// the passes.
__device__ __forceinline__ void idwt_glob_tile(const ProbDev* P, const LayerDev* LD, const IoDev* IO, const Tile& t,
                                               const Filter& F, int src_mode, int out_mode, int iter, int step,
                                               float* A, float* B) {
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[t.mask];  // the global layer index, carried by the tile
  const IoDev& io = IO[t.prob];
  PSrc ps = make_psrc(pr, io, src_mode, iter, 0.f);
  const int n = ly.n, off = ly.off;
  const int m = 1 << t.level, half = m >> 1;
  const int t0 = t.ty * kGT, s0 = t.tx * kGT;
  const gptr_f ll = (gptr_f)(((step & 1) ? pr.tmpb : pr.tmpa) + ly.tmp_off);  // stride half
  const GlobOut g{n, off, m, t0, s0, ly.inv_delta, (gptr_w)(((step & 1) ? pr.tmpa : pr.tmpb) + ly.tmp_off)};
  const int kr0 = (t0 >> 1) - 2, kc0 = (s0 >> 1) - 2;
  const int W1 = kGW + 1;
  // the window's four bands, one per wave (so no wave mixes the coarse
  // block with the coefficient source): wave 0 the coarse block (scratch),
  // waves 1 .. 3 the detail quadrants (by, bx) = (0, 1), (1, 0), (1, 1)
  constexpr int kBand = kGH * kGH, kRounds = (kBand + 63) / 64;
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int by = wv >> 1, bx = wv & 1;
  // loads without branches (window entries past the band clamped)
  float val[kRounds];
  if (wv == 0) {
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {
      const int e = min(lane + 64 * u, kBand - 1);
      const int iy = e / kGH, ix = e - iy * kGH;
      val[u] = ll[((kr0 + iy) & (half - 1)) * half + ((kc0 + ix) & (half - 1))];
    }
  } else {
    CoefLoad v[kRounds];
    int gpos[kRounds];
    BetaLoads<1> bl;
    beta_issue<1>(pr, ps.mode, iter, bl);
    const CoefPtrs cp = coef_ptrs(ps);
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {
      const int e = min(lane + 64 * u, kBand - 1);
      const int iy = e / kGH, ix = e - iy * kGH;
      gpos[u] = off + (by * half + ((kr0 + iy) & (half - 1))) * n + bx * half + ((kc0 + ix) & (half - 1));
      v[u] = coef_load(cp, gpos[u]);
    }
    ps.beta = beta_reduce<1>(ps.mode, bl);
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {
      const int e = lane + 64 * u;
      if (e < kBand) {
        const int iy = e / kGH, ix = e - iy * kGH;
        val[u] = coef_finish(ps, gpos[u], v[u], iy >= 2 && ix >= 2);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kRounds; ++u) {
    const int e = lane + 64 * u;
    if (e < kBand) {
      const int iy = e / kGH, ix = e - iy * kGH;
      A[(by * kGH + iy) * W1 + bx * kGH + ix] = val[u];
    }
  }
  __syncthreads();
  idwt_glob_passes(pr, io, F, out_mode, g, A, B);
}

__device__ __forceinline__ void idwt_glob_passes(const ProbDev& pr, const IoDev& io, const Filter& F, int out_mode,
                                                 const GlobOut& g, float* A, float* B) {
  const int n = g.n, off = g.off, m = g.m, t0 = g.t0, s0 = g.s0;
  const gptr_w nxt = g.nxt;
  const int W1 = kGW + 1;
  const int nt = blockDim.x;
  // columns: one input column and a run of 4 output pairs per task (the
  // taps of consecutive pairs overlap, so a run reads 12 taps, not 48)
  constexpr int kRun = 4;
  for (int task = threadIdx.x; task < kGW * (kGT / 2 / kRun); task += nt) {
    const int lx_ = task % kGW, t0p = (task / kGW) * kRun;
    syn_run<kRun>(A + lx_, A + kGH * W1 + lx_, W1, t0p, F, B + 2 * t0p * W1 + lx_, W1);
  }
  __syncthreads();
  const bool final_level = (m == n);
  const OutDst od = out_dst(pr, io, out_mode);
  for (int e0 = threadIdx.x; e0 < kGT * kGT; e0 += kU * nt) {  // rows
    OutLoad o[kU];
    if (final_level) {
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * nt;
        o[u] = out_fetch(od, off + (t0 + (e >> 5)) * n + s0 + (e & 31));
      }
    }
    // the outputs in pairs, both taps' reads ahead of the store branch
    // (with the branch after every output, the compiler waited for each
    // output's LDS reads before issuing the next's)
    auto row_out = [&](int u) {
      const int e = e0 + u * nt;
      const int lt = e >> 5, ls = e & 31;
      const int par = ls & 1, k = ((ls - par) >> 1) + 2;
      const float* Br = B + lt * W1;
      return F.h[par] * Br[k] + F.h[par + 2] * Br[k - 1] + F.h[par + 4] * Br[k - 2] + F.g[par] * Br[kGH + k] +
             F.g[par + 2] * Br[kGH + k - 1] + F.g[par + 4] * Br[kGH + k - 2];
    };
    static_assert(kU % 2 == 0, "outputs in pairs");
#pragma unroll
    for (int u = 0; u < kU; u += 2) {
      const float a[2] = {row_out(u), row_out(u + 1)};
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int e = e0 + (u + v) * nt;
        if (final_level)
          out_finish(od, off + (t0 + (e >> 5)) * n + s0 + (e & 31), a[v] * g.inv_delta, o[u + v]);
        else
          nxt[(t0 + (e >> 5)) * m + s0 + (e & 31)] = a[v];
      }
    }
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_idwt_glob(const ProbDev* P, const LayerDev* LD, const IoDev* IO,
                                                   const Tile* tiles, Filter F, int src_mode, int out_mode,
                                                   int iter, int step) {
  __shared__ float A[kGW * (kGW + 1)];
  __shared__ float B[kGT * (kGW + 1)];
  const Tile t = my_tile(tiles);
  idwt_glob_tile(P, LD, IO, t, F, src_mode, out_mode, iter, step, A, B);
}

// The last two global levels of a layer in one tile (output side m = n, the
// layer's own side): the inner level (output side m/2) is synthesized in LDS
// for the 18 x 18 window of its output that the outer level's tile needs,
// from 11 x 11 windows of its four bands (coarse block from scratch, detail
// quadrants from the coefficient source with the fused p update), then the
// outer level as a single-level tile.  Neighbouring tiles recompute the
// overlap of their inner windows (about 27 % more inner-level work) and save
// a launch; each inner coefficient's p is written by the tile whose 8 x 8
// stride it falls in (window entries 3 .. 10 in each direction).
constexpr int kGI = kGH / 2 + 2;  // inner band window side (11)
constexpr int kGIW = 2 * kGI;     // 22

__device__ __forceinline__ void idwt_glob2_tile(const ProbDev* P, const LayerDev* LD, const IoDev* IO, const Tile& t,
                                                const Filter& F, int src_mode, int out_mode, int iter, int step,
                                                float* A, float* B, float* A2, float* B2) {
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[t.mask];
  const IoDev& io = IO[t.prob];
  PSrc ps = make_psrc(pr, io, src_mode, iter, 0.f);
  const int n = ly.n, off = ly.off;
  const int m = 1 << t.level, half = m >> 1, quart = m >> 2;
  const int t0 = t.ty * kGT, s0 = t.tx * kGT;
  // the inner level's coarse block (side quart) in this step's scratch
  const gptr_f ll = (gptr_f)(((step & 1) ? pr.tmpb : pr.tmpa) + ly.tmp_off);
  const GlobOut g{n, off, m, t0, s0, ly.inv_delta, (gptr_w)(((step & 1) ? pr.tmpa : pr.tmpb) + ly.tmp_off)};
  const int kr0 = (t0 >> 1) - 2, kc0 = (s0 >> 1) - 2;  // outer band window origin (mod half)
  const int jr0 = (kr0 >> 1) - 2, jc0 = (kc0 >> 1) - 2;  // inner band window origin (mod quart)
  const int W1 = kGW + 1, W2 = kGIW + 1;
  const int nt = blockDim.x;
  constexpr int kIB = kGI * kGI, kIR = (kIB + 63) / 64;    // inner band entries, rounds per lane
  constexpr int kBand = kGH * kGH, kRounds = (kBand + 63) / 64;
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int by = wv >> 1, bx = wv & 1;
  // wave 0: the inner coarse window; waves 1 .. 3: the inner and the outer
  // detail windows of band (by, bx), all loads in flight together
  // loads without branches (window entries past the bands clamped)
  float ival[kIR];
  if (wv == 0) {
#pragma unroll
    for (int u = 0; u < kIR; ++u) {
      const int e = min(lane + 64 * u, kIB - 1);
      const int iy = e / kGI, ix = e - iy * kGI;
      ival[u] = ll[((jr0 + iy) & (quart - 1)) * quart + ((jc0 + ix) & (quart - 1))];
    }
  } else {
    CoefLoad iv[kIR], ov[kRounds];
    int ipos[kIR], opos[kRounds];
    BetaLoads<1> bl;
    beta_issue<1>(pr, ps.mode, iter, bl);
    const CoefPtrs cp = coef_ptrs(ps);
#pragma unroll
    for (int u = 0; u < kIR; ++u) {
      const int e = min(lane + 64 * u, kIB - 1);
      const int iy = e / kGI, ix = e - iy * kGI;
      ipos[u] = off + (by * quart + ((jr0 + iy) & (quart - 1))) * n + bx * quart + ((jc0 + ix) & (quart - 1));
      iv[u] = coef_load(cp, ipos[u]);
    }
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {
      const int e = min(lane + 64 * u, kBand - 1);
      const int iy = e / kGH, ix = e - iy * kGH;
      opos[u] = off + (by * half + ((kr0 + iy) & (half - 1))) * n + bx * half + ((kc0 + ix) & (half - 1));
      ov[u] = coef_load(cp, opos[u]);
    }
    ps.beta = beta_reduce<1>(ps.mode, bl);
#pragma unroll
    for (int u = 0; u < kIR; ++u) {
      const int e = lane + 64 * u;
      if (e < kIB) {
        const int iy = e / kGI, ix = e - iy * kGI;
        ival[u] = coef_finish(ps, ipos[u], iv[u], iy >= 3 && ix >= 3);
      }
    }
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {
      const int e = lane + 64 * u;
      if (e < kBand) {
        const int iy = e / kGH, ix = e - iy * kGH;
        A[(by * kGH + iy) * W1 + bx * kGH + ix] = coef_finish(ps, opos[u], ov[u], iy >= 2 && ix >= 2);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kIR; ++u) {
    const int e = lane + 64 * u;
    if (e < kIB) {
      const int iy = e / kGI, ix = e - iy * kGI;
      A2[(by * kGI + iy) * W2 + bx * kGI + ix] = ival[u];
    }
  }
  __syncthreads();
  // inner level, columns: 22 columns x 9 output pairs (runs of 3) -> B2 rows 0 .. 17
  for (int task = threadIdx.x; task < kGIW * 3; task += nt) {
    const int c = task % kGIW, p0 = (task / kGIW) * 3;
    syn_run<3>(A2 + c, A2 + kGI * W2 + c, W2, p0, F, B2 + 2 * p0 * W2 + c, W2);
  }
  __syncthreads();
  // inner level, rows: 18 rows x 9 output pairs -> the outer window's coarse band
  for (int task = threadIdx.x; task < kGH * 3; task += nt) {
    const int r = task % kGH, p0 = (task / kGH) * 3;
    syn_run<3>(B2 + r * W2, B2 + r * W2 + kGI, 1, p0, F, A + r * W1 + 2 * p0, 1);
  }
  __syncthreads();
  idwt_glob_passes(pr, io, F, out_mode, g, A, B);
}

// A launch of global-level tiles of which some are fused pairs of levels
// (tile pad1 = 1): plans with fused tiles launch this kernel instead of
// k_idwt_glob.
__global__ __launch_bounds__(256) void k_idwt_glob2(const ProbDev* P, const LayerDev* LD, const IoDev* IO,
                                                    const Tile* tiles, Filter F, int src_mode, int out_mode, int iter,
                                                    int step) {
  __shared__ float A[kGW * (kGW + 1)];
  __shared__ float B[kGT * (kGW + 1)];
  __shared__ float A2[kGIW * (kGIW + 1)];
  __shared__ float B2[kGH * (kGIW + 1)];
  const Tile t = my_tile(tiles);
  if (t.pad1)
    idwt_glob2_tile(P, LD, IO, t, F, src_mode, out_mode, iter, step, A, B, A2, B2);
  else
    idwt_glob_tile(P, LD, IO, t, F, src_mode, out_mode, iter, step, A, B);
}

// ------------------------------------------------ forward DWT, one global level
// Input side m = 2^t.level (> the resident side); output 16x16 coefficients of each of
// the four quadrants per tile; input window 36x36 (2k .. 2k+5 per output).
constexpr int kFT = 16;           // output coefficients per direction
constexpr int kFW = 2 * kFT + 4;  // 36 input samples per direction

// EK: the epilogue as a compile-time constant (the PCG one, so that its
// loads are straight-line code), or -1 to take it from epi.
template <int EK>
__device__ __forceinline__ void fdwt_glob_tile(const ProbDev* P, const LayerDev* LD, const IoDev* IO, const Tile t,
                                               const Filter F, int epi_arg, int iter, int step, float* X, float* Rw,
                                               double* sh) {
  const int epi = EK >= 0 ? EK : epi_arg;
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[t.mask];  // the global layer index, carried by the tile
  const IoDev& io = IO[t.prob];
  const int n = ly.n, off = ly.off;
  const int m = 1 << t.level, half = m >> 1;
  const gptr_f in = (gptr_f)((step == 0) ? pr.phiadj + off : (((step & 1) ? pr.tmpa : pr.tmpb) + ly.tmp_off));
  const int istride = (step == 0) ? n : m;
  const gptr_w llout = (gptr_w)(((step & 1) ? pr.tmpb : pr.tmpa) + ly.tmp_off);  // stride half
  const int k0 = t.ty * kFT, l0 = t.tx * kFT;
  const int XW = kFW + 1, RW = 2 * kFT + 1;
  const int nt = blockDim.x;
  // epilogue positions and operands of this thread's outputs (the 512
  // (row, column) pairs of the column pass, 2 per thread, up to 2 outputs
  // each), requested with the input window so both latencies overlap
  int epos[4];
  EpiLoad el[4];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = threadIdx.x + u * nt;
    const int lk = e / (2 * kFT), lc = e - lk * (2 * kFT);
    const int row = k0 + lk;
    const int xd = lc >= kFT;
    const int col = l0 + lc - xd * kFT;
    epos[2 * u] = xd ? off + row * n + (half + col) : -1;  // the a output is a detail only right of the coarse block
    epos[2 * u + 1] = off + (half + row) * n + (xd * half + col);
  }
  // loads without branches, the window's first (so that the compiler's wait
  // for the window leaves the epilogue operands in flight): window entries
  // past the window are clamped, a missing a output reads the line of the
  // thread's d output
  {
    float v[kUG];
#pragma unroll
    for (int u = 0; u < kUG; ++u) {
      const int e = min((int)threadIdx.x + u * nt, kFW * kFW - 1);
      const int ry = e / kFW, rx = e - ry * kFW;
      v[u] = in[((2 * k0 + ry) & (m - 1)) * istride + ((2 * l0 + rx) & (m - 1))];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) el[k] = epi_fetch(pr, io, epi, iter, epos[k] >= 0 ? epos[k] : epos[k | 1]);
#pragma unroll
    for (int u = 0; u < kUG; ++u) {
      const int e = threadIdx.x + u * nt;
      if (e < kFW * kFW) {
        const int ry = e / kFW, rx = e - ry * kFW;
        X[ry * XW + rx] = v[u];
      }
    }
    for (int e = threadIdx.x + kUG * nt; e < kFW * kFW; e += nt) {  // workgroups under 256 threads only
      const int ry = e / kFW, rx = e - ry * kFW;
      X[ry * XW + rx] = in[((2 * k0 + ry) & (m - 1)) * istride + ((2 * l0 + rx) & (m - 1))];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kFW * kFT; e += nt) {  // rows (along x)
    const int ry = e / kFT, lk = e - ry * kFT;
    const float* xr = X + ry * XW + 2 * lk;
    float a = 0.f, d = 0.f;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      a += F.h[i] * xr[i];
      d += F.g[i] * xr[i];
    }
    Rw[ry * RW + lk] = a;
    Rw[ry * RW + kFT + lk] = d;
  }
  __syncthreads();
  double acc = 0.0;
  const float ad = ly.alpha_d[t.level - 1];  // detail blocks of this level have side half = 2^(level - 1)
  const EpiDst dst = epi_dst(pr, io, iter);
  // 512 (row, column) pairs of the column pass, 2 per thread; each yields up to 2 outputs
  {
    float eval[4];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = threadIdx.x + u * nt;
      const int lk = e / (2 * kFT), lc = e - lk * (2 * kFT);
      float a = 0.f, d = 0.f;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const float v = Rw[(2 * lk + i) * RW + lc];
        a += F.h[i] * v;
        d += F.g[i] * v;
      }
      const int row = k0 + lk;
      const int xd = lc >= kFT;
      const int col = l0 + lc - xd * kFT;
      if (!xd)
        llout[row * half + col] = a;  // coarse block for the next level
      else
        eval[2 * u] = a * ly.inv_delta;
      eval[2 * u + 1] = d * ly.inv_delta;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (epos[k] >= 0) epi_finish(dst, epi, epos[k], ad, eval[k], el[k], acc);
  }
  if (epi == EPI_PCG || epi == EPI_RHS || epi == EPI_RHSQ) {
    const double s = block_sum(acc, sh, nt);
    if (threadIdx.x == 0) ((gptr_wd)pr.dots)[(long)dot_group_of(epi, iter) * pr.n_dots + t.slot] = s;
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_fdwt_glob(const ProbDev* P, const LayerDev* LD, const IoDev* IO,
                                                   const Tile* tiles, Filter F, int epi, int iter, int step) {
  __shared__ float X[kFW * (kFW + 1)];
  __shared__ float Rw[kFW * (2 * kFT + 1)];
  __shared__ double sh[4];
  const Tile t = my_tile(tiles);
  if (epi == EPI_PCG)
    fdwt_glob_tile<EPI_PCG>(P, LD, IO, t, F, epi, iter, step, X, Rw, sh);
  else
    fdwt_glob_tile<-1>(P, LD, IO, t, F, epi, iter, step, X, Rw, sh);
}

// The first two global levels of a layer in one tile (input side m = n, the
// layer's own side, at step 0): the outer level (m -> m/2) is analysed for
// the 20 x 20 window of its coarse output that the inner level (m/2 -> m/4)
// needs, plus its own 16 x 16 x 3 detail outputs, from a 44 x 44 input
// window; the inner level gives 8 x 8 outputs of each band.  Both levels'
// details take the epilogue; the inner coarse block goes to scratch where
// the inner level's own launch would have put it.  Each output is the same
// sum as in the single-level tiles (about 56 % more outer coarse work, one
// launch fewer per forward transform).
constexpr int kF2 = 8;                 // inner outputs per band and direction
constexpr int kF1C = 2 * kF2 + 4;      // outer coarse values per direction (20)
constexpr int kF2W = 2 * kF1C + 4;     // input samples per direction (44)

template <int EK>  // as in fdwt_glob_tile
__device__ __forceinline__ void fdwt_glob2_tile(const ProbDev* P, const LayerDev* LD, const IoDev* IO, const Tile& t,
                                                const Filter& F, int epi_arg, int iter, int step, float* X, float* R1,
                                                float* X2, float* R2, double* sh) {
  const int epi = EK >= 0 ? EK : epi_arg;
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[t.mask];
  const IoDev& io = IO[t.prob];
  const int n = ly.n, off = ly.off;
  const int m = 1 << t.level, half = m >> 1, quart = m >> 2;
  const gptr_f in = (gptr_f)((step == 0) ? pr.phiadj + off : (((step & 1) ? pr.tmpa : pr.tmpb) + ly.tmp_off));
  const int istride = (step == 0) ? n : m;
  const gptr_w llout = (gptr_w)((((step + 1) & 1) ? pr.tmpb : pr.tmpa) + ly.tmp_off);  // stride quart
  const int k0 = t.ty * kFT, l0 = t.tx * kFT;  // outer detail outputs (and coarse window) origin
  const int k2 = t.ty * kF2, l2 = t.tx * kF2;  // inner outputs origin
  const int XW = kF2W + 1, R1W = kF1C + kFT + 1, X2W = kF1C + 1, R2W = 2 * kF2 + 1;
  const int nt = blockDim.x;
  // epilogue positions and operands, requested with the input window:
  // outer details e < 768 (band e / 256: (y low, x high), (y high, x low),
  // (y high, x high)), three per thread; inner details e < 192, one per
  // thread.  Loads without branches, the window's first, so that the
  // compiler's wait for the window leaves the epilogue operands in flight (a
  // thread without an inner output reads the line of its first outer one;
  // window entries past the window are clamped).
  int p1[3], p2;
  EpiLoad e1[3], e2;
  constexpr int kIn = kF2W * kF2W, kUI = (kIn + 255) / 256;
  {
    float v[kUI];
#pragma unroll
    for (int u = 0; u < kUI; ++u) {
      const int e = min((int)threadIdx.x + u * nt, kIn - 1);
      const int ry = e / kF2W, rx = e - ry * kF2W;
      v[u] = in[((2 * k0 + ry) & (m - 1)) * istride + ((2 * l0 + rx) & (m - 1))];
    }
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int e = threadIdx.x + u * nt, b = e >> 8, lk = (e & 255) >> 4, lc = e & 15;
      p1[u] = off + ((b >= 1) * half + k0 + lk) * n + (b != 1) * half + l0 + lc;
      e1[u] = epi_fetch(pr, io, epi, iter, p1[u]);
    }
    {
      const int e = threadIdx.x, b = e >> 6, lk = (e & 63) >> 3, lc = e & 7;
      p2 = e < 192 ? off + ((b >= 1) * quart + k2 + lk) * n + (b != 1) * quart + l2 + lc : -1;
      e2 = epi_fetch(pr, io, epi, iter, p2 >= 0 ? p2 : p1[0]);
    }
#pragma unroll
    for (int u = 0; u < kUI; ++u) {
      const int e = threadIdx.x + u * nt;
      if (e < kIn) {
        const int ry = e / kF2W, rx = e - ry * kF2W;
        X[ry * XW + rx] = v[u];
      }
    }
    for (int e = threadIdx.x + kUI * nt; e < kIn; e += nt) {  // workgroups under 256 threads only
      const int ry = e / kF2W, rx = e - ry * kF2W;
      X[ry * XW + rx] = in[((2 * k0 + ry) & (m - 1)) * istride + ((2 * l0 + rx) & (m - 1))];
    }
  }
  __syncthreads();
  // outer rows (along x): 44 rows x (20 low, 16 high)
  for (int e = threadIdx.x; e < kF2W * (kF1C + kFT); e += nt) {
    const int ry = e / (kF1C + kFT), c = e - ry * (kF1C + kFT);
    const bool hi = c >= kF1C;
    const int lk = hi ? c - kF1C : c;
    const float* xr = X + ry * XW + 2 * lk;
    float a = 0.f;
#pragma unroll
    for (int i = 0; i < 6; ++i) a += (hi ? F.g[i] : F.h[i]) * xr[i];
    R1[ry * R1W + c] = a;
  }
  __syncthreads();
  double acc = 0.0;
  const EpiDst dst = epi_dst(pr, io, iter);
  // outer columns: the 20 x 20 coarse window for the inner level ...
  for (int e = threadIdx.x; e < kF1C * kF1C; e += nt) {
    const int lk = e / kF1C, lc = e - lk * kF1C;
    float a = 0.f;
#pragma unroll
    for (int i = 0; i < 6; ++i) a += F.h[i] * R1[(2 * lk + i) * R1W + lc];
    X2[lk * X2W + lc] = a;
  }
  // ... and the outer details with the epilogue
  {
    const float ad = ly.alpha_d[t.level - 1];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int e = threadIdx.x + u * nt, b = e >> 8, lk = (e & 255) >> 4, lc = e & 15;
      const int col = b == 1 ? lc : kF1C + lc;  // x low (b = 1) or x high
      float d = 0.f;
#pragma unroll
      for (int i = 0; i < 6; ++i) d += (b == 0 ? F.h[i] : F.g[i]) * R1[(2 * lk + i) * R1W + col];
      epi_finish(dst, epi, p1[u], ad, d * ly.inv_delta, e1[u], acc);
    }
  }
  __syncthreads();
  // inner rows: 20 rows x (8 low, 8 high)
  for (int e = threadIdx.x; e < kF1C * 2 * kF2; e += nt) {
    const int ry = e / (2 * kF2), c = e - ry * (2 * kF2);
    const bool hi = c >= kF2;
    const int lk = hi ? c - kF2 : c;
    const float* xr = X2 + ry * X2W + 2 * lk;
    float a = 0.f;
#pragma unroll
    for (int i = 0; i < 6; ++i) a += (hi ? F.g[i] : F.h[i]) * xr[i];
    R2[ry * R2W + c] = a;
  }
  __syncthreads();
  // inner columns: the coarse block to scratch, the details with the epilogue
  {
    const float ad = ly.alpha_d[t.level - 2];
    if (threadIdx.x < 4 * kF2 * kF2) {
      const int e = threadIdx.x, b = e >> 6, lk = (e & 63) >> 3, lc = e & 7;
      // b = 0 .. 2: the details as above; b = 3: the coarse block
      const int col = (b == 1 || b == 3) ? lc : kF2 + lc;
      const bool yhi = b == 1 || b == 2;
      float v = 0.f;
#pragma unroll
      for (int i = 0; i < 6; ++i) v += (yhi ? F.g[i] : F.h[i]) * R2[(2 * lk + i) * R2W + col];
      if (b == 3)
        llout[(k2 + lk) * quart + l2 + lc] = v;
      else
        epi_finish(dst, epi, p2, ad, v * ly.inv_delta, e2, acc);
    }
  }
  if (epi == EPI_PCG || epi == EPI_RHS || epi == EPI_RHSQ) {
    const double s = block_sum(acc, sh, nt);
    if (threadIdx.x == 0) ((gptr_wd)pr.dots)[(long)dot_group_of(epi, iter) * pr.n_dots + t.slot] = s;
  }
}

// A launch of forward global-level tiles of which some are fused pairs of
// levels (tile pad1 = 1): plans with fused tiles launch this kernel instead
// of k_fdwt_glob.
__global__ __launch_bounds__(256) void k_fdwt_glob2(const ProbDev* P, const LayerDev* LD, const IoDev* IO,
                                                    const Tile* tiles, Filter F, int epi, int iter, int step) {
  __shared__ float X[kF2W * (kF2W + 1)];
  __shared__ float R1[kF2W * (kF1C + kFT + 1)];
  __shared__ float X2[kF1C * (kF1C + 1)];
  __shared__ float R2[kF1C * (2 * kF2 + 1)];
  __shared__ double sh[4];
  const Tile t = my_tile(tiles);
  if (epi == EPI_PCG) {
    if (t.pad1)
      fdwt_glob2_tile<EPI_PCG>(P, LD, IO, t, F, epi, iter, step, X, R1, X2, R2, sh);
    else
      fdwt_glob_tile<EPI_PCG>(P, LD, IO, t, F, epi, iter, step, X, R1, sh);
  } else {
    if (t.pad1)
      fdwt_glob2_tile<-1>(P, LD, IO, t, F, epi, iter, step, X, R1, X2, R2, sh);
    else
      fdwt_glob_tile<-1>(P, LD, IO, t, F, epi, iter, step, X, R1, sh);
  }
}

// ------------------------------------------------ forward DWT, resident part
// One line of an analysis pass: output pairs K0 .. K0 + NP - 1 of a periodic
// line of side m read at src[x str]:
//   a_k = sum_i h_i x[(2k + i) mod m],  d_k = sum_i g_i x[(2k + i) mod m]
// Consecutive pairs share four of their six taps: 2 NP + 4 reads per line.
// The first 2 NP taps never wrap (K0 + NP <= m / 2) and are read at fixed
// offsets (the stride STR is a compile-time constant); the last four may.
template <int NP, int STR>
__device__ __forceinline__ void ana_line(const float* src, int m, int K0, const Filter& F, float a[NP], float d[NP]) {
  float x[2 * NP + 4];
  const float* b = src + 2 * K0 * STR;
#pragma unroll
  for (int i = 0; i < 2 * NP; ++i) x[i] = b[i * STR];
#pragma unroll
  for (int i = 2 * NP; i < 2 * NP + 4; ++i) x[i] = src[((2 * K0 + i) & (m - 1)) * STR];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    a[p] = 0.f;
    d[p] = 0.f;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      a[p] += F.h[i] * x[2 * p + i];
      d[p] += F.g[i] * x[2 * p + i];
    }
  }
}

// Output pairs per thread and line of an analysis level of side m at 1024
// threads (at least 1).
constexpr int ana_np(int m) { return m * (m / 2) / 1024 > 1 ? m * (m / 2) / 1024 : 1; }
constexpr int ilog2c(int m) { return m <= 1 ? 0 : 1 + ilog2c(m / 2); }

// The epilogue operands of every output of this thread at the levels of side
// M and below (LevelOps) or at level M alone (OneLevelOps), in registers, so
// that they are requested long before the level needs them.  Operands an
// epilogue does not read stay constant zeros and take no registers.
template <int M>
struct OneLevelOps {
  EpiLoad l[2 * ana_np(M)];
};
template <int M>
struct LevelOps {
  EpiLoad l[2 * ana_np(M)];
  LevelOps<M / 2> next;
};
template <>
struct LevelOps<1> {};

// Level M's operands: thread task = column c, output pairs K0 .. K0 + NP - 1
// of the column pass (as in epi_level).
template <int M, int EPI>
__device__ __forceinline__ void epi_fetch_level(const ProbDev& pr, const IoDev& io, int iter, int off, int n, int R,
                                                int m0, EpiLoad* l) {
  // Loads without branches, so that the compiler's waits for one level's
  // operands leave the later levels' in flight: a thread without an output
  // at this level (or a level that is not resident) reads the layer's first
  // coefficient, and the unused first operand of a column in the coarse half
  // reads the line of its second.
  constexpr int NP = ana_np(M), half = M / 2;
  if (EPI == EPI_PLAIN) return;
  const bool act = M <= R && M > m0 && (int)threadIdx.x < M * (half / NP);
  const int c = threadIdx.x & (M - 1), K0 = ((int)threadIdx.x >> ilog2c(M)) * NP;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int k = K0 + p;
    l[2 * p] = epi_fetch(pr, io, EPI, iter, act ? off + (c >= half ? k : half + k) * n + c : off);
    l[2 * p + 1] = epi_fetch(pr, io, EPI, iter, act ? off + (half + k) * n + c : off);
  }
}
template <int M, int EPI>
__device__ __forceinline__ void epi_fetch_levels(const ProbDev& pr, const IoDev& io, int iter, int off, int n, int R,
                                                 int m0, LevelOps<M>& o) {
  epi_fetch_level<M, EPI>(pr, io, iter, off, n, R, m0, o.l);
  if constexpr (M > 2) epi_fetch_levels<M / 2, EPI>(pr, io, iter, off, n, R, m0, o.next);
}

// One analysis level of side M in LDS (A and B with row stride S), NP output
// pairs per thread and line: rows A -> B (lanes on rows), then columns B -> A
// (lanes on consecutive columns) with the epilogue of every detail output
// from operands already in registers; the coarse block stays in A for the
// next level.
template <int M, int S, int EPI>
__device__ __forceinline__ void epi_level(const LayerDev& ly, const EpiDst& dst, float* A, float* B, const Filter& F,
                                          const EpiLoad* el, double& acc) {
  constexpr int NP = ana_np(M), half = M / 2, lm = ilog2c(M);
  const int n = ly.n, off = ly.off;
  const float ad = ly.alpha_d[lm - 1], inv_delta = ly.inv_delta;
  const bool mine = (int)threadIdx.x < M * (half / NP);
  const int c = threadIdx.x & (M - 1), K0 = ((int)threadIdx.x >> lm) * NP;
  if (mine) {  // rows
    float a[NP], d[NP];
    ana_line<NP, 1>(A + c * S, M, K0, F, a, d);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      B[c * S + K0 + p] = a[p];
      B[c * S + half + K0 + p] = d[p];
    }
  }
  __syncthreads();
  if (mine) {  // columns and the epilogue
    float a[NP], d[NP];
    ana_line<NP, S>(B + c, M, K0, F, a, d);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int k = K0 + p;
      if (c >= half) epi_finish(dst, EPI, off + k * n + c, ad, a[p] * inv_delta, el[2 * p], acc);
      epi_finish(dst, EPI, off + (half + k) * n + c, ad, d[p] * inv_delta, el[2 * p + 1], acc);
      A[k * S + c] = a[p];  // rows >= half of A are no longer read
    }
  }
  __syncthreads();
}

template <int M, int S, int EPI>
__device__ __forceinline__ void epi_levels(const LayerDev& ly, const EpiDst& dst, float* A, float* B, int R, int m0,
                                           const Filter& F, const LevelOps<M>& o, double& acc) {
  if (M <= R && M > m0) epi_level<M, S, EPI>(ly, dst, A, B, F, o.l, acc);
  if constexpr (M > 2) epi_levels<M / 2, S, EPI>(ly, dst, A, B, R, m0, F, o.next, acc);
}

// One workgroup per (problem, layer): all analysis levels from the resident
// side R down to the coarsest block run in LDS, rows then columns, with the
// epilogue EPI of every output.  LDS rows have the odd stride S = RMAX + 1
// (strided lane access free of bank conflicts).  The PCG epilogue's operand
// (p) for every level is requested with the input; the others (up to three
// operands per output) request the top level's with the input and all lower
// levels' once the top level is done, so that the registers hold one set.
template <int RMAX, int EPI>
__global__ __launch_bounds__(1024) void k_fdwt_res(const ProbDev* P, const LayerDev* LD, const IoDev* IO,
                                                   const Tile* tiles, Filter F, int iter) {
  static_assert(RMAX * RMAX / 2 <= 8 * 1024, "at most 8 output pairs per thread and line at 1024 threads");
  __shared__ float A[RMAX * (RMAX + 1)];
  __shared__ float B[RMAX * (RMAX + 1)];
  __shared__ double sh[16];
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[t.mask];  // the global layer index, carried by the tile
  const IoDev& io = IO[t.prob];
  const int n = ly.n, R = ly.res, lr = __builtin_ctz(R), off = ly.off;
  constexpr int S = RMAX + 1;
  const int nt = blockDim.x;
  const int ng = ly.n_glob_levels;
  const gptr_f in = (gptr_f)((ng == 0) ? pr.phiadj + off : ((((ng - 1) & 1) ? pr.tmpb : pr.tmpa) + ly.tmp_off));
  const int istride = (ng == 0) ? n : R;
  const int m0 = n >> ly.levels;
  // the whole block's loads in flight together, kUL per thread at 1024
  // threads per workgroup (the launch shape), without branches (indices
  // past the block clamped): with a load under a condition the compiler
  // waited for each before the next
  constexpr int kUL = RMAX * RMAX / 1024 > 0 ? RMAX * RMAX / 1024 : 1;
  float v[kUL];
#pragma unroll
  for (int u = 0; u < kUL; ++u) {
    const int e = min((int)threadIdx.x + u * nt, R * R - 1);
    v[u] = in[(e >> lr) * istride + (e & (R - 1))];
  }
  auto block_to_lds = [&]() {
#pragma unroll
    for (int u = 0; u < kUL; ++u) {
      const int e = threadIdx.x + u * nt;
      if (e < R * R) A[(e >> lr) * S + (e & (R - 1))] = v[u];
    }
    for (int e = threadIdx.x + kUL * nt; e < R * R; e += nt)  // workgroups under 1024 threads only
      A[(e >> lr) * S + (e & (R - 1))] = in[(e >> lr) * istride + (e & (R - 1))];
  };
  double acc = 0.0;
  const EpiDst dst = epi_dst(pr, io, iter);
  if constexpr (EPI == EPI_PCG) {
    // every level's operands requested with the block: one memory round trip
    LevelOps<RMAX> ops;
    epi_fetch_levels<RMAX, EPI>(pr, io, iter, off, n, R, m0, ops);
    block_to_lds();
    __syncthreads();
    epi_levels<RMAX, S, EPI>(ly, dst, A, B, R, m0, F, ops, acc);
  } else {
    block_to_lds();
    {
      OneLevelOps<RMAX> top;
      epi_fetch_level<RMAX, EPI>(pr, io, iter, off, n, R, m0, top.l);
      __syncthreads();
      if (RMAX <= R && RMAX > m0) epi_level<RMAX, S, EPI>(ly, dst, A, B, F, top.l, acc);
    }
    if constexpr (RMAX > 2) {
      LevelOps<RMAX / 2> rest;
      epi_fetch_levels<RMAX / 2, EPI>(pr, io, iter, off, n, R, m0, rest);
      epi_levels<RMAX / 2, S, EPI>(ly, dst, A, B, R, m0, F, rest, acc);
    }
  }
  const float adll = ly.alpha_d[__builtin_ctz(m0)];
  for (int e = threadIdx.x; e < m0 * m0; e += nt) {
    const int r = e / m0, c = e - r * m0;
    const int pos = off + r * n + c;
    const EpiLoad l = epi_fetch(pr, io, EPI, iter, pos);
    epi_finish(dst, EPI, pos, adll, A[r * S + c] * ly.inv_delta, l, acc);
  }
  if (EPI == EPI_PCG || EPI == EPI_RHS || EPI == EPI_RHSQ) {
    const double s = block_sum(acc, sh, nt);
    if (threadIdx.x == 0) ((gptr_wd)pr.dots)[(long)dot_group_of(EPI, iter) * pr.n_dots + t.slot] = s;
  }
}

// ------------------------------------------- propagation + Shack-Hartmann
// Sums of K values over a workgroup of nw waves, in wave order (each as
// block_sum would form it); result valid in thread 0.  One barrier; sh holds
// K nw floats.
template <int K>
__device__ __forceinline__ void block_sumk(float a[K], float* sh, int nw) {
#pragma unroll
  for (int k = 0; k < K; ++k) a[k] = wave_sum(a[k]);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sh[K * w + k] = a[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      float r = 0.f;
      for (int i = 0; i < nw; ++i) r += sh[K * i + k];
      a[k] = r;
    }
}
__device__ __forceinline__ void block_sum4(float a[4], float* sh, int nw) { block_sumk<4>(a, sh, nw); }

// Sensor-stage workgroup: 4 waves, one thread per subaperture of a 16 x 16
// tile and one or two corners of its 17 x 17 corner window (8 workgroups fit
// a CU, where 5-wave ones fit 6).
constexpr int kSensThreads = 256;
static_assert((kTileS + 1) * (kTileS + 1) <= 2 * kSensThreads, "17 x 17 window in two corners per thread");

// Tile of 16x16 subapertures of one sensor: v on the 17x17 corners is the
// sum over layers of the bilinear interpolant (LGS cone factor in the
// tables), then s^x, s^y per active subaperture (Sec. 2).  The subaperture
// operands are requested first; the layers go in groups of three (all table
// loads of a group, then all node loads), so a corner waits on two memory
// round trips per three layers.  The tables are the tile's own (rows, at
// tile.level: per layer the 17 window rows' (cell row, fraction), then the
// 17 columns'), addressed from the tile alone, so they are requested with
// the descriptors.
constexpr int kLG = 3;  // layers per group of table and node loads
template <int mode>
__global__ __launch_bounds__(kSensThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_pgamma(const ProbDev* P, const LayerDev* LD, const WfsDev* WD,
                                                         const IoDev* IO, const Tile* tiles, const int2* rows) {
  constexpr int CW = kTileS + 1;
  __shared__ float V[CW * CW];
  __shared__ float sh[4 * (kSensThreads / 64)];
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const WfsDev& w = WD[t.slot];
  const IoDev& io = IO[t.prob];
  const float* phi = (mode == PG_DENSE)                          ? pr.phi
                     : (mode == PG_POL_IN || mode == PG_APREV) ? io.state + 3L * pr.n_c
                                                               : io.in;
  const int N = w.N, nc = w.nc;
  const int i0 = t.ty * kTileS, j0 = t.tx * kTileS;
  // subaperture owned by this thread and its operands
  const int li = threadIdx.x >> 4, lj = threadIdx.x & 15;
  const int i = i0 + li, j = j0 + lj;
  const bool own = threadIdx.x < kTileS * kTileS && i < N && j < N;
  typedef const int __attribute__((address_space(1)))* gptr_i;
  typedef const unsigned char __attribute__((address_space(1)))* gptr_u8;
  // Loads without branches (a subaperture past the grid reads the grid's
  // last one, used only when owned; without 2 x 2 blocks the block loads read
  // the layers' first values, unused), so that the compiler does not wait for
  // them before the table loads below are requested.
  const int ib = min(i, N - 1), jb = min(j, N - 1);
  int ci = -1;
  bool isact;
  if (mode == PG_COMPACT || mode == PG_POL_IN) {  // the compact slope index
    const int cv = ((gptr_i)pr.cmap)[w.m_off + ib * N + jb];
    ci = own ? cv : -1;
    isact = ci >= 0;
  } else {  // the active flag alone
    const int av = ((gptr_u8)pr.amap)[w.m_off + ib * N + jb];
    isact = own & (av != 0);
  }
  const int si = ((gptr_i)pr.srow)[w.rb_off + ib] + j;  // row-span position (valid when active)
  float dsx = 0.f, dsy = 0.f;
  if (mode == PG_RESID_IN) {  // data residual s - A phi (s placed by the slopes input kernel)
    const gptr_f sd = (gptr_f)(pr.sd + w.sp_off);
    const int sc = min(max(si, 0), w.sp_len - 1);  // in range whatever the flag (used only when active)
    dsx = sd[sc];
    dsy = sd[w.sp_len + sc];
  } else if (mode == PG_POL_IN) {  // measured slopes of the active subaperture
    const int cc = max(ci, 0);
    dsx = ((gptr_f)io.in)[w.cs_off + cc];
    dsy = ((gptr_f)io.in)[w.cs_off + w.n_active + cc];
  }
  const gptr_f cb = (gptr_f)(w.blocks ? pr.cinv + w.cinv_off + 3 * (ib * N + jb) : phi);
  const float cb0 = cb[0], cb1 = cb[1], cb2 = cb[2];
  // corners: thread t takes window corners t and t + 256 (the second only for
  // t < 33); the loads of both go out together.  Raw buffer loads: lane
  // offsets from the corner (ic, jc) and the cell, wave-uniform offsets from
  // the layer, so no per-load address arithmetic (no range limit: the tables
  // and cells are valid by construction).
  // The table and node loads are issued without branches, so that the
  // compiler's waits for one group's tables leave nothing else behind them:
  // a thread's second corner past the window reads the window's last
  // corner's entries, a group's layers past the last read the last layer
  // (both then add nothing), and corners outside the grid have table
  // entries (0, 0), the layer's first cell.
  constexpr int kCorn = (CW * CW + kSensThreads - 1) / kSensThreads;
  int vi[kCorn], vj[kCorn];
  bool cin[kCorn];
#pragma unroll
  for (int u = 0; u < kCorn; ++u) {
    const int e = threadIdx.x + u * kSensThreads, ec = min(e, CW * CW - 1);
    const int lci = ec / CW, lcj = ec - lci * CW;
    const int ic = i0 + lci, jc = j0 + lcj;
    cin[u] = e < CW * CW && ic < nc && jc < nc;
    vi[u] = lci * (int)sizeof(int2);         // the corner's row entry of a layer's tables
    vj[u] = (CW + lcj) * (int)sizeof(int2);  // and its column entry
  }
  const __amdgpu_buffer_rsrc_t trs =  // this tile's tables
      __builtin_amdgcn_make_buffer_rsrc((void*)(rows + t.level), (short)0, 0x7fffffff, 0x00020000);
  const __amdgpu_buffer_rsrc_t prs = __builtin_amdgcn_make_buffer_rsrc((void*)phi, (short)0, 0x7fffffff, 0x00020000);
  auto ld = [](__amdgpu_buffer_rsrc_t rs, int vo, int so) {  // so: wave-uniform (stated, or the
    return __builtin_amdgcn_raw_buffer_load_b32(rs, vo, __builtin_amdgcn_readfirstlane(so), 0);  // load loops)
  };
  // the corner values, KC corners per thread: wave 0 takes the window's
  // second corners as well (its first 33 lanes), the other waves one each
  float v[kCorn];
#pragma unroll
  for (int u = 0; u < kCorn; ++u) v[u] = 0.f;
  auto corners = [&](auto kc) {
    constexpr int KC = decltype(kc)::value;
    for (int l0 = 0; l0 < pr.L; l0 += kLG) {
      int lof[kLG], nl[kLG];
#pragma unroll
      for (int k = 0; k < kLG; ++k) {
        const int l = min(l0 + k, pr.L - 1);
        const LayerDev& ly = LD[t.mask + l];
        lof[k] = ly.off;
        nl[k] = ly.n;
      }
      int cell[KC][kLG];
      float wy[KC][kLG], wx[KC][kLG];
#pragma unroll
      for (int u = 0; u < KC; ++u)
#pragma unroll
        for (int k = 0; k < kLG; ++k) {
          const int so = min(l0 + k, pr.L - 1) * 2 * CW * (int)sizeof(int2);
          const auto ry = __builtin_amdgcn_raw_buffer_load_b64(trs, vi[u], __builtin_amdgcn_readfirstlane(so), 0);
          const auto rx = __builtin_amdgcn_raw_buffer_load_b64(trs, vj[u], __builtin_amdgcn_readfirstlane(so), 0);
          cell[u][k] = lof[k] + (int)ry[0] * nl[k] + (int)rx[0];
          wy[u][k] = __uint_as_float(ry[1]);
          wx[u][k] = __uint_as_float(rx[1]);
        }
      float nd[KC][kLG][4];
#pragma unroll
      for (int u = 0; u < KC; ++u)
#pragma unroll
        for (int k = 0; k < kLG; ++k) {
          const int vo = cell[u][k] * (int)sizeof(float), so = nl[k] * (int)sizeof(float);
          nd[u][k][0] = __uint_as_float(ld(prs, vo, 0));
          nd[u][k][1] = __uint_as_float(ld(prs, vo + (int)sizeof(float), 0));
          nd[u][k][2] = __uint_as_float(ld(prs, vo, so));
          nd[u][k][3] = __uint_as_float(ld(prs, vo + (int)sizeof(float), so));
        }
#pragma unroll
      for (int u = 0; u < KC; ++u)
#pragma unroll
        for (int k = 0; k < kLG; ++k) {
          const float top = (1.f - wx[u][k]) * nd[u][k][0] + wx[u][k] * nd[u][k][1];
          const float bot = (1.f - wx[u][k]) * nd[u][k][2] + wx[u][k] * nd[u][k][3];
          const float vn = v[u] + ((1.f - wy[u][k]) * top + wy[u][k] * bot);
          v[u] = cin[u] && l0 + k < pr.L ? vn : v[u];
        }
    }
  };
  static_assert(kCorn == 2 && CW * CW - kSensThreads <= 64, "second corners in wave 0 only");
  if (__builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) == 0)
    corners(std::integral_constant<int, 2>{});
  else
    corners(std::integral_constant<int, 1>{});
#pragma unroll
  for (int u = 0; u < kCorn; ++u) {
    const int e = threadIdx.x + u * kSensThreads;
    if (e < CW * CW) V[e] = v[u];
  }
  __syncthreads();
  float sx = 0.f, sy = 0.f, cx = 0.f, cy = 0.f;
  const bool act = own && isact;
  if (act) {
    const float v00 = V[li * CW + lj], v01 = V[li * CW + lj + 1];
    const float v10 = V[(li + 1) * CW + lj], v11 = V[(li + 1) * CW + lj + 1];
    sx = 0.5f * ((v01 - v00) + (v11 - v10));
    sy = 0.5f * ((v10 - v00) + (v11 - v01));
    if (mode == PG_RESID_IN) {
      sx = dsx - sx;
      sy = dsy - sy;
    } else if (mode == PG_POL_IN) {  // s + Gamma P a^(i-1)
      sx = dsx + sx;
      sy = dsy + sy;
    }
    if (w.blocks) {
      cx = cb0 * sx + cb1 * sy;
      cy = cb1 * sx + cb2 * sy;
    }
  }
  if (mode == PG_COMPACT) {
    if (act) {
      ((gptr_w)io.out)[w.cs_off + ci] = sx;
      ((gptr_w)io.out)[w.cs_off + w.n_active + ci] = sy;
    }
    return;
  }
  if (act) {
    ((gptr_w)pr.sd)[w.sp_off + si] = sx;
    ((gptr_w)pr.sd)[w.sp_off + w.sp_len + si] = sy;
  }
  float a[4] = {sx, sy, cx, cy};
  block_sum4(a, sh, kSensThreads / 64);
  if (threadIdx.x == 0) {
    const gptr_w pp = (gptr_w)(pr.part + w.part_off + 4 * (t.ty * w.tiles_side + t.tx));
    pp[0] = a[0];
    pp[1] = a[1];
    pp[2] = a[2];
    pp[3] = a[3];
  }
}

// Compact input slopes -> the row-span slope buffer, and the tip/tilt partial sums of every
// 16 x 16 subaperture tile (the tiles of the propagation stage, whose sums
// the sensor adjoint reads).  A workgroup takes 2 x 2 such tiles, thread t
// subaperture (t / 16, t mod 16) of each, so all its loads are in flight
// together; each tile's sums are formed as over a workgroup of its own.
template <int ADD>  // add the mirrors' slope response already in the slope buffer (closed loop)
__global__ __launch_bounds__(256) void k_slopes_in(const ProbDev* P, const WfsDev* WD, const IoDev* IO,
                                                   const Tile* tiles) {
  __shared__ float sh[16 * 4];
  typedef const int __attribute__((address_space(1)))* gptr_i;
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const WfsDev& w = WD[t.slot];
  const IoDev& io = IO[t.prob];
  const int N = w.N, ts = w.tiles_side;
  const int li = threadIdx.x >> 4, lj = threadIdx.x & 15;
  const gptr_i cmap = (gptr_i)(pr.cmap + w.m_off);
  const gptr_f in = (gptr_f)io.in;
  const gptr_f cinv = (gptr_f)(pr.cinv + w.cinv_off);
  const gptr_w sd = (gptr_w)(pr.sd + w.sp_off);
  const gptr_i srow = (gptr_i)(pr.srow + w.rb_off);
  const int cs0 = w.cs_off, cs1 = w.cs_off + w.n_active;
  // Loads without per-subaperture branches (indices past the grid or of an
  // inactive subaperture clamped, their values unused), so that the
  // compiler's waits do not hold each map load before the next is requested.
  int pos[4], ci[4], si[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = (2 * t.ty + (u >> 1)) * kTileS + li, j = (2 * t.tx + (u & 1)) * kTileS + lj;
    const bool in_grid = i < N && j < N;
    const int ib = min(i, N - 1), jb = min(j, N - 1);
    const int cv = cmap[ib * N + jb], sr = srow[ib];
    pos[u] = in_grid ? i * N + j : -1;
    ci[u] = in_grid ? cv : -1;
    si[u] = min(max(sr + j, 0), w.sp_len - 1);  // row-span position (the right one when active)
  }
  // the slopes (and their mirror part) first; the 2 x 2 blocks, under a
  // branch of their own, last, so that its waits hold nothing else back
  float sx[4], sy[4], c0[4], c1[4], c2[4], ox[4], oy[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int cc = max(ci[u], 0);
    sx[u] = in[cs0 + cc];
    sy[u] = in[cs1 + cc];
    ox[u] = oy[u] = 0.f;
    if (ADD) {
      ox[u] = ((gptr_f)sd)[si[u]];
      oy[u] = ((gptr_f)sd)[w.sp_len + si[u]];
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) c0[u] = c1[u] = c2[u] = 0.f;
  if (w.blocks) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int pc = 3 * max(pos[u], 0);
      c0[u] = cinv[pc];
      c1[u] = cinv[pc + 1];
      c2[u] = cinv[pc + 2];
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const bool act = ci[u] >= 0;
    sx[u] = act ? sx[u] : 0.f;
    sy[u] = act ? sy[u] : 0.f;
    ox[u] = act ? ox[u] : 0.f;
    oy[u] = act ? oy[u] : 0.f;
    c0[u] = act ? c0[u] : 0.f;
    c1[u] = act ? c1[u] : 0.f;
    c2[u] = act ? c2[u] : 0.f;
  }
  float a[16];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (ADD) {  // s + Gamma P a^(i-1), the sum the propagation kernel forms in one pass
      sx[u] = sx[u] + ox[u];
      sy[u] = sy[u] + oy[u];
    }
    a[4 * u] = sx[u];
    a[4 * u + 1] = sy[u];
    a[4 * u + 2] = c0[u] * sx[u] + c1[u] * sy[u];
    a[4 * u + 3] = c1[u] * sx[u] + c2[u] * sy[u];
    if (ci[u] >= 0) {
      sd[si[u]] = sx[u];
      sd[w.sp_len + si[u]] = sy[u];
    }
  }
  block_sumk<16>(a, sh, 4);
  if (threadIdx.x == 0)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ty = 2 * t.ty + (u >> 1), tx = 2 * t.tx + (u & 1);
      if (ty < ts && tx < ts) {
        const gptr_w pp = (gptr_w)(pr.part + w.part_off + 4 * (ty * ts + tx));
        pp[0] = a[4 * u];
        pp[1] = a[4 * u + 1];
        pp[2] = a[4 * u + 2];
        pp[3] = a[4 * u + 3];
      }
    }
}

// ------------------------------------- noise weighting + Shack-Hartmann adjoint
// Tile of 32x32 corners (4 per thread); the weighted slopes of the 33x33
// subapertures that touch them are formed in LDS (thread t takes window
// entries t, t + 256, ...), all their loads in flight together.  The
// window's rows come from the tile's row table (span base, active flags),
// read with the tile, so only active subapertures' slopes are loaded:
// C_hat^{-1} = (I - T) C^{-1} (I - T) for LGS with tip/tilt removal (means
// from the per-tile partial sums, Sec. 3.2), C^{-1} otherwise; GT_PLAIN
// applies Gamma^T alone.  The subaperture operands are requested before the
// means are reduced.
__global__ __launch_bounds__(256) void k_gammaT(const ProbDev* P, const WfsDev* WD, const Tile* tiles,
                                                const int2* rows, int mode) {
  constexpr int SW = kGtS + 1;                    // subaperture window of the tile
  constexpr int kR = (SW * SW + 255) / 256;       // window elements per thread
  constexpr int kC = kGtS * kGtS / 256;           // corners per thread
  __shared__ float YX[SW * SW];
  __shared__ float YY[SW * SW];
  __shared__ float mean[4];
  typedef const int __attribute__((address_space(1)))* gptr_i;
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const WfsDev& w = WD[t.slot];
  const int N = w.N, nc = w.nc;
  const bool weighted = mode == GT_WEIGHTED;
  const int ci0 = t.ty * kGtS, cj0 = t.tx * kGtS;
  const gptr_f sd = (gptr_f)(pr.sd + w.sp_off);
  typedef int v2i __attribute__((ext_vector_type(2)));
  typedef const v2i __attribute__((address_space(1)))* gptr_i2;
  v2i rw[kR];
#pragma unroll
  for (int u = 0; u < kR; ++u) {
    const int e = threadIdx.x + u * 256;
    rw[u] = v2i{0, 0};
    if (e < SW * SW) rw[u] = ((gptr_i2)rows)[t.level + e / SW];
  }
  bool act[kR];
  float sx[kR], sy[kR], cb0[kR], cb1[kR], cb2[kR];
#pragma unroll
  for (int u = 0; u < kR; ++u) {
    const int e = threadIdx.x + u * 256;
    act[u] = false;
    sx[u] = sy[u] = cb0[u] = cb1[u] = cb2[u] = 0.f;
    if (e < SW * SW) {
      const int li = e / SW, lj = e - li * SW;
      const int i = ci0 - 1 + li, j = cj0 - 1 + lj;  // subaperture
      // flags of columns 0 .. 31 in .y, of column 32 in bit 0 of .x (inactive outside the grid)
      act[u] = lj < 32 ? ((unsigned)rw[u].y >> lj) & 1u : rw[u].x & 1;
      if (act[u]) {
        const int si = (rw[u].x >> 1) + j;  // row-span position
        sx[u] = sd[si];
        sy[u] = sd[w.sp_len + si];
      }
      if (i >= 0 && j >= 0 && i < N && j < N) {
        if (weighted && w.blocks) {
          const gptr_f cb = (gptr_f)(pr.cinv + w.cinv_off + 3 * (i * N + j));
          cb0[u] = cb[0];
          cb1[u] = cb[1];
          cb2[u] = cb[2];
        }
      }
    }
  }
  if (weighted && w.tt) {
    if (threadIdx.x < 64) {  // wave 0: tip/tilt means from the tile partials
      float px = 0.f, py = 0.f, pcx = 0.f, pcy = 0.f;
      const gptr_f pp = (gptr_f)(pr.part + w.part_off);
      for (int k = threadIdx.x; k < w.n_tiles_s; k += 64) {
        px += pp[4 * k];
        py += pp[4 * k + 1];
        pcx += pp[4 * k + 2];
        pcy += pp[4 * k + 3];
      }
      px = wave_sum(px);
      py = wave_sum(py);
      pcx = wave_sum(pcx);
      pcy = wave_sum(pcy);
      if (threadIdx.x == 0) {
        const float mx = px * w.inv_nM, my = py * w.inv_nM;
        mean[0] = mx;
        mean[1] = my;
        mean[2] = w.blocks ? (pcx - (w.sum_cinv[0] * mx + w.sum_cinv[1] * my)) * w.inv_nM : 0.f;
        mean[3] = w.blocks ? (pcy - (w.sum_cinv[2] * mx + w.sum_cinv[3] * my)) * w.inv_nM : 0.f;
      }
    }
  } else if (threadIdx.x < 4) {
    mean[threadIdx.x] = 0.f;
  }
  __syncthreads();
  const float m0 = mean[0], m1 = mean[1], m2 = mean[2], m3 = mean[3];
#pragma unroll
  for (int u = 0; u < kR; ++u) {
    const int e = threadIdx.x + u * 256;
    if (e >= SW * SW) continue;
    float yx = 0.f, yy = 0.f;
    if (act[u]) {
      if (!weighted) {
        yx = sx[u];
        yy = sy[u];
      } else if (w.blocks) {
        const float dx = sx[u] - m0, dy = sy[u] - m1;
        yx = cb0[u] * dx + cb1[u] * dy - m2;
        yy = cb1[u] * dx + cb2[u] * dy - m3;
      } else {
        yx = w.inv_sigma2 * (sx[u] - m0);
        yy = w.inv_sigma2 * (sy[u] - m1);
      }
    }
    YX[e] = yx;
    YY[e] = yy;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kC; ++u) {
    const int e = threadIdx.x + u * 256;
    const int li = e / kGtS, lj = e % kGtS;
    const int i = ci0 + li, j = cj0 + lj;
    if (i < nc && j < nc) {
      // subapertures (i-1, j-1), (i-1, j), (i, j-1), (i, j) sit at local (li, lj) .. (li+1, lj+1)
      const float xa = YX[li * SW + lj], xb = YX[li * SW + lj + 1];
      const float xc = YX[(li + 1) * SW + lj], xd = YX[(li + 1) * SW + lj + 1];
      const float ya = YY[li * SW + lj], yb = YY[li * SW + lj + 1];
      const float yc = YY[(li + 1) * SW + lj], yd = YY[(li + 1) * SW + lj + 1];
      const float v = 0.5f * ((xc - xd) + (xa - xb)) + 0.5f * ((ya + yb) - (yc + yd));
      ((gptr_w)pr.vadj)[w.v_off + i * nc + j] = v;
    }
  }
}

// ------------------------------------------------ propagation adjoint (gather)
// Node (p, q) of a layer gathers from every sensor the corners whose bilinear
// cell touches it, weighted by the transpose of the forward interpolation:
//   phi(p, q) = sum_g sum_{i,j} hat_y(i, p) hat_x(j, q) v_g(i, j).
// The hats are precomputed per (sensor, layer) on the host (HatEnt: first
// corner and K = 2 or 3 weights per node row and per node column), so the
// kernel does no index arithmetic beyond the taps.  Tile = 4 RPT node rows x
// 64 node columns: lane = column, wave w owns the RPT consecutive rows
// w RPT .. w RPT + RPT - 1 (RPT = 4 or 8), so a row's hat is uniform across
// the wave (scalar loads).  The gather is separable: the corner rows that the
// RPT node rows touch form one band (first corners never decrease along an
// axis), each band row is interpolated along x once and reused by every node
// row whose hat covers it; a record's step pattern fixes at compile time
// which band rows each node row reads.  A tile lists only the sensors with a
// nonzero hat in its rows and columns.  Sensors sampling the layer finer than
// 2/3 of its spacing (K = 4 .. 6) take dense band records of up to 15 rows;
// finer than 1/3, or with a band that would not fit (kmax = 0), a general
// loop.  No atomics: every node is written once.
template <int RPT>
__device__ __forceinline__ void pt_general(const GLPar& gp, const float* vadj, int q, int p0, int n,
                                           float acc[RPT]) {
  const double cx = ((double)q - gp.t0x) * gp.inv_rho;
  const int jlo = max((int)floor(cx - gp.inv_rho) + 1, 0), jhi = min((int)ceil(cx + gp.inv_rho) - 1, gp.nc - 1);
  if (jhi < jlo) return;
  const gptr_f va = (gptr_f)(vadj + gp.v_off);
  const float r = (float)gp.rho;
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int p = p0 + u;
    if (p >= n) break;
    const double cy = ((double)p - gp.t0y) * gp.inv_rho;
    const int ilo = max((int)floor(cy - gp.inv_rho) + 1, 0), ihi = min((int)ceil(cy + gp.inv_rho) - 1, gp.nc - 1);
    float s = 0.f;
    for (int i = ilo; i <= ihi; ++i) {
      const float wy = fmaxf(0.f, 1.f - r * fabsf((float)((double)i - cy)));
      float rr = 0.f;
      for (int j = jlo; j <= jhi; ++j) rr += fmaxf(0.f, 1.f - r * fabsf((float)((double)j - cx))) * va[i * gp.nc + j];
      s += wy * rr;
    }
    acc[u] += s;
  }
}


// Wave-uniform read of propagation parameters, which no kernel writes while it
// runs: through the constant address space, i.e. scalar loads.
__device__ __forceinline__ GLPar load_glpar(const GLPar* p) {
  typedef const __attribute__((address_space(4))) double* cdbl;
  typedef const __attribute__((address_space(4))) int* cint;
  const cdbl d = (cdbl)p;
  const cint i = (cint)(d + 4);
  GLPar g;
  g.t0y = d[0];
  g.t0x = d[1];
  g.rho = d[2];
  g.inv_rho = d[3];
  g.nc = i[0];
  g.v_off = i[1];
  g.kmax = i[2];
  g.hat_off = i[3];
  return g;
}

// Head of a band record (scalar loads): first band row, pattern, dense rows.
struct BandHdr {
  int so0, pat, nrows;
};
__device__ __forceinline__ BandHdr load_hdr(const BandRec* rec) {
  typedef const __attribute__((address_space(4))) int* cint;
  const cint p = (cint)rec;
  return BandHdr{p[0], p[1], p[2]};
}

// One band row, K corners per lane: raw buffer loads with the lane's column
// offset vo (from the column hat) and the wave-uniform row offset off.
template <int K>
__device__ __forceinline__ void pt_row(__amdgpu_buffer_rsrc_t rs, int vo, int off, float v[K]) {
#pragma unroll
  for (int b = 0; b < K; ++b)
    v[b] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, vo + b * (int)sizeof(float), off, 0));
}

// One band record with step pattern PAT: the band rows that its node rows
// read (d_3 + K of them), each interpolated along x with the column hat; node
// row u takes its K y taps from band row d_u on.
template <int K, int PAT>
__device__ __forceinline__ void pt_pattern(__amdgpu_buffer_rsrc_t rs, int vo, int so0, int rowb, const BandRec* rec,
                                           const HatEnt& hx, float acc[kBandRows]) {
  typedef const __attribute__((address_space(4))) BandRec* crec;
  constexpr int s0 = K == 3 ? 1 : 0;  // least step
  constexpr int d1 = s0 + (PAT & 1), d2 = d1 + s0 + ((PAT >> 1) & 1), d3 = d2 + s0 + ((PAT >> 2) & 1);
  constexpr int NB = d3 + K;
  static_assert(NB <= pt_band(K, kBandRows), "pattern inside the band");
  float v[NB][K];
#pragma unroll
  for (int s = 0; s < NB; ++s) pt_row<K>(rs, vo, so0 + s * rowb, v[s]);
  float r[NB];
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    float t = hx.w[0] * v[s][0];
#pragma unroll
    for (int b = 1; b < K; ++b) t = fmaf(hx.w[b], v[s][b], t);
    r[s] = t;
  }
  const crec br = (crec)rec;
  constexpr int d[kBandRows] = {0, d1, d2, d3};
#pragma unroll
  for (int u = 0; u < kBandRows; ++u) {
    float t = br->wk[u][0] * r[d[u]];
#pragma unroll
    for (int k = 1; k < K; ++k) t = fmaf(br->wk[u][k], r[d[u] + k], t);
    acc[u] += t;
  }
}

// A band record without a step pattern: its nrows band rows (the rest of the
// band lies past the grid and has zero weights), then dense sums with the
// record's y weights as scalar operands.
template <int K>
__device__ __forceinline__ void pt_dense(__amdgpu_buffer_rsrc_t rs, int vo, const BandHdr& h, int rowb,
                                         const BandRec* rec, const HatEnt& hx, float acc[kBandRows]) {
  typedef const __attribute__((address_space(4))) BandRec* crec;
  constexpr int SB = pt_band(K, kBandRows);
  float v[SB][K];
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    if (s < h.nrows) {
      pt_row<K>(rs, vo, h.so0 + s * rowb, v[s]);
    } else {
#pragma unroll
      for (int b = 0; b < K; ++b) v[s][b] = 0.f;
    }
  }
  float r[SB];
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    float t = hx.w[0] * v[s][0];
#pragma unroll
    for (int b = 1; b < K; ++b) t = fmaf(hx.w[b], v[s][b], t);
    r[s] = t;
  }
  const crec br = (crec)rec;
#pragma unroll
  for (int u = 0; u < kBandRows; ++u) {
    float t = 0.f;
#pragma unroll
    for (int s = 0; s < SB; ++s) t = fmaf(br->w[u][s], r[s], t);
    acc[u] += t;
  }
}

// One band record of one sensor, by its pattern; a record of zero weights
// issues nothing.
template <int K>
__device__ __forceinline__ void pt_record(__amdgpu_buffer_rsrc_t rs, int vo, int rowb, const BandHdr& h,
                                          const BandRec* rec, const HatEnt& hx, float acc[kBandRows]) {
  switch (h.pat) {
    case 0: pt_pattern<K, 0>(rs, vo, h.so0, rowb, rec, hx, acc); break;
    case 1: pt_pattern<K, 1>(rs, vo, h.so0, rowb, rec, hx, acc); break;
    case 2: pt_pattern<K, 2>(rs, vo, h.so0, rowb, rec, hx, acc); break;
    case 3: pt_pattern<K, 3>(rs, vo, h.so0, rowb, rec, hx, acc); break;
    case 4: pt_pattern<K, 4>(rs, vo, h.so0, rowb, rec, hx, acc); break;
    case 5: pt_pattern<K, 5>(rs, vo, h.so0, rowb, rec, hx, acc); break;
    case 6: pt_pattern<K, 6>(rs, vo, h.so0, rowb, rec, hx, acc); break;
    case 7: pt_pattern<K, 7>(rs, vo, h.so0, rowb, rec, hx, acc); break;
    case kPatZero: break;
    default: pt_dense<K>(rs, vo, h, rowb, rec, hx, acc); break;
  }
}

// One sensor of the fast path: a wave's one or two (RPT = 8) band records.
template <int K, int RPT>
__device__ __forceinline__ void pt_sensor(const float* vsens, int nc, const BandRec* rec, const BandHdr& h,
                                          const HatEnt& hx, int ngrp, float acc[RPT]) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)vsens, (short)0, nc * nc * (int)sizeof(float), 0x00020000);
  const int vo = hx.lo * (int)sizeof(float);
  const int rowb = nc * (int)sizeof(float);
  pt_record<K>(rs, vo, rowb, h, rec, hx, acc);
#pragma unroll
  for (int j = 1; j < RPT / kBandRows; ++j) {
    if (j >= ngrp) break;
    pt_record<K>(rs, vo, rowb, load_hdr(rec + j), rec + j, hx, acc + j * kBandRows);
  }
}

// One sensor of a wide pair (K = 4 .. 6 corners per node, corner spacing
// from 1/3 to 2/3 of the node spacing): every record dense, its band rows
// interpolated along x with the column hat's K weights (wx), then node row u
// sums them with the record's weights w[u][s] as scalar operands.  Rows past
// the record's nrows lie outside the grid and have zero weights.
template <int K>
__device__ __forceinline__ void pt_wide_record(__amdgpu_buffer_rsrc_t rs, int vo, int rowb, const BandHdr& h,
                                               const BandRec* rec, const float wx[K], float acc[kBandRows]) {
  typedef const __attribute__((address_space(4))) BandRecW* crec;
  constexpr int SB = pt_band_wide(K);
  if (h.pat == kPatZero) return;
  float v[SB][K];
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    if (s < h.nrows) {
      pt_row<K>(rs, vo, h.so0 + s * rowb, v[s]);
    } else {
#pragma unroll
      for (int b = 0; b < K; ++b) v[s][b] = 0.f;
    }
  }
  float r[SB];
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    float t = wx[0] * v[s][0];
#pragma unroll
    for (int b = 1; b < K; ++b) t = fmaf(wx[b], v[s][b], t);
    r[s] = t;
  }
  const crec br = (crec)rec;
#pragma unroll
  for (int u = 0; u < kBandRows; ++u) {
    float t = 0.f;
#pragma unroll
    for (int s = 0; s < SB; ++s) t = fmaf(br->w[u][s], r[s], t);
    acc[u] += t;
  }
}

template <int K, int RPT>
__device__ __forceinline__ void pt_sensor_wide(const float* vsens, int nc, const BandRec* rec, const BandHdr& h,
                                               const HatEnt& hx, const HatEnt& hx2, int ngrp, float acc[RPT]) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)vsens, (short)0, nc * nc * (int)sizeof(float), 0x00020000);
  const int vo = hx.lo * (int)sizeof(float);
  const int rowb = nc * (int)sizeof(float);
  float wx[K];
#pragma unroll
  for (int b = 0; b < K; ++b) wx[b] = b < 3 ? hx.w[b] : hx2.w[b - 3];
  pt_wide_record<K>(rs, vo, rowb, h, rec, wx, acc);
#pragma unroll
  for (int j = 1; j < RPT / kBandRows; ++j) {
    if (j >= ngrp) break;
    pt_wide_record<K>(rs, vo, rowb, load_hdr(rec + j), rec + j, wx, acc + j * kBandRows);
  }
}

// Tile = 4 RPT node rows x 64 node columns; wave w owns the RPT rows from
// p0 = 4 RPT ty + RPT w (RPT / kBandRows band records).  The tile's sensor
// list (the sensors whose footprint meets it, at most 63, built on the host,
// then a pad entry) is loaded once, entry i in lane i, and read back with
// readlane.  The sensor loop is software-pipelined: the column hat and
// band-record head of the next sensor are requested, unconditionally, before
// the current sensor's loads.
// WIDE: the instantiation with the wide-pair path (more registers), launched
// only for plans that have wide pairs.  SPLIT (RPT = kBandRows): a tile is one
// band record's kBandRows node rows x 64 columns, and its sensor list is
// split over the 4 waves (sensor i to wave i mod 4), whose sums are added in
// LDS in wave order: a quarter of the serial sensor chain per wave, for
// launches with few tiles (single frames).
template <int RPT, bool WIDE, bool SPLIT>
__global__ __launch_bounds__(256) void k_pT(const ProbDev* P, const LayerDev* LD, const WfsDev* WD, const IoDev* IO,
                                            const Tile* tiles, const HatEnt* __restrict__ hats, int n_hats,
                                            const BandRec* __restrict__ bands, const PtEnt* __restrict__ ents,
                                            int mode) {
  static_assert(RPT % kBandRows == 0, "whole band records per wave");
  static_assert(!SPLIT || RPT == kBandRows, "split tiles are one band record");
  typedef const int __attribute__((address_space(1)))* gptr_i;
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const int n = t.mask, loff = t.pad1;  // the layer's side and offset, carried by the tile
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int ne = t.level;  // sensors in the tile's list (<= 63; the pad entry follows)
  // the list, entry i in lane i (loaded by every lane, before any returns)
  int m0 = 0, m1 = 0, m2 = 0, m3 = 0;
  if (lane <= ne) {
    const gptr_i e = (gptr_i)(ents + t.slot + lane);
    m0 = e[0];
    m1 = e[1];
    m2 = e[2];
    m3 = e[3];
  }
  auto ent = [&](int i) {
    return PtEnt{__builtin_amdgcn_readlane(m0, i), __builtin_amdgcn_readlane(m1, i),
                 __builtin_amdgcn_readlane(m2, i), __builtin_amdgcn_readlane(m3, i)};
  };
  const int q = t.tx * kPtW + lane;
  const int p0 = SPLIT ? t.ty * kBandRows : t.ty * 4 * RPT + wv * RPT;
  if (p0 >= n) return;  // wave-uniform (SPLIT: the tile's rows, uniform over the workgroup)
  // lanes past the layer's last column run the sensor loop on that column
  // (every lane stays active for the readlane reads of the list) and store
  // nothing
  const int qc = min(q, n - 1);
  const int wrec = SPLIT ? 0 : wv * (RPT / kBandRows);  // this wave's first record past the tile's
  const int ngrp = min(RPT / kBandRows, (n - p0 + kBandRows - 1) / kBandRows);  // records inside the layer
  float acc[RPT];
#pragma unroll
  for (int u = 0; u < RPT; ++u) acc[u] = 0.f;
  // column hats by buffer loads: lane offset fixed, entry offset wave-uniform
  const __amdgpu_buffer_rsrc_t hrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)hats, (short)0, n_hats * (int)sizeof(HatEnt), 0x00020000);
  const int hlane = (qc - t.tx * kPtW) * (int)sizeof(HatEnt);
  // a wide pair's node has two hat entries
  auto lane_off = [&](const PtEnt& e) { return (WIDE && (e.nck & 7) > 3) ? 2 * hlane : hlane; };
  auto fetch = [&](const PtEnt& e, HatEnt& hx, BandHdr& hd) {  // valid for every entry (see PtEnt)
    const auto h = __builtin_amdgcn_raw_buffer_load_b128(hrs, lane_off(e), e.hx * (int)sizeof(HatEnt), 0);
    hx.lo = (int)h[0];
    hx.w[0] = __uint_as_float(h[1]);
    hx.w[1] = __uint_as_float(h[2]);
    hx.w[2] = __uint_as_float(h[3]);
    hd = load_hdr(bands + e.band + wrec);
  };
  auto sensor = [&](const PtEnt& cur, const HatEnt& hx, const BandHdr& hd) {
    const int K = cur.nck & 7, nc = cur.nck >> 3;
    const float* vs = pr.vadj + cur.v_off;
    const BandRec* rec = bands + cur.band + wrec;
    if (K == 0) {
      pt_general<RPT>(load_glpar(pr.gl + (cur.nck >> 3)), pr.vadj, qc, p0, n, acc);
    } else if (K == 2) {
      pt_sensor<2, RPT>(vs, nc, rec, hd, hx, ngrp, acc);
    } else if (!WIDE || K == 3) {
      pt_sensor<3, RPT>(vs, nc, rec, hd, hx, ngrp, acc);
    } else if constexpr (WIDE) {
      // the second half of the column hat (weights 3 .. 5)
      const auto h2 = __builtin_amdgcn_raw_buffer_load_b128(hrs, 2 * hlane + (int)sizeof(HatEnt),
                                                            cur.hx * (int)sizeof(HatEnt), 0);
      const HatEnt hx2{0, {__uint_as_float(h2[1]), __uint_as_float(h2[2]), __uint_as_float(h2[3])}};
      if (K == 4)
        pt_sensor_wide<4, RPT>(vs, nc, rec, hd, hx, hx2, ngrp, acc);
      else if (K == 5)
        pt_sensor_wide<5, RPT>(vs, nc, rec, hd, hx, hx2, ngrp, acc);
      else
        pt_sensor_wide<6, RPT>(vs, nc, rec, hd, hx, hx2, ngrp, acc);
    }
  };
  HatEnt hx, hxn;
  BandHdr hd, hdn;
  constexpr int step = SPLIT ? 4 : 1;
  const int i0 = SPLIT ? wv : 0;
  fetch(ent(min(i0, ne)), hx, hd);
  for (int i = i0; i < ne; i += step) {
    fetch(ent(min(i + step, ne)), hxn, hdn);  // issued first: the waits for this sensor's loads cover it
    sensor(ent(i), hx, hd);
    hx = hxn;
    hd = hdn;
  }
  const IoDev& io = IO[t.prob];
  const gptr_w dst = (gptr_w)((mode == PT_USER) ? io.out : pr.phiadj);
  if constexpr (SPLIT) {
    __shared__ float red[4][kBandRows][64];
#pragma unroll
    for (int u = 0; u < kBandRows; ++u) red[wv][u][lane] = acc[u];
    __syncthreads();
    const int p = p0 + wv;  // wave w stores node row p0 + w
    if (q < n && p < n)
      dst[loff + p * n + q] = ((red[0][wv][lane] + red[1][wv][lane]) + red[2][wv][lane]) + red[3][wv][lane];
  } else if (q < n) {
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int p = p0 + u;
      if (p < n) dst[loff + p * n + q] = acc[u];
    }
  }
}

// ------------------------------------------------------- augmented PCG
// The previous frame's directions W (m of them) and A W in the state, after
// a_prev and a; their count follows them.
struct AugView {
  const float* P;
  const float* Q;
  int m;
};
__device__ __forceinline__ AugView aug_view(const ProbDev& pr, const IoDev& io) {
  const float* base = io.state + 3L * pr.n_c + 2L * pr.n_act;
  AugView v;
  v.P = base;
  v.Q = base + (long)pr.aug_keep * pr.n_c;
  const float cnt = ((gptr_f)(base + 2L * pr.aug_keep * pr.n_c))[0];
  v.m = (cnt >= 1.f && cnt <= (float)pr.aug_keep) ? (int)cnt : 0;
  return v;
}

// Sums of K doubles over a workgroup of nw waves in wave order; result in
// thread 0's a[].
template <int K>
__device__ __forceinline__ void block_sumk_d(double a[K], double* sh, int nw) {
#pragma unroll
  for (int k = 0; k < K; ++k) a[k] = wave_sum(a[k]);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sh[K * w + k] = a[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double r = 0.0;
      for (int i = 0; i < nw; ++i) r += sh[K * i + k];
      a[k] = r;
    }
  __syncthreads();
}

// Cholesky factor of the m x m Gram matrix W^T A W (lower triangle in g,
// g[r][k] = W_r . (A W)_k for k <= r); a direction whose pivot is not
// positive is dropped (kept = 0, its row and column unused).  Every lane
// computes the same factor.
struct AugFactor {
  double L[kAugMax][kAugMax];
  int kept[kAugMax];
};
__device__ __forceinline__ void aug_factor(const double g[kAugMax][kAugMax], int m, AugFactor& f) {
#pragma unroll
  for (int k = 0; k < kAugMax; ++k) {
    f.kept[k] = 0;
#pragma unroll
    for (int i = 0; i < kAugMax; ++i) f.L[k][i] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < kAugMax; ++k) {
    if (k >= m) break;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < k; ++i)
      if (f.kept[i]) acc += f.L[k][i] * f.L[k][i];
    const double d = g[k][k] - acc;
    if (!(d > 0.0) || !(d < INFINITY)) continue;
    f.kept[k] = 1;
    f.L[k][k] = sqrt(d);
#pragma unroll
    for (int r = k + 1; r < kAugMax; ++r) {
      if (r >= m) break;
      double a2 = 0.0;
#pragma unroll
      for (int i = 0; i < k; ++i)
        if (f.kept[i]) a2 += f.L[r][i] * f.L[k][i];
      f.L[r][k] = (g[r][k] - a2) / f.L[k][k];
    }
  }
}
// x = (W^T A W)^{-1} v on the kept directions (0 on dropped ones).
__device__ __forceinline__ void aug_solve(const AugFactor& f, int m, const double v[kAugMax], double x[kAugMax]) {
  double y[kAugMax];
#pragma unroll
  for (int k = 0; k < kAugMax; ++k) y[k] = x[k] = 0.0;
#pragma unroll
  for (int k = 0; k < kAugMax; ++k)
    if (k < m && f.kept[k]) {
      double a = 0.0;
#pragma unroll
      for (int i = 0; i < k; ++i)
        if (f.kept[i]) a += f.L[k][i] * y[i];
      y[k] = (v[k] - a) / f.L[k][k];
    }
#pragma unroll
  for (int k = kAugMax - 1; k >= 0; --k)
    if (k < m && f.kept[k]) {
      double a = 0.0;
#pragma unroll
      for (int i = k + 1; i < kAugMax; ++i)
        if (i < m && f.kept[i]) a += f.L[i][k] * x[i];
      x[k] = (y[k] - a) / f.L[k][k];
    }
}
__device__ __forceinline__ double aug_group_sum(const ProbDev& pr, int g) {
  return wave_sum_slots(pr.aug_slots + (long)g * pr.n_slots_upd, pr.n_slots_upd);
}

// Partial sums of W^T r_0 and of the lower triangle of W^T A W over one
// chunk of coefficients (r_0: the warm-start residual in the state).
__global__ __launch_bounds__(256) void k_aug_gram(const ProbDev* P, const IoDev* IO, const Tile* tiles) {
  __shared__ double sh[(kAugMax + kAugMax * (kAugMax + 1) / 2) * 4];
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const IoDev& io = IO[t.prob];
  const AugView w = aug_view(pr, io);
  constexpr int NG = kAugMax + kAugMax * (kAugMax + 1) / 2;
  double a[NG];
#pragma unroll
  for (int k = 0; k < NG; ++k) a[k] = 0.0;
  const int e0 = t.ty * kUpdChunk, e1 = min(e0 + kUpdChunk, pr.n_c);
  const gptr_f r = (gptr_f)(io.state + 2L * pr.n_c);
  for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
    const double re = r[e];
    double qv[kAugMax];
#pragma unroll
    for (int l = 0; l < kAugMax; ++l) qv[l] = l < w.m ? (double)((gptr_f)(w.Q + (long)l * pr.n_c))[e] : 0.0;
#pragma unroll
    for (int k = 0; k < kAugMax; ++k) {
      if (k >= w.m) break;
      const double pk = ((gptr_f)(w.P + (long)k * pr.n_c))[e];
      a[kAugD + k] += pk * re;
#pragma unroll
      for (int l = 0; l <= k; ++l) a[kAugMax + k * (k + 1) / 2 + l] += pk * qv[l];  // row k, column l
    }
  }
  block_sumk_d<NG>(a, sh, 4);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NG; ++k) ((gptr_wd)pr.aug_slots)[(long)(kAugD + k) * pr.n_slots_upd + t.slot] = a[k];
}

// The projected start of the augmented PCG: y = G^{-1} W^T r_0,
// x_0 = c + W y, r_0 <- r_0 - (A W) y (in the state), and the partial sums
// of rho_0 = r_0^T J^{-1} r_0 and of (A W)^T J^{-1} r_0.  The first chunk also
// stores the factor of G for the direction kernel.
__global__ __launch_bounds__(256) void k_aug_init(const ProbDev* P, const IoDev* IO, const Tile* tiles) {
  __shared__ double sh[(kAugMax + 1) * 4];
  __shared__ double ys[kAugMax];
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const IoDev& io = IO[t.prob];
  const AugView w = aug_view(pr, io);
  if (threadIdx.x < 64) {  // wave 0: the small system (every lane the same)
    double g[kAugMax][kAugMax], d[kAugMax], y[kAugMax];
#pragma unroll
    for (int k = 0; k < kAugMax; ++k) {
      d[k] = k < w.m ? aug_group_sum(pr, kAugD + k) : 0.0;
#pragma unroll
      for (int l = 0; l < kAugMax; ++l) g[k][l] = (l <= k && k < w.m) ? aug_group_sum(pr, kAugG + k * (k + 1) / 2 + l) : 0.0;
    }
    AugFactor f;
    aug_factor(g, w.m, f);
    aug_solve(f, w.m, d, y);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < kAugMax; ++k) ys[k] = y[k];
      if (t.ty == 0) {
#pragma unroll
        for (int k = 0; k < kAugMax; ++k) {
#pragma unroll
          for (int l = 0; l < kAugMax; ++l) ((gptr_wd)pr.aug_fac)[k * kAugMax + l] = f.L[k][l];
          ((gptr_wd)pr.aug_fac)[kAugMax * kAugMax + k] = (double)f.kept[k];
        }
      }
    }
  }
  __syncthreads();
  const int e0 = t.ty * kUpdChunk, e1 = min(e0 + kUpdChunk, pr.n_c);
  const gptr_w x = (gptr_w)io.state;
  const gptr_w r = (gptr_w)(io.state + 2L * pr.n_c);
  const gptr_f jv = (gptr_f)pr.jinv;
  float yk[kAugMax];
#pragma unroll
  for (int k = 0; k < kAugMax; ++k) yk[k] = (float)ys[k];
  double a[kAugMax + 1] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
    float xe = x[e], re = r[e];
    float qv[kAugMax];
#pragma unroll
    for (int k = 0; k < kAugMax; ++k) {
      qv[k] = 0.f;
      if (k < w.m) {
        qv[k] = ((gptr_f)(w.Q + (long)k * pr.n_c))[e];
        xe = fmaf(yk[k], ((gptr_f)(w.P + (long)k * pr.n_c))[e], xe);
        re = fmaf(-yk[k], qv[k], re);
      }
    }
    x[e] = xe;
    r[e] = re;
    const double z = (double)re * (double)jv[e];
    a[0] += (double)re * z;
#pragma unroll
    for (int k = 0; k < kAugMax; ++k)
      if (k < w.m) a[1 + k] += (double)qv[k] * z;
  }
  block_sumk_d<kAugMax + 1>(a, sh, 4);
  if (threadIdx.x == 0) {
    ((gptr_wd)pr.aug_slots)[(long)kAugRho0 * pr.n_slots_upd + t.slot] = a[0];
#pragma unroll
    for (int k = 0; k < kAugMax; ++k)
      if (k < w.m) ((gptr_wd)pr.aug_slots)[(long)(kAugT + k) * pr.n_slots_upd + t.slot] = a[1 + k];
  }
}

// Direction j of the augmented PCG: z_j = J^{-1} r_j, beta = rho_j / rho_{j-1}
// (0 at j = 0), mu = G^{-1} (A W)^T z_j, p_j = z_j + beta p_{j-1} - W mu.
__global__ __launch_bounds__(256) void k_aug_p(const ProbDev* P, const IoDev* IO, const Tile* tiles, int iter) {
  __shared__ float cs[kAugMax + 1];
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const IoDev& io = IO[t.prob];
  const AugView w = aug_view(pr, io);
  if (threadIdx.x < 64) {
    AugFactor f;
#pragma unroll
    for (int k = 0; k < kAugMax; ++k) {
#pragma unroll
      for (int l = 0; l < kAugMax; ++l) f.L[k][l] = ((gptr_d)pr.aug_fac)[k * kAugMax + l];
      f.kept[k] = ((gptr_d)pr.aug_fac)[kAugMax * kAugMax + k] != 0.0;
    }
    double tv[kAugMax], mu[kAugMax];
#pragma unroll
    for (int k = 0; k < kAugMax; ++k) tv[k] = k < w.m ? aug_group_sum(pr, kAugT + (iter & 1) * kAugMax + k) : 0.0;
    aug_solve(f, w.m, tv, mu);
    double beta = 0.0;
    if (iter > 0) {
      double rk, rkm;
      rho_sum2(pr, iter, rk, rkm);
      beta = rkm != 0.0 ? rk / rkm : 0.0;
    }
    if (threadIdx.x == 0) {
      cs[0] = (float)beta;
#pragma unroll
      for (int k = 0; k < kAugMax; ++k) cs[1 + k] = (float)mu[k];
    }
  }
  __syncthreads();
  const float beta = cs[0];
  const int e0 = t.ty * kUpdChunk, e1 = min(e0 + kUpdChunk, pr.n_c);
  const gptr_f r = (gptr_f)(io.state + 2L * pr.n_c);
  const gptr_f jv = (gptr_f)pr.jinv;
  const gptr_f pold = (gptr_f)p_loc(pr, iter - 1);
  const gptr_w pnew = (gptr_w)p_loc(pr, iter);
  for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
    const float z = r[e] * jv[e];
    float pe = iter > 0 ? fmaf(beta, pold[e], z) : z;
#pragma unroll
    for (int k = 0; k < kAugMax; ++k)
      if (k < w.m) pe = fmaf(-cs[1 + k], ((gptr_f)(w.P + (long)k * pr.n_c))[e], pe);
    pnew[e] = pe;
  }
}

// The frame's first min(iters, aug_keep) directions and images become the
// state's W and A W for the next frame (count after them).
__global__ __launch_bounds__(256) void k_aug_store(const ProbDev* P, const IoDev* IO, const Tile* tiles, int iters) {
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const IoDev& io = IO[t.prob];
  const int kd = min(iters, pr.aug_keep);
  float* base = io.state + 3L * pr.n_c + 2L * pr.n_act;
  const int e0 = t.ty * kUpdChunk, e1 = min(e0 + kUpdChunk, pr.n_c);
  for (int k = 0; k < kd; ++k) {
    const gptr_f ps = (gptr_f)(pr.aug_pdir + (long)k * pr.n_c), qs = (gptr_f)(pr.aug_qdir + (long)k * pr.n_c);
    const gptr_w pd = (gptr_w)(base + (long)k * pr.n_c), qd = (gptr_w)(base + (long)(pr.aug_keep + k) * pr.n_c);
    for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
      pd[e] = ps[e];
      qd[e] = qs[e];
    }
  }
  if (t.ty == 0 && threadIdx.x == 0) ((gptr_w)(base + 2L * pr.aug_keep * pr.n_c))[0] = (float)kd;
}

// ------------------------------------------------------------ PCG update
// a = rho_k / pi_k; x += a p; r -= a q; partial rho_{k+1} = r^T J^{-1} r.
// 2048 coefficients per workgroup as float4: 2 per thread, loads first.
// rho_k with the coarse-level correction of the converged solves:
// r^T z = r^T J^{-1} r + (Z^T r)^T E^{-1} Z^T r (the second part's slots,
// written by k_coarse).
__device__ __forceinline__ const double* coarse_slots(const CoarseDev& c, int k) {
  return c.slots + (long)(k & (kDotRing - 1)) * c.n_slots;
}

// XM: the x update of this step.  UPD_X_ONE: x += a_k p_k.  A frame takes
// two steps' x updates in one pass (the search directions p_{k-1} and p_k
// are both still held): UPD_X_DEFER leaves x for the next step, which as
// UPD_X_PAIR forms x += a_{k-1} p_{k-1}, then += a_k p_k: the same two
// rounded products and sums in the same order (bitwise the same x), with
// a_{k-1} summed again from the same slots; 8 of every 56 bytes per
// coefficient less over the pair.
template <int XM>
__global__ __launch_bounds__(256) void k_update(const ProbDev* P, const IoDev* IO, const Tile* tiles, int iter,
                                                const CoarseDev* C) {
  __shared__ double sh[4];
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const IoDev& io = IO[t.prob];
  const gptr_f4 p = (gptr_f4)p_loc(pr, iter);
  const gptr_f4 pm = (gptr_f4)p_loc(pr, XM == UPD_X_PAIR ? iter - 1 : iter);  // p_{k-1}: pairs only
  const gptr_f4 q = (gptr_f4)q_loc(pr, iter);
  const gptr_f4 jv = (gptr_f4)pr.jinv;
  const gptr_w4 x = (gptr_w4)io.state;
  const gptr_w4 r = (gptr_w4)(io.state + 2L * pr.n_c);
  const int e0 = t.ty * (kUpdChunk / 4);
  const int e1 = min(e0 + kUpdChunk / 4, pr.n_c / 4);
  double acc = 0.0;
  constexpr int V = kUpdChunk / 4 / 256;  // float4 per thread
  v4f xp[V], pp[V], pq[V], rr[V], qq[V], jj[V], rnv[V];
  // rho_k (plus the coarse correction's part in a converged solve) and pi_k
  // (for a pair also rho_{k-1} and pi_{k-1}): slot loads first, summed by
  // every wave itself in the same fixed order (no barrier) while its vector
  // loads are in flight
  int nr, nrm = 0;
  const double* sr = rho_slots(pr, iter, nr);
  const double* srm = XM == UPD_X_PAIR ? rho_slots(pr, iter - 1, nrm) : sr;
  const double* const sl[5] = {sr, dot_group(pr, pi_grp(iter)), C ? coarse_slots(C[t.prob], iter) : sr, srm,
                               XM == UPD_X_PAIR ? dot_group(pr, pi_grp(iter - 1)) : sr};
  const int nn[5] = {nr, pr.n_slots_fdwt, C ? C[t.prob].n_slots : 0, nrm, XM == UPD_X_PAIR ? pr.n_slots_fdwt : 0};
  SlotLoads<5, 2> sloads;
  slots_issue<5, 2>(sl, nn, sloads);
  // loads without branches (indices clamped to the chunk), so that the slot
  // sums below wait only for the slots
#pragma unroll
  for (int u = 0; u < V; ++u) {
    const int e = min(e0 + (int)threadIdx.x + u * 256, e1 - 1);
    if (XM != UPD_X_DEFER) {
      xp[u] = x[e];
      pp[u] = p[e];
    }
    if (XM == UPD_X_PAIR) pq[u] = pm[e];
    rr[u] = r[e];
    qq[u] = q[e];
    jj[u] = jv[e];
  }
  // alpha = rho_k / pi_k
  double o[5];
  slots_reduce<5, 2>(sl, nn, sloads, o);
  const double rho = o[0] + o[2], pi = o[1];
  const float a = (float)((pi > 0.0) ? rho / pi : 0.0);
  // a_{k-1} as the previous step formed it (a frame's steps have no coarse part)
  const double rhom = o[3] + 0.0, pim = o[4];
  const float am = (float)((pim > 0.0) ? rhom / pim : 0.0);
  // breakdown: a nonzero residual with p^T M p <= 0 (M is positive definite,
  // so only rounding or non-finite inputs get here), or a negative or
  // non-finite rho; the step then leaves x and r unchanged (alpha = 0) and
  // the next call on the plan reports it
  if (threadIdx.x == 0 && t.ty == 0 && ((!(pi > 0.0) && rho != 0.0) || !(rho >= 0.0)))
    __hip_atomic_store(pr.numflag, t.prob + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
#pragma unroll
  for (int u = 0; u < V; ++u) {
    const int e = e0 + threadIdx.x + u * 256;
    if (e < e1) {
      v4f xn, rn;
      if (XM == UPD_X_PAIR) {
        xp[u].x = fmaf(am, pq[u].x, xp[u].x);
        xp[u].y = fmaf(am, pq[u].y, xp[u].y);
        xp[u].z = fmaf(am, pq[u].z, xp[u].z);
        xp[u].w = fmaf(am, pq[u].w, xp[u].w);
      }
      if (XM != UPD_X_DEFER) {
        xn.x = fmaf(a, pp[u].x, xp[u].x);
        xn.y = fmaf(a, pp[u].y, xp[u].y);
        xn.z = fmaf(a, pp[u].z, xp[u].z);
        xn.w = fmaf(a, pp[u].w, xp[u].w);
        x[e] = xn;
      }
      rn.x = fmaf(-a, qq[u].x, rr[u].x);
      rn.y = fmaf(-a, qq[u].y, rr[u].y);
      rn.z = fmaf(-a, qq[u].z, rr[u].z);
      rn.w = fmaf(-a, qq[u].w, rr[u].w);
      r[e] = rn;
      rnv[u] = rn;
      acc += (double)rn.x * (double)rn.x * (double)jj[u].x;
      acc += (double)rn.y * (double)rn.y * (double)jj[u].y;
      acc += (double)rn.z * (double)rn.z * (double)jj[u].z;
      acc += (double)rn.w * (double)rn.w * (double)jj[u].w;
    }
  }
  if (pr.aug_keep == 0) {
    const double s = block_sum(acc, sh, blockDim.x);
    if (threadIdx.x == 0) ((gptr_wd)pr.dots)[(long)rho_grp(iter + 1) * pr.n_dots + t.slot] = s;
    return;
  }
  // augmented PCG: also (A W)^T z_{j+1}, z = J^{-1} r, for the next direction
  const AugView w = aug_view(pr, io);
  double tk[kAugMax + 1] = {acc, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < kAugMax; ++k) {
    if (k >= w.m) break;
    const gptr_f4 qk = (gptr_f4)(w.Q + (long)k * pr.n_c);
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int e = e0 + threadIdx.x + u * 256;
      if (e < e1) {
        const v4f a4 = qk[e], r4 = rnv[u];
        tk[1 + k] += (double)a4.x * ((double)r4.x * (double)jj[u].x) + (double)a4.y * ((double)r4.y * (double)jj[u].y) +
                     (double)a4.z * ((double)r4.z * (double)jj[u].z) + (double)a4.w * ((double)r4.w * (double)jj[u].w);
      }
    }
  }
  __shared__ double shk[(kAugMax + 1) * 4];
  block_sumk_d<kAugMax + 1>(tk, shk, blockDim.x >> 6);
  if (threadIdx.x == 0) {
    ((gptr_wd)pr.dots)[(long)rho_grp(iter + 1) * pr.n_dots + t.slot] = tk[0];
#pragma unroll
    for (int k = 0; k < kAugMax; ++k)
      if (k < w.m)
        ((gptr_wd)pr.aug_slots)[(long)(kAugT + ((iter + 1) & 1) * kAugMax + k) * pr.n_slots_upd + t.slot] = tk[1 + k];
  }
}

// ------------------------------------------------- PCG run to a tolerance
// Start of a solve M x = b from x = 0: x = 0, r = b and the partials of
// rho_0 = b^T J^{-1} b.  One workgroup per producer slot of rho_0 (the forward
// transform's count), each over a contiguous float4 range.
__global__ __launch_bounds__(256) void k_solve_init(const ProbDev* P, const IoDev* IO, const Tile* tiles) {
  __shared__ double sh[4];
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const IoDev& io = IO[t.prob];
  const int n4 = pr.n_c / 4, ns = pr.n_slots_fdwt;
  const int chunk = (n4 + ns - 1) / ns;
  const int e0 = t.slot * chunk, e1 = min(e0 + chunk, n4);
  const float4* b = (const float4*)io.in;
  const float4* jv = (const float4*)pr.jinv;
  float4* x = (float4*)io.state;
  float4* r = (float4*)(io.state + 2L * pr.n_c);
  double acc = 0.0;
  for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
    const float4 v = b[e], j = jv[e];
    x[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    r[e] = v;
    acc += (double)v.x * (double)v.x * (double)j.x + (double)v.y * (double)v.y * (double)j.y +
           (double)v.z * (double)v.z * (double)j.z + (double)v.w * (double)v.w * (double)j.w;
  }
  const double s = block_sum(acc, sh, blockDim.x);
  if (threadIdx.x == 0) pr.dots[(long)rho_grp(0) * pr.n_dots + t.slot] = s;
}

// Coarse-level correction, per problem and block of kCoarseRows outputs:
// y = E^{-1} Z^T r on those outputs, stored at their coarse indices of zc,
// and the block's partial of (Z^T r)^T y into slot (k, block); r is r_k of
// the solve's state.  E^{-1} is symmetric, so output i sums column i, read
// along rows: lane = output (coalesced), the 4 waves split the rows and
// their partial sums are added in a fixed order.  Z^T r is gathered into
// LDS by every block.
__global__ __launch_bounds__(256) void k_coarse(const ProbDev* P, const IoDev* IO, const CoarseDev* C,
                                                const Tile* tiles, int k) {
  typedef const int __attribute__((address_space(1)))* gptr_i;
  __shared__ float rc[kCoarseMax];
  __shared__ float part[4][kCoarseRows];
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const CoarseDev& c = C[t.prob];
  const int m = c.m;
  const gptr_f r = (gptr_f)(IO[t.prob].state + 2L * pr.n_c);
  const gptr_i idx = (gptr_i)c.idx;
  for (int j = threadIdx.x; j < m; j += 256) rc[j] = r[idx[j]];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = t.ty * kCoarseRows + lane;
  const int ic = min(i, m - 1);  // lanes past the last output read a valid column
  const int per = (m + 3) / 4, j0 = wv * per, j1 = min(j0 + per, m);
  const gptr_f col = (gptr_f)(c.einv + ic);
  float acc = 0.f;
  int j = j0;
  for (; j + 8 <= j1; j += 8) {
    float e[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) e[u] = col[(long)(j + u) * m];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = fmaf(e[u], rc[j + u], acc);
  }
  for (; j < j1; ++j) acc = fmaf(col[(long)j * m], rc[j], acc);
  part[wv][lane] = acc;
  __syncthreads();
  if (wv == 0) {
    const float y = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
    double d = 0.0;
    if (i < m) {
      ((gptr_w)c.zc)[idx[i]] = y;
      d = (double)rc[i] * (double)y;
    }
    d = wave_sum(d);
    if (lane == 0) ((gptr_wd)c.slots)[(long)(k & (kDotRing - 1)) * c.n_slots + t.ty] = d;
  }
}

// Search direction of the coarse-corrected solve, over the vector-update
// chunks: p_k = J^{-1} r_k + zc + beta_k p_{k-1} (beta_0 = 0), with rho
// including the coarse part; the inverse transform then reads p_k (SRC_PJ).
__global__ __launch_bounds__(256) void k_coarse_p(const ProbDev* P, const IoDev* IO, const CoarseDev* C,
                                                  const Tile* tiles, int iter) {
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  float beta = 0.f;
  if (iter > 0) {
    int n0, n1;
    const CoarseDev& c = C[t.prob];
    const double* const sl[4] = {rho_slots(pr, iter, n0), coarse_slots(c, iter), rho_slots(pr, iter - 1, n1),
                                 coarse_slots(c, iter - 1)};
    const int nn[4] = {n0, c.n_slots, n1, c.n_slots};
    double o[4];
    wave_sum_slots_n<4>(sl, nn, o);
    const double rk = o[0] + o[1], rkm = o[2] + o[3];
    beta = (float)(rkm != 0.0 ? rk / rkm : 0.0);
  }
  const int e0 = t.ty * kUpdChunk, e1 = min(e0 + kUpdChunk, pr.n_c);
  const gptr_f r = (gptr_f)(IO[t.prob].state + 2L * pr.n_c);
  const gptr_f jv = (gptr_f)pr.jinv;
  const gptr_f zc = (gptr_f)C[t.prob].zc;
  const gptr_f pold = (gptr_f)p_loc(pr, iter - 1);
  const gptr_w pnew = (gptr_w)p_loc(pr, iter);
  for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
    const float z = fmaf(r[e], jv[e], zc[e]);
    pnew[e] = iter > 0 ? fmaf(beta, pold[e], z) : z;
  }
}

// Set-up of E = Z^T M Z, round t: every problem sets its unit vector to the
// column it probes in this round (and clears the previous round's).
__global__ void k_coarse_unit(const CoarseProbe* Q, int t) {
  const CoarseProbe& q = Q[blockIdx.x];
  if (threadIdx.x != 0) return;
  const int prev = (t - 1) * q.count + q.rank, col = t * q.count + q.rank;
  if (t > 0 && prev < q.m) ((gptr_w)q.in)[q.idx[prev]] = 0.f;
  if (col < q.m) ((gptr_w)q.in)[q.idx[col]] = 1.f;
}
// ... and stores Z^T M e_col as column col of its system's E.
__global__ void k_coarse_col(const CoarseProbe* Q, int t) {
  const CoarseProbe& q = Q[blockIdx.x];
  const int col = t * q.count + q.rank;
  if (col >= q.m) return;
  for (int i = threadIdx.x; i < q.m; i += blockDim.x) ((gptr_w)q.E)[(long)i * q.m + col] = q.out[q.idx[i]];
}

// ------------------------------------------------- parameter gradients
// Height term of one (sensor, layer) pair over a 16x16 corner tile:
//   sum_corners u(i, j) * d/dh [P_gl v](i, j)
// with u = Gamma^T C_hat^{-1} (...) in the corner-grid buffer and v = W^{-1} lambda
// (term 0) or W^{-1} c (term 1).  d/dh of the bilinear sample is
// dt_x/dh d/dt_x + dt_y/dh d/dt_y; on a grid line the derivative along that
// axis is the central difference (average of the one-sided ones).
__global__ __launch_bounds__(256) void k_grad_height(const ProbDev* P, const LayerDev* LD, const WfsDev* WD,
                                                     const Tile* tiles, int term) {
  __shared__ double sh[4];
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const WfsDev& w = WD[pr.wfs0 + t.item];
  const int l = t.level;
  const LayerDev& ly = LD[pr.layer0 + l];
  const float* v = (term == 0 ? pr.glam : pr.gphi) + ly.off;
  const int nc = w.nc, n = ly.n;
  const int i = t.ty * kTileS + (threadIdx.x >> 4), j = t.tx * kTileS + (threadIdx.x & 15);
  double acc = 0.0;
  if (i < nc && j < nc) {
    const int base = w.gtab_off + l * 4 * nc;
    const int* it = pr.gitab + base;
    const float* ft = pr.gftab + base;
    const int qy = it[i], qx = it[nc + j], tiey = it[2 * nc + i], tiex = it[3 * nc + j];
    const float wy = ft[i], wx = ft[nc + j], dty = ft[2 * nc + i], dtx = ft[3 * nc + j];
    // along x on row rr: slope (central on a grid line) and the sample value
    auto slope_x = [&](int rr) {
      const float* row = v + rr * n + qx;
      return tiex ? 0.5f * (row[1] - row[-1]) : row[1] - row[0];
    };
    auto value_x = [&](int rr) { return v[rr * n + qx] + wx * slope_x(rr); };
    float ddx, ddy;
    if (tiey) {
      ddx = slope_x(qy);
      ddy = 0.5f * (value_x(qy + 1) - value_x(qy - 1));
    } else {
      ddx = (1.f - wy) * slope_x(qy) + wy * slope_x(qy + 1);
      ddy = value_x(qy + 1) - value_x(qy);
    }
    const float d = dtx * ddx + dty * ddy;
    acc = (double)pr.vadj[w.v_off + i * nc + j] * (double)d;
  }
  const double s = block_sum(acc, sh, blockDim.x);
  if (threadIdx.x == 0) pr.gslots[pr.n_gp + term * pr.n_gh + t.slot] = s;
}

// Prior term of one layer over a chunk of coefficients: sum lambda_e D_e c_e.
__global__ __launch_bounds__(256) void k_grad_prior(const ProbDev* P, const LayerDev* LD, const GradIo* GIO,
                                                    const Tile* tiles) {
  __shared__ double sh[4];
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[pr.layer0 + t.item];
  const GradIo& g = GIO[t.prob];
  const int n = ly.n, nn = n * n;
  const int m0 = n >> ly.levels, jmin = ly.log2n - ly.levels;
  const int e0 = t.ty * kGradChunk, e1 = min(e0 + kGradChunk, nn);
  double acc = 0.0;
  for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
    const int r = e >> ly.log2n, c = e & (n - 1), mx = max(r, c);
    const int j = (mx < m0) ? jmin : 31 - __clz(mx);
    acc += (double)g.lam[ly.off + e] * (double)g.c[ly.off + e] * ly.d64[j];
  }
  const double s = block_sum(acc, sh, blockDim.x);
  if (threadIdx.x == 0) pr.gslots[ly.gp_off + t.ty] = s;
}

// One wave per problem: fixed-order sums of the slots into
//   g_alpha = -sum_l t_l,  g_gamma_l = alpha t_l / gamma_l,  g_h_l = term0_l - term1_l
// with t_l = lambda_l^T D_l c_l.
__global__ __launch_bounds__(64) void k_grad_final(const ProbDev* P, const LayerDev* LD, const GradIo* GIO) {
  const ProbDev& pr = P[blockIdx.x];
  const GradIo& g = GIO[blockIdx.x];
  double ta = 0.0;
  for (int l = 0; l < pr.L; ++l) {
    const LayerDev& ly = LD[pr.layer0 + l];
    const double tl = wave_sum_slots(pr.gslots + ly.gp_off, ly.gp_n);
    const double h0 = wave_sum_slots(pr.gslots + pr.n_gp + ly.gh_off, ly.gh_n);
    const double h1 = wave_sum_slots(pr.gslots + pr.n_gp + pr.n_gh + ly.gh_off, ly.gh_n);
    ta += tl;
    if (threadIdx.x == 0) {
      g.out[1 + l] = pr.alpha * tl / ly.cn2;
      g.out[1 + pr.L + l] = h0 - h1;
    }
  }
  if (threadIdx.x == 0) g.out[0] = -ta;
}

// ------------------------------------------------------------ DM fitting
// Wavefront of a set of grids (layers of the reconstruction, or DMs) at the
// fitting-pupil corners in one direction, bilinear, masked to the pupil:
//   u_k = M sum_grid grid(x + h theta_k).   Tile = 16x16 corners.
__global__ __launch_bounds__(256) void k_fit_fwd(const ProbDev* P, const LayerDev* LD, const WfsDev* WD,
                                                 const Tile* tiles) {
  const Tile t = my_tile(tiles);
  const ProbDev& pr = P[t.prob];
  const WfsDev& w = WD[pr.wfs0 + t.item];
  const int nc = w.nc;
  const int i = t.ty * kTileS + (threadIdx.x >> 4), j = t.tx * kTileS + (threadIdx.x & 15);
  if (i >= nc || j >= nc) return;
  float v = 0.f;
  if (pr.cmap[w.m_off + i * nc + j] >= 0) {
    for (int l = 0; l < pr.L; ++l) {
      const LayerDev& ly = LD[pr.layer0 + l];
      const int base = w.tab_off + l * w.tab_stride;
      const int qy = pr.itab[base + i], qx = pr.itab[base + nc + j];
      const float wy = pr.ftab[base + 2 * nc + i], wx = pr.ftab[base + 3 * nc + j];
      const float* ph = pr.phi + ly.off + qy * ly.n + qx;
      const float top = (1.f - wx) * ph[0] + wx * ph[1];
      const float bot = (1.f - wx) * ph[ly.n] + wx * ph[ly.n + 1];
      v += (1.f - wy) * top + wy * bot;
    }
  }
  pr.vadj[w.v_off + i * nc + j] = v;
}

// CG on the fitting normal equations, one workgroup per fitted problem; the
// operator's data part sum_k B_k^T M B_k p arrives in adj (FIT_ITER), the
// right-hand side sum_k B_k^T M P_k phi in adj (FIT_INIT).  FP64 inner
// products, fixed-order block sums.  FIT_FINAL applies the open-loop control
// of Algorithm 1 with the fitted commands.
__global__ __launch_bounds__(1024) void k_fit_cg(const FitDev* F, const ProbDev* P, const IoDev* IO, int phase) {
  __shared__ double sh[16];
  __shared__ double s_val;
  const FitDev& f = F[blockIdx.x];
  const int n = f.n_act, nt = blockDim.x;
  if (phase == FIT_INIT) {
    double acc = 0.0;
    for (int e = threadIdx.x; e < n; e += nt) {
      const float b = f.adj[e];
      f.x[e] = 0.f;
      f.r[e] = b;
      f.p[e] = b;
      acc += (double)b * (double)b;
    }
    const double rho = block_sum(acc, sh, nt);
    if (threadIdx.x == 0) f.scal[0] = rho;
    return;
  }
  if (phase == FIT_ITER) {
    double acc = 0.0;
    for (int e = threadIdx.x; e < n; e += nt) {
      const float q = f.adj[e] + f.eps * f.p[e];
      acc += (double)f.p[e] * (double)q;
    }
    const double pi = block_sum(acc, sh, nt);
    if (threadIdx.x == 0) s_val = pi;
    __syncthreads();
    const double rho = f.scal[0];
    const float al = (float)((s_val > 0.0) ? rho / s_val : 0.0);
    if (threadIdx.x == 0 && ((!(s_val > 0.0) && rho != 0.0) || !(rho >= 0.0)))
      __hip_atomic_store(f.numflag, f.main + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    acc = 0.0;
    for (int e = threadIdx.x; e < n; e += nt) {
      const float pe = f.p[e];
      const float q = f.adj[e] + f.eps * pe;
      f.x[e] = fmaf(al, pe, f.x[e]);
      const float re = fmaf(-al, q, f.r[e]);
      f.r[e] = re;
      acc += (double)re * (double)re;
    }
    const double rho2 = block_sum(acc, sh, nt);
    if (threadIdx.x == 0) s_val = rho2;
    __syncthreads();
    const float be = (float)((rho > 0.0) ? s_val / rho : 0.0);
    for (int e = threadIdx.x; e < n; e += nt) f.p[e] = fmaf(be, f.p[e], f.r[e]);
    __syncthreads();
    if (threadIdx.x == 0) f.scal[0] = s_val;
    return;
  }
  // FIT_FINAL
  const ProbDev& pr = P[f.main];
  const IoDev& io = IO[f.main];
  float* aprev = io.state + 3L * pr.n_c;
  float* a = aprev + pr.n_act;
  for (int e = threadIdx.x; e < n; e += nt) {
    const float old = a[e];
    const float nw = (1.0f - f.gain) * old + f.gain * f.x[e];
    aprev[e] = old;
    a[e] = nw;
    if (io.dm_out) io.dm_out[e] = nw;
  }
}

// ------------------------------------------------------------ launchers

// The resident kernels are instantiated for LDS capacities 32, 64 and 128 and
// launched with the smallest that holds the plan's resident side.
void launch_idwt_res(const LaunchArgs& a, const Tile* tiles, int ntiles, int src_mode, int out_mode, int iter) {
  if (ntiles <= 0) return;
  if (a.res_max <= 32)
    k_idwt_res<32><<<ntiles, 1024, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, src_mode, out_mode, iter);
  else if (a.res_max <= 64)
    k_idwt_res<64><<<ntiles, 1024, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, src_mode, out_mode, iter);
  else
    k_idwt_res<128><<<ntiles, 1024, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, src_mode, out_mode, iter);
}
void launch_idwt_res4(const LaunchArgs& a, const Tile* tiles, int ntiles, int src_mode, int out_mode, int iter) {
  if (ntiles <= 0) return;
  if (a.res_max <= 32)
    k_idwt_res4<32><<<ntiles, 512, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, src_mode, out_mode, iter);
  else if (a.res_max <= 64)
    k_idwt_res4<64><<<ntiles, 512, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, src_mode, out_mode, iter);
  else
    k_idwt_res4<128><<<ntiles, 512, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, src_mode, out_mode, iter);
}
void launch_idwt_glob(const LaunchArgs& a, const Tile* tiles, int ntiles, int src_mode, int out_mode, int iter,
                      int step) {
  if (ntiles <= 0) return;
  if (a.glob_fuse)
    k_idwt_glob2<<<ntiles, 256, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, src_mode, out_mode, iter, step);
  else
    k_idwt_glob<<<ntiles, 256, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, src_mode, out_mode, iter, step);
}
void launch_fdwt_glob(const LaunchArgs& a, const Tile* tiles, int ntiles, int epi, int iter, int step) {
  if (ntiles <= 0) return;
  if (a.glob_fuse)
    k_fdwt_glob2<<<ntiles, 256, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, epi, iter, step);
  else
    k_fdwt_glob<<<ntiles, 256, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, epi, iter, step);
}
template <int RMAX>
static void launch_fdwt_res_r(const LaunchArgs& a, const Tile* tiles, int ntiles, int epi, int iter) {
  switch (epi) {
    case EPI_APPLYM: k_fdwt_res<RMAX, EPI_APPLYM><<<ntiles, 1024, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, iter); break;
    case EPI_PCG: k_fdwt_res<RMAX, EPI_PCG><<<ntiles, 1024, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, iter); break;
    case EPI_RHS: k_fdwt_res<RMAX, EPI_RHS><<<ntiles, 1024, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, iter); break;
    case EPI_RHSQ: k_fdwt_res<RMAX, EPI_RHSQ><<<ntiles, 1024, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, iter); break;
    default: k_fdwt_res<RMAX, EPI_PLAIN><<<ntiles, 1024, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, iter); break;
  }
}
void launch_fdwt_res(const LaunchArgs& a, const Tile* tiles, int ntiles, int epi, int iter) {
  if (ntiles <= 0) return;
  if (a.res_max <= 32)
    launch_fdwt_res_r<32>(a, tiles, ntiles, epi, iter);
  else if (a.res_max <= 64)
    launch_fdwt_res_r<64>(a, tiles, ntiles, epi, iter);
  else
    launch_fdwt_res_r<128>(a, tiles, ntiles, epi, iter);
}
void launch_pgamma(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode) {
  if (ntiles <= 0) return;
#define FEWHA_PG(M) k_pgamma<M><<<ntiles, kSensThreads, 0, a.stream>>>(a.P, a.L, a.W, a.IO, tiles, a.pgrows)
  switch (mode) {
    case PG_COMPACT: FEWHA_PG(PG_COMPACT); break;
    case PG_DENSE: FEWHA_PG(PG_DENSE); break;
    case PG_DENSE_IN: FEWHA_PG(PG_DENSE_IN); break;
    case PG_RESID_IN: FEWHA_PG(PG_RESID_IN); break;
    case PG_POL_IN: FEWHA_PG(PG_POL_IN); break;
    default: FEWHA_PG(PG_APREV); break;
  }
#undef FEWHA_PG
}
void launch_slopes_in(const LaunchArgs& a, const Tile* tiles, int ntiles, int add) {
  if (ntiles <= 0) return;
  if (add)
    k_slopes_in<1><<<ntiles, 256, 0, a.stream>>>(a.P, a.W, a.IO, tiles);
  else
    k_slopes_in<0><<<ntiles, 256, 0, a.stream>>>(a.P, a.W, a.IO, tiles);
}
void launch_gammaT(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode) {
  if (ntiles > 0) k_gammaT<<<ntiles, 256, 0, a.stream>>>(a.P, a.W, tiles, a.gtrows, mode);
}
void launch_pT(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode) {
  if (ntiles <= 0) return;
#define FEWHA_PT(RPT, WIDE, SPLIT)                                                                      \
  k_pT<RPT, WIDE, SPLIT><<<ntiles, 256, 0, a.stream>>>(a.P, a.L, a.W, a.IO, tiles, a.hats, a.n_hats, a.bands, \
                                                       a.pents, mode)
  if (a.pt_split) {
    if (a.pt_wide)
      FEWHA_PT(4, true, true);
    else
      FEWHA_PT(4, false, true);
  } else if (a.pt_wide) {
    if (a.pt_rows == 8)
      FEWHA_PT(8, true, false);
    else
      FEWHA_PT(4, true, false);
  } else if (a.pt_rows == 8) {
    FEWHA_PT(8, false, false);
  } else {
    FEWHA_PT(4, false, false);
  }
#undef FEWHA_PT
}
void launch_update(const LaunchArgs& a, const Tile* tiles, int ntiles, int iter, const CoarseDev* C, int xm) {
  if (ntiles <= 0) return;
  if (xm == UPD_X_DEFER)
    k_update<UPD_X_DEFER><<<ntiles, 256, 0, a.stream>>>(a.P, a.IO, tiles, iter, C);
  else if (xm == UPD_X_PAIR)
    k_update<UPD_X_PAIR><<<ntiles, 256, 0, a.stream>>>(a.P, a.IO, tiles, iter, C);
  else
    k_update<UPD_X_ONE><<<ntiles, 256, 0, a.stream>>>(a.P, a.IO, tiles, iter, C);
}
void launch_coarse(const LaunchArgs& a, const CoarseDev* C, const Tile* tiles, int ntiles, int k) {
  if (ntiles > 0) k_coarse<<<ntiles, 256, 0, a.stream>>>(a.P, a.IO, C, tiles, k);
}
void launch_coarse_p(const LaunchArgs& a, const CoarseDev* C, const Tile* tiles, int ntiles, int iter) {
  if (ntiles > 0) k_coarse_p<<<ntiles, 256, 0, a.stream>>>(a.P, a.IO, C, tiles, iter);
}
void launch_coarse_probe(const CoarseProbe* Q, int nprob, int t, bool store, hipStream_t s) {
  if (nprob <= 0) return;
  if (store)
    k_coarse_col<<<nprob, 256, 0, s>>>(Q, t);
  else
    k_coarse_unit<<<nprob, 64, 0, s>>>(Q, t);
}
void launch_solve_init(const LaunchArgs& a, const Tile* tiles, int ntiles) {
  if (ntiles > 0) k_solve_init<<<ntiles, 256, 0, a.stream>>>(a.P, a.IO, tiles);
}
void launch_grad_height(const LaunchArgs& a, const Tile* tiles, int ntiles, int term) {
  if (ntiles > 0) k_grad_height<<<ntiles, 256, 0, a.stream>>>(a.P, a.L, a.W, tiles, term);
}
void launch_grad_prior(const LaunchArgs& a, const GradIo* g, const Tile* tiles, int ntiles) {
  if (ntiles > 0) k_grad_prior<<<ntiles, 256, 0, a.stream>>>(a.P, a.L, g, tiles);
}
void launch_grad_final(const LaunchArgs& a, const GradIo* g, int nprob) {
  if (nprob > 0) k_grad_final<<<nprob, 64, 0, a.stream>>>(a.P, a.L, g);
}
void launch_aug_gram(const LaunchArgs& a, const Tile* tiles, int ntiles) {
  if (ntiles > 0) k_aug_gram<<<ntiles, 256, 0, a.stream>>>(a.P, a.IO, tiles);
}
void launch_aug_init(const LaunchArgs& a, const Tile* tiles, int ntiles) {
  if (ntiles > 0) k_aug_init<<<ntiles, 256, 0, a.stream>>>(a.P, a.IO, tiles);
}
void launch_aug_p(const LaunchArgs& a, const Tile* tiles, int ntiles, int iter) {
  if (ntiles > 0) k_aug_p<<<ntiles, 256, 0, a.stream>>>(a.P, a.IO, tiles, iter);
}
void launch_aug_store(const LaunchArgs& a, const Tile* tiles, int ntiles, int iters) {
  if (ntiles > 0) k_aug_store<<<ntiles, 256, 0, a.stream>>>(a.P, a.IO, tiles, iters);
}
void launch_fit_fwd(const LaunchArgs& a, const Tile* tiles, int ntiles) {
  if (ntiles > 0) k_fit_fwd<<<ntiles, 256, 0, a.stream>>>(a.P, a.L, a.W, tiles);
}
void launch_fit_cg(const LaunchArgs& a, const FitDev* F, int nfit, int phase) {
  if (nfit > 0) k_fit_cg<<<nfit, 1024, 0, a.stream>>>(F, a.P, a.IO, phase);
}

}  // namespace fewha
