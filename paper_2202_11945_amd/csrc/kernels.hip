// gfx950 kernels of the FEWHA hot path.  Every kernel walks a work list of
// tiles spanning all problems of a plan, so one launch serves one stage of a
// whole batch.  Bulk arithmetic is FP32; PCG inner products are accumulated
// in FP64 per workgroup and summed across workgroups in a fixed order
// (deterministic: no atomics anywhere).
#include "kernels.h"

namespace fewha {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
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

__device__ __forceinline__ double sum_slots(const double* s, int n) {
  double a = 0.0;
  for (int i = 0; i < n; ++i) a += s[i];
  return a;
}

__device__ __forceinline__ const double* dot_group(const ProbDev& pr, int g) {
  return pr.dots + (long)g * pr.n_dots;
}
__device__ __forceinline__ int rho_count(const ProbDev& pr, int k) {
  return k == 0 ? pr.n_slots_fdwt : pr.n_slots_upd;
}

// Search-direction source of the inverse transform (fused p update).
struct PSrc {
  const float* src;   // plain source (SRC_IN / SRC_STATE_C)
  const float* r;
  const float* jinv;
  const float* pold;
  float* pnew;
  float beta;
  int mode;
};

__device__ __forceinline__ PSrc make_psrc(const ProbDev& pr, const IoDev& io, int mode, int iter,
                                          const double* sbeta) {
  PSrc s;
  s.mode = mode;
  s.src = (mode == SRC_IN) ? io.in : io.state;  // state starts with c
  s.r = io.state + 2L * pr.n_c;
  s.jinv = pr.jinv;
  s.pnew = (iter & 1) ? pr.pbuf1 : pr.pbuf0;
  s.pold = (iter & 1) ? pr.pbuf0 : pr.pbuf1;
  s.beta = (float)(*sbeta);
  return s;
}

__device__ __forceinline__ float load_coef(const PSrc& s, int e, bool owner) {
  if (s.mode == SRC_IN || s.mode == SRC_STATE_C) return s.src[e];
  const float z = s.r[e] * s.jinv[e];
  const float p = (s.mode == SRC_PUPD0) ? z : fmaf(s.beta, s.pold[e], z);
  if (owner) s.pnew[e] = p;
  return p;
}

// beta_k = rho_k / rho_{k-1} (computed by thread 0, broadcast through LDS)
__device__ __forceinline__ void compute_beta(const ProbDev& pr, int mode, int iter, double* sbeta) {
  if (threadIdx.x == 0) {
    double b = 0.0;
    if (mode == SRC_PUPD) {
      const double rk = sum_slots(dot_group(pr, 2 * iter), rho_count(pr, iter));
      const double rkm = sum_slots(dot_group(pr, 2 * (iter - 1)), rho_count(pr, iter - 1));
      b = (rkm != 0.0) ? rk / rkm : 0.0;
    }
    *sbeta = b;
  }
  __syncthreads();
}

// Final output of the inverse transform: phi = delta^{-1} W^T c, optionally
// with the open-loop control update of Algorithm 1 (F = I).
__device__ __forceinline__ void idwt_out(const ProbDev& pr, const IoDev& io, int out_mode, int e, float v) {
  if (out_mode == OUT_PHI) {
    pr.phi[e] = v;
  } else if (out_mode == OUT_USER) {
    io.out[e] = v;
  } else {  // OUT_FIT
    if (io.layers_out) io.layers_out[e] = v;
    float* aprev = io.state + 3L * pr.n_c;
    float* a = aprev + pr.n_act;
    const float old = a[e];
    const float nw = (1.0f - pr.gain) * old + pr.gain * v;
    aprev[e] = old;
    a[e] = nw;
    if (io.dm_out) io.dm_out[e] = nw;
  }
}

// ------------------------------------------------ inverse DWT, resident part
// One workgroup per (problem, layer): all synthesis levels whose output side
// is at most kResMax run in LDS.  Columns then rows, periodic, Mallat layout.
__global__ __launch_bounds__(1024) void k_idwt_res(const ProbDev* P, const LayerDev* LD, const IoDev* IO,
                                                   const Tile* tiles, Filter F, int src_mode, int out_mode,
                                                   int iter) {
  __shared__ float A[kResMax * kResMax];
  __shared__ float B[kResMax * kResMax];
  __shared__ double sbeta;
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[pr.layer0 + t.item];
  const IoDev& io = IO[t.prob];
  compute_beta(pr, src_mode, iter, &sbeta);
  const PSrc ps = make_psrc(pr, io, src_mode, iter, &sbeta);
  const int n = ly.n, R = ly.res, lr = __builtin_ctz(R);
  const int m0 = n >> ly.levels;
  const int off = ly.off;
  const int nt = blockDim.x;
  for (int e = threadIdx.x; e < m0 * m0; e += nt) {
    const int r = e / m0, c = e - r * m0;
    A[(r << lr) + c] = load_coef(ps, off + r * n + c, true);
  }
  __syncthreads();
  for (int m = 2 * m0; m <= R; m <<= 1) {
    const int half = m >> 1, lm = __builtin_ctz(m);
    for (int e = threadIdx.x; e < m * m; e += nt) {
      const int r = e >> lm, c = e & (m - 1);
      if (r < half && c < half) continue;
      A[(r << lr) + c] = load_coef(ps, off + r * n + c, true);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m * m; e += nt) {  // columns (along y)
      const int tt = e >> lm, c = e & (m - 1);
      const int par = tt & 1, k0 = (tt - par) >> 1;
      const int ka = k0 & (half - 1), kb = (k0 - 1) & (half - 1), kc = (k0 - 2) & (half - 1);
      const float acc = F.h[par] * A[(ka << lr) + c] + F.h[par + 2] * A[(kb << lr) + c] +
                        F.h[par + 4] * A[(kc << lr) + c] + F.g[par] * A[((half + ka) << lr) + c] +
                        F.g[par + 2] * A[((half + kb) << lr) + c] + F.g[par + 4] * A[((half + kc) << lr) + c];
      B[(tt << lr) + c] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m * m; e += nt) {  // rows (along x)
      const int r = e >> lm, tt = e & (m - 1);
      const int par = tt & 1, k0 = (tt - par) >> 1;
      const int ka = k0 & (half - 1), kb = (k0 - 1) & (half - 1), kc = (k0 - 2) & (half - 1);
      const float* Br = B + (r << lr);
      const float acc = F.h[par] * Br[ka] + F.h[par + 2] * Br[kb] + F.h[par + 4] * Br[kc] +
                        F.g[par] * Br[half + ka] + F.g[par + 2] * Br[half + kb] + F.g[par + 4] * Br[half + kc];
      A[(r << lr) + tt] = acc;
    }
    __syncthreads();
  }
  if (n == R) {
    for (int e = threadIdx.x; e < R * R; e += nt) {
      const int r = e >> lr, c = e & (R - 1);
      idwt_out(pr, io, out_mode, off + r * n + c, A[e] * ly.inv_delta);
    }
  } else {
    float* dst = pr.tmpa + ly.tmp_off;
    for (int e = threadIdx.x; e < R * R; e += nt) dst[e] = A[e];
  }
}

// ----------------------------------------------- inverse DWT, one global level
// Output tile 32x32 of the level with side m = 2^t.level (> kResMax).  The
// coarse block comes from scratch, the three detail quadrants from the
// coefficient source; 2 halo coefficients per direction (6 taps, 3 per phase).
constexpr int kGT = 32;           // output tile side
constexpr int kGH = kGT / 2 + 2;  // coefficients per band and direction (18)
constexpr int kGW = 2 * kGH;      // 36

__global__ __launch_bounds__(256) void k_idwt_glob(const ProbDev* P, const LayerDev* LD, const IoDev* IO,
                                                   const Tile* tiles, Filter F, int src_mode, int out_mode,
                                                   int iter, int step) {
  __shared__ float A[kGW * (kGW + 1)];
  __shared__ float B[kGT * (kGW + 1)];
  __shared__ double sbeta;
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[pr.layer0 + t.item];
  const IoDev& io = IO[t.prob];
  compute_beta(pr, src_mode, iter, &sbeta);
  const PSrc ps = make_psrc(pr, io, src_mode, iter, &sbeta);
  const int n = ly.n, off = ly.off;
  const int m = 1 << t.level, half = m >> 1;
  const int t0 = t.ty * kGT, s0 = t.tx * kGT;
  const float* ll = ((step & 1) ? pr.tmpb : pr.tmpa) + ly.tmp_off;  // stride half
  float* nxt = ((step & 1) ? pr.tmpa : pr.tmpb) + ly.tmp_off;       // stride m
  const int kr0 = (t0 >> 1) - 2, kc0 = (s0 >> 1) - 2;
  const int W1 = kGW + 1;
  for (int e = threadIdx.x; e < kGW * kGW; e += blockDim.x) {
    const int ly_ = e / kGW, lx_ = e - ly_ * kGW;
    const int by = ly_ >= kGH, bx = lx_ >= kGH;
    const int iy = ly_ - by * kGH, ix = lx_ - bx * kGH;
    const int kr = (kr0 + iy) & (half - 1), kc = (kc0 + ix) & (half - 1);
    float v;
    if (!by && !bx) {
      v = ll[kr * half + kc];
    } else {
      const bool owner = iy >= 2 && ix >= 2;
      v = load_coef(ps, off + (by * half + kr) * n + (bx * half + kc), owner);
    }
    A[ly_ * W1 + lx_] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kGT * kGW; e += blockDim.x) {  // columns
    const int lt = e / kGW, lx_ = e - lt * kGW;
    const int par = lt & 1, k = ((lt - par) >> 1) + 2;
    const float acc = F.h[par] * A[k * W1 + lx_] + F.h[par + 2] * A[(k - 1) * W1 + lx_] +
                      F.h[par + 4] * A[(k - 2) * W1 + lx_] + F.g[par] * A[(kGH + k) * W1 + lx_] +
                      F.g[par + 2] * A[(kGH + k - 1) * W1 + lx_] + F.g[par + 4] * A[(kGH + k - 2) * W1 + lx_];
    B[lt * W1 + lx_] = acc;
  }
  __syncthreads();
  const bool final_level = (m == n);
  for (int e = threadIdx.x; e < kGT * kGT; e += blockDim.x) {  // rows
    const int lt = e >> 5, ls = e & 31;
    const int par = ls & 1, k = ((ls - par) >> 1) + 2;
    const float* Br = B + lt * W1;
    const float acc = F.h[par] * Br[k] + F.h[par + 2] * Br[k - 1] + F.h[par + 4] * Br[k - 2] +
                      F.g[par] * Br[kGH + k] + F.g[par + 2] * Br[kGH + k - 1] + F.g[par + 4] * Br[kGH + k - 2];
    const int row = t0 + lt, col = s0 + ls;
    if (final_level)
      idwt_out(pr, io, out_mode, off + row * n + col, acc * ly.inv_delta);
    else
      nxt[row * m + col] = acc;
  }
}

// --------------------------------------------------- forward DWT epilogue
// value v = delta^{-1} (W x)_e at layer position e with level index j.
__device__ __forceinline__ void fdwt_out(const ProbDev& pr, const LayerDev& ly, const IoDev& io, int epi, int iter,
                                         int e, int j, float v, double& acc) {
  const float ad = ly.alpha_d[j];
  if (epi == EPI_APPLYM) {
    io.out[e] = v + ad * io.in[e];
  } else if (epi == EPI_PCG) {
    const float* p = (iter & 1) ? pr.pbuf1 : pr.pbuf0;
    const float pe = p[e];
    const float qe = v + ad * pe;
    pr.q[e] = qe;
    acc += (double)pe * (double)qe;
  } else if (epi == EPI_RHS) {
    float* b = io.state + pr.n_c;
    float* r = io.state + 2L * pr.n_c;
    const float r0 = (v - b[e]) + r[e];
    b[e] = v;
    r[e] = r0;
    acc += (double)r0 * (double)r0 * (double)pr.jinv[e];
  } else {  // EPI_PLAIN
    io.out[e] = v;
  }
}

__device__ __forceinline__ int dot_group_of(int epi, int iter) {
  return epi == EPI_PCG ? 2 * iter + 1 : 0;
}

// ------------------------------------------------ forward DWT, one global level
// Input side m = 2^t.level (> kResMax); output 16x16 coefficients of each of
// the four quadrants per tile; input window 36x36 (2k .. 2k+5 per output).
constexpr int kFT = 16;             // output coefficients per direction
constexpr int kFW = 2 * kFT + 4;    // 36 input samples per direction

__global__ __launch_bounds__(256) void k_fdwt_glob(const ProbDev* P, const LayerDev* LD, const IoDev* IO,
                                                   const Tile* tiles, Filter F, int epi, int iter, int step) {
  __shared__ float X[kFW * (kFW + 1)];
  __shared__ float Rw[kFW * (2 * kFT + 1)];
  __shared__ double sh[4];
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[pr.layer0 + t.item];
  const IoDev& io = IO[t.prob];
  const int n = ly.n, off = ly.off;
  const int m = 1 << t.level, half = m >> 1;
  const float* in = (step == 0) ? pr.phiadj + off : (((step & 1) ? pr.tmpa : pr.tmpb) + ly.tmp_off);
  float* llout = ((step & 1) ? pr.tmpb : pr.tmpa) + ly.tmp_off;  // stride half
  const int k0 = t.ty * kFT, l0 = t.tx * kFT;
  const int XW = kFW + 1, RW = 2 * kFT + 1;
  for (int e = threadIdx.x; e < kFW * kFW; e += blockDim.x) {
    const int ry = e / kFW, rx = e - ry * kFW;
    const int gy = (2 * k0 + ry) & (m - 1), gx = (2 * l0 + rx) & (m - 1);
    X[ry * XW + rx] = in[gy * (step == 0 ? n : m) + gx];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kFW * kFT; e += blockDim.x) {  // rows (along x)
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
  const int j = t.level - 1;  // detail blocks of this level have side half = 2^j
  for (int e = threadIdx.x; e < kFT * 2 * kFT; e += blockDim.x) {  // columns (along y)
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
    if (!xd) {
      llout[row * half + col] = a;  // coarse block for the next level
    } else {
      fdwt_out(pr, ly, io, epi, iter, off + row * n + (half + col), j, a * ly.inv_delta, acc);
    }
    fdwt_out(pr, ly, io, epi, iter, off + (half + row) * n + (xd * half + col), j, d * ly.inv_delta, acc);
  }
  if (epi == EPI_PCG || epi == EPI_RHS) {
    const double s = block_sum(acc, sh, blockDim.x);
    if (threadIdx.x == 0) pr.dots[(long)dot_group_of(epi, iter) * pr.n_dots + t.slot] = s;
  }
}

// ------------------------------------------------ forward DWT, resident part
__global__ __launch_bounds__(1024) void k_fdwt_res(const ProbDev* P, const LayerDev* LD, const IoDev* IO,
                                                   const Tile* tiles, Filter F, int epi, int iter) {
  __shared__ float A[kResMax * kResMax];
  __shared__ float B[kResMax * kResMax];
  __shared__ double sh[16];
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[pr.layer0 + t.item];
  const IoDev& io = IO[t.prob];
  const int n = ly.n, R = ly.res, lr = __builtin_ctz(R), off = ly.off;
  const int nt = blockDim.x;
  const int ng = ly.n_glob_levels;
  const float* in = (ng == 0) ? pr.phiadj + off : ((((ng - 1) & 1) ? pr.tmpb : pr.tmpa) + ly.tmp_off);
  const int istride = (ng == 0) ? n : R;
  for (int e = threadIdx.x; e < R * R; e += nt) {
    const int r = e >> lr, c = e & (R - 1);
    A[e] = in[r * istride + c];
  }
  __syncthreads();
  double acc = 0.0;
  const int m0 = n >> ly.levels;
  for (int m = R; m > m0; m >>= 1) {
    const int half = m >> 1, lm = __builtin_ctz(m), lh = lm - 1;
    for (int e = threadIdx.x; e < m * half; e += nt) {  // rows: A -> B
      const int r = e >> lh, k = e & (half - 1);
      const float* Ar = A + (r << lr);
      float a = 0.f, d = 0.f;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const float v = Ar[(2 * k + i) & (m - 1)];
        a += F.h[i] * v;
        d += F.g[i] * v;
      }
      B[(r << lr) + k] = a;
      B[(r << lr) + half + k] = d;
    }
    __syncthreads();
    const int j = lm - 1;
    for (int e = threadIdx.x; e < half * m; e += nt) {  // columns: B -> A
      const int k = e >> lm, c = e & (m - 1);
      float a = 0.f, d = 0.f;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const float v = B[(((2 * k + i) & (m - 1)) << lr) + c];
        a += F.h[i] * v;
        d += F.g[i] * v;
      }
      if (c >= half) fdwt_out(pr, ly, io, epi, iter, off + k * n + c, j, a * ly.inv_delta, acc);
      fdwt_out(pr, ly, io, epi, iter, off + (half + k) * n + c, j, d * ly.inv_delta, acc);
      A[(k << lr) + c] = a;  // rows >= half of A are no longer read
    }
    __syncthreads();
  }
  const int jll = __builtin_ctz(m0);
  for (int e = threadIdx.x; e < m0 * m0; e += nt) {
    const int r = e / m0, c = e - r * m0;
    fdwt_out(pr, ly, io, epi, iter, off + r * n + c, jll, A[(r << lr) + c] * ly.inv_delta, acc);
  }
  if (epi == EPI_PCG || epi == EPI_RHS) {
    const double s = block_sum(acc, sh, nt);
    if (threadIdx.x == 0) pr.dots[(long)dot_group_of(epi, iter) * pr.n_dots + t.slot] = s;
  }
}

// ------------------------------------------- propagation + Shack-Hartmann
// Tile of 16x16 subapertures of one sensor: v on the 17x17 corners is the
// sum over layers of the bilinear interpolant (LGS cone factor in the
// tables), then s^x, s^y per active subaperture (Sec. 2).
__global__ __launch_bounds__(256) void k_pgamma(const ProbDev* P, const LayerDev* LD, const WfsDev* WD,
                                                const IoDev* IO, const Tile* tiles, int mode) {
  __shared__ float V[(kTileS + 1) * (kTileS + 1)];
  __shared__ float sh[4 * 4];
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const WfsDev& w = WD[pr.wfs0 + t.item];
  const IoDev& io = IO[t.prob];
  const float* phi = (mode == PG_COMPACT) ? io.in : pr.phi;
  const int N = w.N, nc = w.nc;
  const int i0 = t.ty * kTileS, j0 = t.tx * kTileS;
  constexpr int CW = kTileS + 1;
  for (int e = threadIdx.x; e < CW * CW; e += blockDim.x) {
    const int li = e / CW, lj = e - li * CW;
    const int i = i0 + li, j = j0 + lj;
    float v = 0.f;
    if (i < nc && j < nc) {
      for (int l = 0; l < pr.L; ++l) {
        const LayerDev& ly = LD[pr.layer0 + l];
        const int base = w.tab_off + l * w.tab_stride;
        const int* it = pr.itab + base;
        const float* ft = pr.ftab + base;
        const int qy = it[i], qx = it[nc + j];
        const float wy = ft[2 * nc + i], wx = ft[3 * nc + j];
        const float* ph = phi + ly.off + qy * ly.n + qx;
        const float top = (1.f - wx) * ph[0] + wx * ph[1];
        const float bot = (1.f - wx) * ph[ly.n] + wx * ph[ly.n + 1];
        v += (1.f - wy) * top + wy * bot;
      }
    }
    V[e] = v;
  }
  __syncthreads();
  const int li = threadIdx.x >> 4, lj = threadIdx.x & 15;
  const int i = i0 + li, j = j0 + lj;
  float sx = 0.f, sy = 0.f, cx = 0.f, cy = 0.f;
  bool act = false;
  int ci = -1;
  if (i < N && j < N) {
    ci = pr.cmap[w.m_off + i * N + j];
    act = ci >= 0;
  }
  if (act) {
    const float v00 = V[li * CW + lj], v01 = V[li * CW + lj + 1];
    const float v10 = V[(li + 1) * CW + lj], v11 = V[(li + 1) * CW + lj + 1];
    sx = 0.5f * ((v01 - v00) + (v11 - v10));
    sy = 0.5f * ((v10 - v00) + (v11 - v01));
    if (w.blocks) {
      const float* cb = pr.cinv + w.cinv_off + 3 * (i * N + j);
      cx = cb[0] * sx + cb[1] * sy;
      cy = cb[1] * sx + cb[2] * sy;
    }
  }
  if (mode == PG_COMPACT) {
    if (act) {
      io.out[w.cs_off + ci] = sx;
      io.out[w.cs_off + w.n_active + ci] = sy;
    }
    return;
  }
  if (i < N && j < N) {
    pr.sd[w.s_off + i * N + j] = sx;
    pr.sd[w.s_off + N * N + i * N + j] = sy;
  }
  const float a0 = block_sum(sx, sh, blockDim.x);
  const float a1 = block_sum(sy, sh + 4, blockDim.x);
  const float a2 = block_sum(cx, sh + 8, blockDim.x);
  const float a3 = block_sum(cy, sh + 12, blockDim.x);
  if (threadIdx.x == 0) {
    float* pp = pr.part + w.part_off + 4 * (t.ty * w.tiles_side + t.tx);
    pp[0] = a0;
    pp[1] = a1;
    pp[2] = a2;
    pp[3] = a3;
  }
}

// compact input slopes -> dense grid + tip/tilt partial sums
__global__ __launch_bounds__(256) void k_slopes_in(const ProbDev* P, const WfsDev* WD, const IoDev* IO,
                                                   const Tile* tiles) {
  __shared__ float sh[16];
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const WfsDev& w = WD[pr.wfs0 + t.item];
  const IoDev& io = IO[t.prob];
  const int N = w.N;
  const int i = t.ty * kTileS + (threadIdx.x >> 4), j = t.tx * kTileS + (threadIdx.x & 15);
  float sx = 0.f, sy = 0.f, cx = 0.f, cy = 0.f;
  if (i < N && j < N) {
    const int ci = pr.cmap[w.m_off + i * N + j];
    if (ci >= 0) {
      sx = io.in[w.cs_off + ci];
      sy = io.in[w.cs_off + w.n_active + ci];
      if (w.blocks) {
        const float* cb = pr.cinv + w.cinv_off + 3 * (i * N + j);
        cx = cb[0] * sx + cb[1] * sy;
        cy = cb[1] * sx + cb[2] * sy;
      }
    }
    pr.sd[w.s_off + i * N + j] = sx;
    pr.sd[w.s_off + N * N + i * N + j] = sy;
  }
  const float a0 = block_sum(sx, sh, blockDim.x);
  const float a1 = block_sum(sy, sh + 4, blockDim.x);
  const float a2 = block_sum(cx, sh + 8, blockDim.x);
  const float a3 = block_sum(cy, sh + 12, blockDim.x);
  if (threadIdx.x == 0) {
    float* pp = pr.part + w.part_off + 4 * (t.ty * w.tiles_side + t.tx);
    pp[0] = a0;
    pp[1] = a1;
    pp[2] = a2;
    pp[3] = a3;
  }
}

// ------------------------------------- noise weighting + Shack-Hartmann adjoint
// Tile of 16x16 corners; the weighted slopes of the 17x17 subapertures that
// touch them are formed in LDS: C_hat^{-1} = (I - T) C^{-1} (I - T) for LGS
// with tip/tilt removal (means from the per-tile partial sums, Sec. 3.2),
// C^{-1} otherwise; GT_PLAIN applies Gamma^T alone.
__global__ __launch_bounds__(256) void k_gammaT(const ProbDev* P, const WfsDev* WD, const Tile* tiles, int mode) {
  constexpr int SW = kTileS + 1;
  __shared__ float YX[SW * SW];
  __shared__ float YY[SW * SW];
  __shared__ float mean[4];
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const WfsDev& w = WD[pr.wfs0 + t.item];
  const int N = w.N, nc = w.nc;
  const bool weighted = mode == GT_WEIGHTED;
  if (threadIdx.x == 0) {
    float mx = 0.f, my = 0.f, m2x = 0.f, m2y = 0.f;
    if (weighted && w.tt) {
      float sx = 0.f, sy = 0.f, scx = 0.f, scy = 0.f;
      const float* pp = pr.part + w.part_off;
      for (int k = 0; k < w.n_tiles_s; ++k) {
        sx += pp[4 * k];
        sy += pp[4 * k + 1];
        scx += pp[4 * k + 2];
        scy += pp[4 * k + 3];
      }
      mx = sx * w.inv_nM;
      my = sy * w.inv_nM;
      if (w.blocks) {
        m2x = (scx - (w.sum_cinv[0] * mx + w.sum_cinv[1] * my)) * w.inv_nM;
        m2y = (scy - (w.sum_cinv[2] * mx + w.sum_cinv[3] * my)) * w.inv_nM;
      }
    }
    mean[0] = mx;
    mean[1] = my;
    mean[2] = m2x;
    mean[3] = m2y;
  }
  __syncthreads();
  const int ci0 = t.ty * kTileS, cj0 = t.tx * kTileS;
  for (int e = threadIdx.x; e < SW * SW; e += blockDim.x) {
    const int li = e / SW, lj = e - li * SW;
    const int i = ci0 - 1 + li, j = cj0 - 1 + lj;  // subaperture
    float yx = 0.f, yy = 0.f;
    if (i >= 0 && j >= 0 && i < N && j < N && pr.cmap[w.m_off + i * N + j] >= 0) {
      const float sx = pr.sd[w.s_off + i * N + j];
      const float sy = pr.sd[w.s_off + N * N + i * N + j];
      if (!weighted) {
        yx = sx;
        yy = sy;
      } else if (w.blocks) {
        const float* cb = pr.cinv + w.cinv_off + 3 * (i * N + j);
        const float dx = sx - mean[0], dy = sy - mean[1];
        yx = cb[0] * dx + cb[1] * dy - mean[2];
        yy = cb[1] * dx + cb[2] * dy - mean[3];
      } else {
        yx = w.inv_sigma2 * (sx - mean[0]);
        yy = w.inv_sigma2 * (sy - mean[1]);
      }
    }
    YX[e] = yx;
    YY[e] = yy;
  }
  __syncthreads();
  const int li = threadIdx.x >> 4, lj = threadIdx.x & 15;
  const int i = ci0 + li, j = cj0 + lj;
  if (i < nc && j < nc) {
    // subapertures (i-1, j-1), (i-1, j), (i, j-1), (i, j) sit at local (li, lj) .. (li+1, lj+1)
    const float xa = YX[li * SW + lj], xb = YX[li * SW + lj + 1];
    const float xc = YX[(li + 1) * SW + lj], xd = YX[(li + 1) * SW + lj + 1];
    const float ya = YY[li * SW + lj], yb = YY[li * SW + lj + 1];
    const float yc = YY[(li + 1) * SW + lj], yd = YY[(li + 1) * SW + lj + 1];
    const float v = 0.5f * ((xc - xd) + (xa - xb)) + 0.5f * ((ya + yb) - (yc + yd));
    pr.vadj[w.v_off + i * nc + j] = v;
  }
}

// ------------------------------------------------ propagation adjoint (gather)
// Tile of 32x32 nodes of one layer: each node gathers, from every sensor, the
// corners whose bilinear cell touches it, with the forward weights.  No
// atomics: each node is written by exactly one thread.
__global__ __launch_bounds__(256) void k_pT(const ProbDev* P, const LayerDev* LD, const WfsDev* WD, const IoDev* IO,
                                            const Tile* tiles, int mode) {
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[pr.layer0 + t.item];
  const IoDev& io = IO[t.prob];
  const int n = ly.n;
  const int q = t.tx * kTileN + (threadIdx.x & 31);
  const int pbase = t.ty * kTileN + (threadIdx.x >> 5);
  if (q >= n) return;  // layers narrower than a tile (no barriers below)
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int g = 0; g < pr.G; ++g) {
    const WfsDev& w = WD[pr.wfs0 + g];
    const int nc = w.nc;
    const int base = w.tab_off + t.item * w.tab_stride;
    const int* it = pr.itab + base;
    const float* ft = pr.ftab + base;
    const int* ay0 = it + 4 * nc;  // int slots [2nc, 4nc) are the float weights' positions
    const int* ayc = ay0 + n;
    const int* ax0 = ayc + n;
    const int* axc = ax0 + n;
    const int* q0y = it;
    const int* q0x = it + nc;
    const float* wyv = ft + 2 * nc;
    const float* wxv = ft + 3 * nc;
    const float* va = pr.vadj + w.v_off;
    const int jx0 = ax0[q], jxc = axc[q];
    if (jxc == 0) continue;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int p = pbase + 8 * u;
      if (p >= n) continue;
      const int iy0 = ay0[p], iyc = ayc[p];
      float s = 0.f;
      for (int a = 0; a < iyc; ++a) {
        const int i = iy0 + a;
        const float wy = (q0y[i] == p) ? 1.f - wyv[i] : wyv[i];
        float r = 0.f;
        for (int b = 0; b < jxc; ++b) {
          const int j = jx0 + b;
          const float wx = (q0x[j] == q) ? 1.f - wxv[j] : wxv[j];
          r += wx * va[i * nc + j];
        }
        s += wy * r;
      }
      acc[u] += s;
    }
  }
  float* dst = (mode == PT_USER) ? io.out : pr.phiadj;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (pbase + 8 * u < n) dst[ly.off + (pbase + 8 * u) * n + q] = acc[u];
}

// ------------------------------------------------------------ PCG update
// a = rho_k / pi_k; x += a p; r -= a q; partial rho_{k+1} = r^T J^{-1} r.
__global__ __launch_bounds__(256) void k_update(const ProbDev* P, const IoDev* IO, const Tile* tiles, int iter) {
  __shared__ double sh[4];
  __shared__ double salpha;
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const IoDev& io = IO[t.prob];
  if (threadIdx.x == 0) {
    const double rho = sum_slots(dot_group(pr, 2 * iter), rho_count(pr, iter));
    const double pi = sum_slots(dot_group(pr, 2 * iter + 1), pr.n_slots_fdwt);
    salpha = (pi > 0.0) ? rho / pi : 0.0;
  }
  __syncthreads();
  const float a = (float)salpha;
  const float* p = (iter & 1) ? pr.pbuf1 : pr.pbuf0;
  float* x = io.state;
  float* r = io.state + 2L * pr.n_c;
  const int e0 = t.ty * kUpdChunk;
  const int e1 = min(e0 + kUpdChunk, pr.n_c);
  double acc = 0.0;
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    x[e] = fmaf(a, p[e], x[e]);
    const float re = fmaf(-a, pr.q[e], r[e]);
    r[e] = re;
    acc += (double)re * (double)re * (double)pr.jinv[e];
  }
  const double s = block_sum(acc, sh, blockDim.x);
  if (threadIdx.x == 0) pr.dots[(long)(2 * (iter + 1)) * pr.n_dots + t.slot] = s;
}

// ------------------------------------------------------------ launchers

void launch_idwt_res(const LaunchArgs& a, const Tile* tiles, int ntiles, int src_mode, int out_mode, int iter) {
  if (ntiles > 0)
    k_idwt_res<<<ntiles, 1024, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, src_mode, out_mode, iter);
}
void launch_idwt_glob(const LaunchArgs& a, const Tile* tiles, int ntiles, int src_mode, int out_mode, int iter,
                      int step) {
  if (ntiles > 0)
    k_idwt_glob<<<ntiles, 256, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, src_mode, out_mode, iter, step);
}
void launch_fdwt_glob(const LaunchArgs& a, const Tile* tiles, int ntiles, int epi, int iter, int step) {
  if (ntiles > 0) k_fdwt_glob<<<ntiles, 256, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, epi, iter, step);
}
void launch_fdwt_res(const LaunchArgs& a, const Tile* tiles, int ntiles, int epi, int iter) {
  if (ntiles > 0) k_fdwt_res<<<ntiles, 1024, 0, a.stream>>>(a.P, a.L, a.IO, tiles, a.F, epi, iter);
}
void launch_pgamma(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode) {
  if (ntiles > 0) k_pgamma<<<ntiles, 256, 0, a.stream>>>(a.P, a.L, a.W, a.IO, tiles, mode);
}
void launch_slopes_in(const LaunchArgs& a, const Tile* tiles, int ntiles) {
  if (ntiles > 0) k_slopes_in<<<ntiles, 256, 0, a.stream>>>(a.P, a.W, a.IO, tiles);
}
void launch_gammaT(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode) {
  if (ntiles > 0) k_gammaT<<<ntiles, 256, 0, a.stream>>>(a.P, a.W, tiles, mode);
}
void launch_pT(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode) {
  if (ntiles > 0) k_pT<<<ntiles, 256, 0, a.stream>>>(a.P, a.L, a.W, a.IO, tiles, mode);
}
void launch_update(const LaunchArgs& a, const Tile* tiles, int ntiles, int iter) {
  if (ntiles > 0) k_update<<<ntiles, 256, 0, a.stream>>>(a.P, a.IO, tiles, iter);
}

}  // namespace fewha
