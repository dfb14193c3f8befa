// FP64 residual of the refined solves (mixed-precision iterative refinement:
// the correction solves run the FP32 PCG, the residual that drives them is
// evaluated here in double precision so that the refined solution is limited
// neither by the rounding of the FP32 operator nor by a rounded right-hand
// side):
//   r = b + W^{-T} (A^T C_hat^{-1} (s - A W^{-1} x) + g) - alpha D x
// with each of b (coefficients), s (slopes) and g (layers) optional, i.e.
// r = b' - M x for b' = b + W^{-T} A^T C_hat^{-1} s + W^{-T} g (eq. fewha, eq. M).
//
// The chain runs step by step in
// global memory: the transforms level by level (one launch per separable
// pass), propagation + Shack-Hartmann per subaperture, the noise weighting
// with tip/tilt removal per sensor, and the adjoints as gathers (every output
// is written by one thread: deterministic, no atomics).  Called a few times
// per solve, so plain code is preferred over LDS tiling here.
#include "kernels.h"

namespace fewha {
namespace {

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sum of two values; results valid in every thread.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
  a = wave_sum64(a);
  b = wave_sum64(b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sh[2 * w] = a;
    sh[2 * w + 1] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  for (int i = 0; i < nw; ++i) {
    a += sh[2 * i];
    b += sh[2 * i + 1];
  }
}

// level index j of Mallat position (r, c): the coarse block and the first
// detail band share j = log2(n) - levels; finer bands j = floor(log2(max(r, c)))
__device__ __forceinline__ int level_j(const LayerDev& ly, int r, int c) {
  const int m0 = ly.n >> ly.levels, mx = max(r, c);
  return (mx < m0) ? ly.log2n - ly.levels : 31 - __clz(mx);
}

__device__ __forceinline__ int layer_of(const ProbDev& pr, const LayerDev* LD, int e) {
  int l = 0;
  while (l + 1 < pr.L && e >= LD[pr.layer0 + l + 1].off) ++l;
  return l;
}

}  // namespace

// the iterate x64 -> a64 (upd tiles)
__global__ __launch_bounds__(256) void k64_load(const ProbDev* P, const Tile* tiles) {
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const int e0 = t.ty * kUpdChunk, e1 = min(e0 + kUpdChunk, pr.n_c);
  for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) pr.a64[e] = pr.x64[e];
}

// One separable pass of one synthesis level (side m = 2^t.level) over the
// elements of a tile chunk.  pass 0: columns a64 -> b64; pass 1: rows b64 -> a64.
//   x_t = sum_{i = t mod 2} h_i a[(t-i)/2] + g_i d[(t-i)/2]   (indices mod m/2)
__global__ __launch_bounds__(256) void k64_idwt_pass(const ProbDev* P, const LayerDev* LD, const Tile* tiles,
                                                     Filter64 F, int pass) {
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[pr.layer0 + t.item];
  const int n = ly.n, m = 1 << t.level, half = m >> 1, lm = t.level;
  double* A = pr.a64 + ly.off;
  double* B = pr.b64 + ly.off;
  const int e0 = t.ty * 1024, e1 = min(e0 + 1024, m * m);
  for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
    const int row = e >> lm, col = e & (m - 1);
    if (pass == 0) {
      const int par = row & 1, k0 = row >> 1;
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int k = (k0 - q) & (half - 1);
        acc += F.h[par + 2 * q] * A[k * n + col] + F.g[par + 2 * q] * A[(half + k) * n + col];
      }
      B[row * n + col] = acc;
    } else {
      const int par = col & 1, k0 = col >> 1;
      const double* Br = B + row * n;
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int k = (k0 - q) & (half - 1);
        acc += F.h[par + 2 * q] * Br[k] + F.g[par + 2 * q] * Br[half + k];
      }
      A[row * n + col] = acc;
    }
  }
}

// One separable pass of one analysis level (input side m = 2^t.level).
// pass 0: rows a64 -> b64; pass 1: columns b64 -> a64.
//   a_k = sum_i h_i x[(2k + i) mod m],  d_k = sum_i g_i x[(2k + i) mod m]
__global__ __launch_bounds__(256) void k64_fdwt_pass(const ProbDev* P, const LayerDev* LD, const Tile* tiles,
                                                     Filter64 F, int pass) {
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const LayerDev& ly = LD[pr.layer0 + t.item];
  const int n = ly.n, m = 1 << t.level, half = m >> 1, lh = t.level - 1;
  double* A = pr.a64 + ly.off;
  double* B = pr.b64 + ly.off;
  const int e0 = t.ty * 1024, e1 = min(e0 + 1024, m * half);
  for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
    double a = 0.0, d = 0.0;
    if (pass == 0) {
      const int row = e >> lh, k = e & (half - 1);
      const double* Ar = A + row * n;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const double v = Ar[(2 * k + i) & (m - 1)];
        a += F.h[i] * v;
        d += F.g[i] * v;
      }
      B[row * n + k] = a;
      B[row * n + half + k] = d;
    } else {
      const int k = e / m, col = e - k * m;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const double v = B[((2 * k + i) & (m - 1)) * n + col];
        a += F.h[i] * v;
        d += F.g[i] * v;
      }
      A[k * n + col] = a;
      A[(half + k) * n + col] = d;
    }
  }
}

// s - A phi per subaperture (pg tiles): the wavefront at the four corners is
// the sum over layers of the bilinear samples of phi = delta^{-1} a64.
__global__ __launch_bounds__(256) void k64_pgamma(const ProbDev* P, const LayerDev* LD, const WfsDev* WD,
                                                  const IoDev* IO, const Tile* tiles) {
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const WfsDev& w = WD[pr.wfs0 + t.item];
  const IoDev& io = IO[t.prob];
  const int N = w.N, nc = w.nc;
  const int i = t.ty * kTileS + (threadIdx.x >> 4), j = t.tx * kTileS + (threadIdx.x & 15);
  if (i >= N || j >= N) return;
  double sx = 0.0, sy = 0.0;
  const int ci0 = pr.cmap[w.m_off + i * N + j];
  if (ci0 >= 0) {
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int ci = i + (k >> 1), cj = j + (k & 1);
      double acc = 0.0;
      for (int l = 0; l < pr.L; ++l) {
        const LayerDev& ly = LD[pr.layer0 + l];
        const int base = w.tab_off + l * w.tab_stride;
        const int qy = pr.itab[base + ci], qx = pr.itab[base + nc + cj];
        const double wy = pr.ftab64[base + 2 * nc + ci], wx = pr.ftab64[base + 3 * nc + cj];
        const double* ph = pr.a64 + ly.off + qy * ly.n + qx;
        const double top = (1.0 - wx) * ph[0] + wx * ph[1];
        const double bot = (1.0 - wx) * ph[ly.n] + wx * ph[ly.n + 1];
        acc += ((1.0 - wy) * top + wy * bot) * ly.inv_delta64;
      }
      v[k] = acc;
    }
    sx = -0.5 * ((v[1] - v[0]) + (v[3] - v[2]));
    sy = -0.5 * ((v[2] - v[0]) + (v[3] - v[1]));
    if (io.rs) {
      sx += (double)io.rs[w.cs_off + ci0];
      sy += (double)io.rs[w.cs_off + w.n_active + ci0];
    }
  }
  pr.sd64[w.s_off + i * N + j] = sx;
  pr.sd64[w.s_off + N * N + i * N + j] = sy;
}

// C_hat^{-1} of one sensor in place (one workgroup per (problem, sensor)):
// (I - T) C^{-1} (I - T) with T the projector onto constant x / y slopes over
// the active subapertures (LGS with tip/tilt removal), C^{-1} otherwise.
__global__ __launch_bounds__(1024) void k64_noise(const ProbDev* P, const WfsDev* WD, const Tile* tiles) {
  __shared__ double sh[32];
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const WfsDev& w = WD[pr.wfs0 + t.item];
  const int N = w.N, NN = N * N;
  double* sx = pr.sd64 + w.s_off;
  double* sy = sx + NN;
  const int* cm = pr.cmap + w.m_off;
  if (w.tt) {
    double mx = 0.0, my = 0.0;
    for (int k = threadIdx.x; k < NN; k += blockDim.x) {
      mx += sx[k];
      my += sy[k];
    }
    block_sum2(mx, my, sh);
    mx *= w.inv_nM_d;
    my *= w.inv_nM_d;
    for (int k = threadIdx.x; k < NN; k += blockDim.x)
      if (cm[k] >= 0) {
        sx[k] -= mx;
        sy[k] -= my;
      }
  }
  for (int k = threadIdx.x; k < NN; k += blockDim.x) {
    if (cm[k] < 0) continue;
    const double x = sx[k], y = sy[k];
    if (w.blocks) {
      const double* cb = pr.cinv64 + w.cinv_off + 3 * k;
      sx[k] = cb[0] * x + cb[1] * y;
      sy[k] = cb[1] * x + cb[2] * y;
    } else {
      sx[k] = w.inv_sigma2_d * x;
      sy[k] = w.inv_sigma2_d * y;
    }
  }
  if (w.tt) {
    __syncthreads();
    double mx = 0.0, my = 0.0;
    for (int k = threadIdx.x; k < NN; k += blockDim.x) {
      mx += sx[k];
      my += sy[k];
    }
    block_sum2(mx, my, sh);
    mx *= w.inv_nM_d;
    my *= w.inv_nM_d;
    for (int k = threadIdx.x; k < NN; k += blockDim.x)
      if (cm[k] >= 0) {
        sx[k] -= mx;
        sy[k] -= my;
      }
  }
}

// Gamma^T per corner (gt tiles): each subaperture's slopes reach its four
// corners with weights +-1/2 (adjoint of the stencil of Sec. 2).
__global__ __launch_bounds__(256) void k64_gammaT(const ProbDev* P, const WfsDev* WD, const Tile* tiles) {
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const WfsDev& w = WD[pr.wfs0 + t.item];
  const int N = w.N, nc = w.nc, NN = N * N;
  const int i = t.ty * kTileS + (threadIdx.x >> 4), j = t.tx * kTileS + (threadIdx.x & 15);
  if (i >= nc || j >= nc) return;
  const double* yx = pr.sd64 + w.s_off;
  const double* yy = yx + NN;
  double u = 0.0;
  // subaperture (a, b) holds this corner at (i - a, j - b) in {0, 1}^2
#pragma unroll
  for (int da = 0; da < 2; ++da)
#pragma unroll
    for (int db = 0; db < 2; ++db) {
      const int a = i - da, b = j - db;
      if (a < 0 || b < 0 || a >= N || b >= N) continue;
      const int k = a * N + b;
      const double cx = db ? 0.5 : -0.5;  // d s^x / d v: +1/2 right column, -1/2 left
      const double cy = da ? 0.5 : -0.5;  // d s^y / d v: +1/2 lower row, -1/2 upper
      u += cx * yx[k] + cy * yy[k];
    }
  pr.u64[w.v_off + i * nc + j] = u;
}

// P^T per layer node (pt tiles of 32x32 nodes): gather over every sensor of
// the corners whose bilinear cell touches the node, with the forward weights
// (exact transpose of the propagation), plus g.  Output into a64 (layer layout).
__global__ __launch_bounds__(256) void k64_pT(const ProbDev* P, const LayerDev* LD, const WfsDev* WD,
                                              const IoDev* IO, const Tile* tiles) {
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const IoDev& io = IO[t.prob];
  const int l = t.item;
  const LayerDev& ly = LD[pr.layer0 + l];
  const int n = ly.n;
  for (int e = threadIdx.x; e < kTileN * kTileN; e += 256) {
    const int p = t.ty * kTileN + e / kTileN, q = t.tx * kTileN + e % kTileN;
    if (p >= n || q >= n) continue;
    double acc = io.rg ? (double)io.rg[ly.off + p * n + q] : 0.0;
    for (int g = 0; g < pr.G; ++g) {
      const WfsDev& w = WD[pr.wfs0 + g];
      const GLPar& gp = pr.gl[g * pr.L + l];
      const int nc = w.nc, base = w.tab_off + l * w.tab_stride;
      const int ylo = max(0, (int)floor((p - 1 - gp.t0y) * gp.inv_rho) - 1);
      const int yhi = min(nc - 1, (int)ceil((p + 1 - gp.t0y) * gp.inv_rho) + 1);
      const int xlo = max(0, (int)floor((q - 1 - gp.t0x) * gp.inv_rho) - 1);
      const int xhi = min(nc - 1, (int)ceil((q + 1 - gp.t0x) * gp.inv_rho) + 1);
      const double* u = pr.u64 + w.v_off;
      for (int ky = ylo; ky <= yhi; ++ky) {
        const int qy = pr.itab[base + ky];
        const double wy = pr.ftab64[base + 2 * nc + ky];
        const double fy = (qy == p) ? 1.0 - wy : (qy == p - 1 ? wy : 0.0);
        if (fy == 0.0) continue;
        double row = 0.0;
        for (int kx = xlo; kx <= xhi; ++kx) {
          const int qx = pr.itab[base + nc + kx];
          const double wx = pr.ftab64[base + 3 * nc + kx];
          const double fx = (qx == q) ? 1.0 - wx : (qx == q - 1 ? wx : 0.0);
          row += fx * u[ky * nc + kx];
        }
        acc += fy * row;
      }
    }
    pr.a64[ly.off + p * n + q] = acc;
  }
}

// r = b + delta^{-1} (W a64) - alpha D x64 per coefficient (upd tiles),
// written as float; per tile the FP64 partial sum of r^2.
__global__ __launch_bounds__(256) void k64_resid(const ProbDev* P, const LayerDev* LD, const IoDev* IO,
                                                 const Tile* tiles) {
  __shared__ double sh[8];
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const IoDev& io = IO[t.prob];
  const int e0 = t.ty * kUpdChunk, e1 = min(e0 + kUpdChunk, pr.n_c);
  double rr = 0.0, bb = 0.0;
  for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
    const LayerDev& ly = LD[pr.layer0 + layer_of(pr, LD, e)];
    const int loc = e - ly.off, r = loc >> ly.log2n, c = loc & (ly.n - 1);
    const double b = io.in ? (double)io.in[e] : 0.0;
    const double res = b + pr.a64[e] * ly.inv_delta64 - pr.alpha * ly.d64[level_j(ly, r, c)] * pr.x64[e];
    io.out[e] = (float)res;
    rr += res * res;
  }
  block_sum2(rr, bb, sh);
  if (threadIdx.x == 0) {
    pr.rslots[2 * t.slot] = rr;
    pr.rslots[2 * t.slot + 1] = bb;
  }
}

// Iterate bookkeeping (upd tiles):
//   mode 0: x64 = 0;  mode 1: x64 += d (io.in);  mode 2: x = (float) x64 (io.state)
__global__ __launch_bounds__(256) void k64_iterate(const ProbDev* P, const IoDev* IO, const Tile* tiles, int mode) {
  const Tile t = tiles[blockIdx.x];
  const ProbDev& pr = P[t.prob];
  const IoDev& io = IO[t.prob];
  const int e0 = t.ty * kUpdChunk, e1 = min(e0 + kUpdChunk, pr.n_c);
  for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
    if (mode == 0)
      pr.x64[e] = 0.0;
    else if (mode == 1)
      pr.x64[e] += (double)io.in[e];
    else
      io.state[e] = (float)pr.x64[e];
  }
}

void launch64_resid_chain(const LaunchArgs& a, const Resid64Tiles& rt, const Filter64& F) {
  if (rt.upd_n == 0) return;
  k64_load<<<rt.upd_n, 256, 0, a.stream>>>(a.P, rt.upd);
  for (int s = 0; s < rt.n_steps; ++s) {
    if (rt.inv_n[s] == 0) continue;
    k64_idwt_pass<<<rt.inv_n[s], 256, 0, a.stream>>>(a.P, a.L, rt.inv[s], F, 0);
    k64_idwt_pass<<<rt.inv_n[s], 256, 0, a.stream>>>(a.P, a.L, rt.inv[s], F, 1);
  }
  if (rt.pg_n > 0) k64_pgamma<<<rt.pg_n, 256, 0, a.stream>>>(a.P, a.L, a.W, a.IO, rt.pg);
  if (rt.wfs_n > 0) k64_noise<<<rt.wfs_n, 1024, 0, a.stream>>>(a.P, a.W, rt.wfs);
  if (rt.gt_n > 0) k64_gammaT<<<rt.gt_n, 256, 0, a.stream>>>(a.P, a.W, rt.gt);
  if (rt.pt_n > 0) k64_pT<<<rt.pt_n, 256, 0, a.stream>>>(a.P, a.L, a.W, a.IO, rt.pt);
  for (int s = 0; s < rt.n_steps; ++s) {
    if (rt.fwd_n[s] == 0) continue;
    k64_fdwt_pass<<<rt.fwd_n[s], 256, 0, a.stream>>>(a.P, a.L, rt.fwd[s], F, 0);
    k64_fdwt_pass<<<rt.fwd_n[s], 256, 0, a.stream>>>(a.P, a.L, rt.fwd[s], F, 1);
  }
  k64_resid<<<rt.upd_n, 256, 0, a.stream>>>(a.P, a.L, a.IO, rt.upd);
}

void launch64_iterate(const LaunchArgs& a, const Tile* tiles, int ntiles, int mode) {
  if (ntiles > 0) k64_iterate<<<ntiles, 256, 0, a.stream>>>(a.P, a.IO, tiles, mode);
}

}  // namespace fewha
