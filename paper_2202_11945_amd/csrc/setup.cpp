// Host set-up of one FEWHA problem: sensor masks, bilinear propagation
// tables with the LGS cone factor (Sec. 2), spot-elongated noise blocks
// (eq. LGS-noise), the diagonal wavelet prior D (Sec. 3.1) and the exact
// Jacobi diagonal J (eq. precond), all in double precision.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "fewha_internal.h"

namespace fewha {

// Daubechies' extremal-phase filter with 3 vanishing moments in closed form
// (radicals of sqrt 10 and sqrt(5 + 2 sqrt 10)), normalised to sum sqrt 2.
void db3_filter(double h[6]) {
  const double a = std::sqrt(10.0);
  const double b = std::sqrt(5.0 + 2.0 * a);
  const double s = std::sqrt(2.0) / 32.0;
  h[0] = s * (1.0 + a + b);
  h[1] = s * (5.0 + a + 3.0 * b);
  h[2] = s * (10.0 - 2.0 * a + 2.0 * b);
  h[3] = s * (10.0 - 2.0 * a - 2.0 * b);
  h[4] = s * (5.0 + a - 3.0 * b);
  h[5] = s * (1.0 + a - b);
}

namespace {

int ilog2(int n) {
  int k = 0;
  while ((1 << k) < n) ++k;
  return k;
}

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// 1-D periodic synthesis of [a; d] (length m) in place, the transpose of
// a_k = sum_i h_i x[(2k+i) mod m], d_k = sum_i g_i x[(2k+i) mod m].
void synth1d(std::vector<double>& x, int m, const double* h, const double* g) {
  std::vector<double> y(m, 0.0);
  const int half = m / 2;
  for (int k = 0; k < half; ++k) {
    const double a = x[k], d = x[half + k];
    if (a == 0.0 && d == 0.0) continue;
    for (int i = 0; i < 6; ++i) y[(2 * k + i) % m] += h[i] * a + g[i] * d;
  }
  for (int t = 0; t < m; ++t) x[t] = y[t];
}

// 1-D basis function of level k (1-based) on a length-n periodic grid:
// wavelet (type 1) or scaling function (type 0) with index r.
std::vector<double> basis1d(int n, int k, int type, int r, const double* h, const double* g) {
  int m = n >> (k - 1);
  std::vector<double> v(n, 0.0);
  v[type ? (m / 2 + r) : r] = 1.0;
  for (int lev = k; lev >= 1; --lev) {
    m = n >> (lev - 1);
    synth1d(v, m, h, g);  // entries beyond m are zero
  }
  return v;
}

}  // namespace

fewha_status build_model(HostModel& m, std::string& err) {
  char buf[256];
  if (!m.have_pupil || !m.have_wfs || !m.have_layers) {
    err = "finalize: pupil, sensors and layers must be set first";
    return FEWHA_ESTATE;
  }
  db3_filter(m.h);
  for (int i = 0; i < 6; ++i) m.g[i] = ((i & 1) ? -1.0 : 1.0) * m.h[5 - i];

  const double D = m.D;
  const int G = (int)m.wfs.size();
  const int L = (int)m.layers.size();

  // ---- layers and the prior ----
  m.layer_off.assign(L + 1, 0);
  for (int l = 0; l < L; ++l) {
    LayerHost& lh = m.layers[l];
    const int n = lh.d.n;
    if (!is_pow2(n) || n < 8 || n > 2048) {
      std::snprintf(buf, sizeof buf, "layer %d: grid side %d must be a power of two in [8, 2048]", l, n);
      err = buf;
      return FEWHA_EGEOM;
    }
    const int J = ilog2(n);
    if (lh.d.levels < 1 || lh.d.levels > J || (n >> lh.d.levels) > kResMax) {
      std::snprintf(buf, sizeof buf, "layer %d: levels %d unsupported for n = %d", l, lh.d.levels, n);
      err = buf;
      return FEWHA_EGEOM;
    }
    if (!(lh.d.cn2 > 0.0) || !(lh.d.h >= 0.0)) {
      std::snprintf(buf, sizeof buf, "layer %d: need cn2 > 0 and h >= 0", l);
      err = buf;
      return FEWHA_EINVAL;
    }
    lh.delta = m.L / n;
    lh.dtab.assign(kMaxLevelsJ, 0.0);
    for (int j = J - lh.d.levels; j < J; ++j) {
      const double f = std::pow(2.0, j) / m.L;
      const double psd = 0.023 * lh.d.cn2 * std::pow(m.r0, -5.0 / 3.0) *
                         std::pow(f * f + std::pow(m.L0, -2.0), -11.0 / 6.0);
      lh.dtab[j] = 1.0 / psd;
    }
    m.layer_off[l + 1] = m.layer_off[l] + n * n;
  }
  m.n_c = m.layer_off[L];
  m.Dprior.assign(m.n_c, 0.0);
  for (int l = 0; l < L; ++l) {
    const LayerHost& lh = m.layers[l];
    const int n = lh.d.n, J = ilog2(n), jmin = J - lh.d.levels;
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) {
        const int mx = std::max(r, c);
        int j = jmin;
        if (mx >= (1 << jmin)) j = ilog2(mx + 1) - 1;
        m.Dprior[m.layer_off[l] + r * n + c] = lh.dtab[j];
      }
  }

  // ---- sensors: masks, compact maps, noise blocks ----
  m.slope_off.assign(G + 1, 0);
  for (int gi = 0; gi < G; ++gi) {
    WfsHost& w = m.wfs[gi];
    const int N = w.d.n_subap;
    const double d = D / N;
    if (w.mask.empty()) {
      w.mask.assign(N * N, 0);
      const double r_in = std::sqrt(m.obs) * 0.5 * D;
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
          const double X = -0.5 * D + (j + 0.5) * d;
          const double Y = -0.5 * D + (i + 0.5) * d;
          const double r = std::sqrt(X * X + Y * Y);
          w.mask[i * N + j] = (r >= r_in && r <= 0.5 * D) ? 1 : 0;
        }
    }
    w.cmap.assign(N * N, -1);
    int cnt = 0;
    for (int k = 0; k < N * N; ++k)
      if (w.mask[k]) w.cmap[k] = cnt++;
    if (cnt == 0) {
      std::snprintf(buf, sizeof buf, "sensor %d has no active subaperture", gi);
      err = buf;
      return FEWHA_EGEOM;
    }
    w.n_active = cnt;
    m.slope_off[gi + 1] = m.slope_off[gi] + 2 * cnt;
    // C_ij^{-1}: sigma^{-2} I, or with elongation beta = FWHM/H^2 (centre - launch):
    // (sigma^2 (I + k beta beta^T))^{-1} = sigma^{-2} (I - k beta beta^T / (1 + k |beta|^2))
    const double is2 = 1.0 / (w.d.sigma * w.d.sigma);
    const bool elong = w.d.kind == FEWHA_LGS && m.alpha_eta > 0.0;
    const double kap = m.alpha_eta * m.alpha_eta / (m.spot_fwhm * m.spot_fwhm);
    w.cinv.assign(3 * N * N, 0.0);
    for (int v = 0; v < 4; ++v) w.sum_cinv[v] = 0.0;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        const int k = i * N + j;
        if (!w.mask[k]) continue;
        double a = is2, b = 0.0, c = is2;
        if (elong) {
          const double X = -0.5 * D + (j + 0.5) * d;
          const double Y = -0.5 * D + (i + 0.5) * d;
          const double bx = m.na_fwhm / (w.d.H * w.d.H) * (X - w.d.launch_x);
          const double by = m.na_fwhm / (w.d.H * w.d.H) * (Y - w.d.launch_y);
          const double den = 1.0 + kap * (bx * bx + by * by);
          a = is2 * (1.0 - kap * bx * bx / den);
          b = -is2 * kap * bx * by / den;
          c = is2 * (1.0 - kap * by * by / den);
        }
        w.cinv[3 * k] = a;
        w.cinv[3 * k + 1] = b;
        w.cinv[3 * k + 2] = c;
        w.sum_cinv[0] += a;
        w.sum_cinv[1] += b;
        w.sum_cinv[2] += b;
        w.sum_cinv[3] += c;
      }
  }
  m.n_slopes = m.slope_off[G];

  // ---- propagation tables (no periodic wrap: the footprint must fit) ----
  m.tab.assign(G, std::vector<GLTables>(L));
  for (int gi = 0; gi < G; ++gi) {
    const WfsHost& w = m.wfs[gi];
    const int N = w.d.n_subap, nc = N + 1;
    for (int l = 0; l < L; ++l) {
      const LayerHost& lh = m.layers[l];
      const int n = lh.d.n;
      const double hgt = lh.d.h;
      if (w.d.kind == FEWHA_LGS && !(hgt < w.d.H)) {
        std::snprintf(buf, sizeof buf, "sensor %d: layer %d at or above the LGS altitude", gi, l);
        err = buf;
        return FEWHA_EGEOM;
      }
      const double scale = (w.d.kind == FEWHA_LGS) ? 1.0 - hgt / w.d.H : 1.0;
      GLTables& t = m.tab[gi][l];
      t.q0y.resize(nc);
      t.q0x.resize(nc);
      t.wy.resize(nc);
      t.wx.resize(nc);
      for (int j = 0; j < nc; ++j) {
        const double x = -0.5 * D + j * (D / N);
        const double tx = (scale * x + hgt * w.d.theta_x + 0.5 * m.L) / lh.delta;
        const double ty = (scale * x + hgt * w.d.theta_y + 0.5 * m.L) / lh.delta;
        const double fx = std::floor(tx), fy = std::floor(ty);
        if (fx < 0 || fy < 0 || fx > n - 2 || fy > n - 2) {
          std::snprintf(buf, sizeof buf, "sensor %d footprint leaves layer %d", gi, l);
          err = buf;
          return FEWHA_EGEOM;
        }
        t.q0x[j] = (int)fx;
        t.wx[j] = tx - fx;
        t.q0y[j] = (int)fy;
        t.wy[j] = ty - fy;
      }
    }
  }

  // ---- derivative of the propagation with respect to the layer height ----
  // t(h) = (c(h) x + h theta + L/2) / delta with c = 1 - h/H (LGS) or 1, so
  // dt/dh = (theta - x/H) / delta or theta / delta.  On a grid line the
  // bilinear interpolant has no derivative; the average of the two one-sided
  // derivatives is used (the cell is centred on the node).
  m.gtab.assign(G, std::vector<GradTables>(L));
  m.grad_ok = true;
  m.grad_msg.clear();
  for (int gi = 0; gi < G; ++gi) {
    const WfsHost& w = m.wfs[gi];
    const int N = w.d.n_subap, nc = N + 1;
    const bool lgs = w.d.kind == FEWHA_LGS;
    for (int l = 0; l < L; ++l) {
      const LayerHost& lh = m.layers[l];
      const int n = lh.d.n;
      const double hgt = lh.d.h;
      const double scale = lgs ? 1.0 - hgt / w.d.H : 1.0;
      GradTables& t = m.gtab[gi][l];
      for (auto* v : {&t.qy, &t.qx, &t.tiey, &t.tiex}) v->assign(nc, 0);
      for (auto* v : {&t.wy, &t.wx, &t.dty, &t.dtx}) v->assign(nc, 0.0);
      for (int j = 0; j < nc; ++j) {
        const double x = -0.5 * D + j * (D / N);
        const double th[2] = {w.d.theta_x, w.d.theta_y};
        for (int ax = 0; ax < 2; ++ax) {
          const double tt = (scale * x + hgt * th[ax] + 0.5 * m.L) / lh.delta;
          const double r = std::nearbyint(tt);
          const bool tie = std::fabs(tt - r) < kTie;
          const int q = tie ? (int)r : (int)std::floor(tt);
          const double wf = tie ? 0.0 : tt - std::floor(tt);
          const double dt = ((lgs ? -x / w.d.H : 0.0) + th[ax]) / lh.delta;
          if ((tie && (q < 1 || q > n - 2)) || (!tie && (q < 0 || q > n - 2))) {
            if (m.grad_ok) {
              std::snprintf(buf, sizeof buf, "sensor %d: height-derivative stencil leaves layer %d", gi, l);
              m.grad_msg = buf;
            }
            m.grad_ok = false;
          }
          (ax == 0 ? t.qx : t.qy)[j] = q;
          (ax == 0 ? t.tiex : t.tiey)[j] = tie ? 1 : 0;
          (ax == 0 ? t.wx : t.wy)[j] = wf;
          (ax == 0 ? t.dtx : t.dty)[j] = dt;
        }
      }
    }
  }

  // ---- DM fitting: pupil corners, propagation tables, regularisation ----
  if (m.fit.on) {
    FitHost& f = m.fit;
    const int N = f.N, nc = N + 1;
    const double d = D / N;
    const double r_in = std::sqrt(m.obs) * 0.5 * D;
    std::vector<uint8_t> sub(N * N, 0);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        const double X = -0.5 * D + (j + 0.5) * d, Y = -0.5 * D + (i + 0.5) * d;
        const double r = std::sqrt(X * X + Y * Y);
        sub[i * N + j] = (r >= r_in && r <= 0.5 * D) ? 1 : 0;
      }
    f.cmap.assign(nc * nc, -1);
    int cnt = 0;
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j < nc; ++j) {
        bool in = false;
        for (int di = -1; di <= 0; ++di)
          for (int dj = -1; dj <= 0; ++dj) {
            const int a = i + di, b = j + dj;
            if (a >= 0 && b >= 0 && a < N && b < N && sub[a * N + b]) in = true;
          }
        if (in) f.cmap[i * nc + j] = cnt++;
      }
    const int K = (int)f.dirs.size() / 2;
    // layers -> corners (no cone effect), DMs -> corners (centred actuator grids)
    // t = (x + shift + add) / spacing + offset, floor and fraction per corner row / column
    auto table = [&](double shift_x, double shift_y, double add, double spacing, double offset, int n,
                     GLTables& t) -> bool {
      t.q0y.resize(nc);
      t.q0x.resize(nc);
      t.wy.resize(nc);
      t.wx.resize(nc);
      for (int j = 0; j < nc; ++j) {
        const double x = -0.5 * D + j * (D / N);
        const double tx = (x + shift_x + add) / spacing + offset;
        const double ty = (x + shift_y + add) / spacing + offset;
        const double fx = std::floor(tx), fy = std::floor(ty);
        if (fx < 0 || fy < 0 || fx > n - 2 || fy > n - 2) return false;
        t.q0x[j] = (int)fx;
        t.wx[j] = tx - fx;
        t.q0y[j] = (int)fy;
        t.wy[j] = ty - fy;
      }
      return true;
    };
    f.tabL.assign(K, std::vector<GLTables>(L));
    f.tabD.assign(K, std::vector<GLTables>(f.dms.size()));
    f.dm_off.assign(f.dms.size() + 1, 0);
    for (size_t q = 0; q < f.dms.size(); ++q) f.dm_off[q + 1] = f.dm_off[q] + f.dms[q].n_act * f.dms[q].n_act;
    f.n_act = f.dm_off.back();
    std::vector<double> diag(f.n_act, 0.0);
    for (int k = 0; k < K; ++k) {
      const double thx = f.dirs[2 * k], thy = f.dirs[2 * k + 1];
      for (int l = 0; l < L; ++l) {
        const LayerHost& lh = m.layers[l];
        if (!table(lh.d.h * thx, lh.d.h * thy, 0.5 * m.L, lh.delta, 0.0, lh.d.n, f.tabL[k][l])) {
          std::snprintf(buf, sizeof buf, "fitting direction %d leaves layer %d", k, l);
          err = buf;
          return FEWHA_EGEOM;
        }
      }
      for (size_t q = 0; q < f.dms.size(); ++q) {
        const fewha_dm_desc& dm = f.dms[q];
        GLTables& t = f.tabD[k][q];
        if (!table(dm.h * thx, dm.h * thy, 0.0, dm.pitch, 0.5 * (dm.n_act - 1), dm.n_act, t)) {
          std::snprintf(buf, sizeof buf, "fitting direction %d leaves DM %d", k, (int)q);
          err = buf;
          return FEWHA_EGEOM;
        }
        for (int i = 0; i < nc; ++i)
          for (int j = 0; j < nc; ++j) {
            if (f.cmap[i * nc + j] < 0) continue;
            const double wy[2] = {1.0 - t.wy[i], t.wy[i]}, wx[2] = {1.0 - t.wx[j], t.wx[j]};
            for (int a = 0; a < 2; ++a)
              for (int b = 0; b < 2; ++b)
                diag[f.dm_off[q] + (t.q0y[i] + a) * dm.n_act + t.q0x[j] + b] += wy[a] * wy[a] * wx[b] * wx[b];
          }
      }
    }
    double mean = 0.0;
    for (double v : diag) mean += v;
    mean /= (double)f.n_act;
    f.eps = f.eps_rel * mean;
  }

  // ---- exact Jacobi diagonal, eq. (precond) ----
  // Every 2-D basis function is a product u(y) v(x) of 1-D periodic basis
  // functions of one level, so its propagated wavefront is U(i) V(j) and its
  // slopes are s^x_ij = (V_{j+1}-V_j)(U_i+U_{i+1})/2, s^y_ij = (U_{i+1}-U_i)(V_j+V_{j+1})/2.
  // The diagonal entry is delta^{-2} sum_g s_g^T C_hat_g^{-1} s_g, with the
  // tip/tilt projection expanded over the full mask.
  m.J.assign(m.n_c, 0.0);
  for (int l = 0; l < L; ++l) {
    const LayerHost& lh = m.layers[l];
    const int n = lh.d.n, levels = lh.d.levels;
    // 1-D basis functions per (level, type, index): propagated to every
    // sensor's corner rows (y tables) and columns (x tables)
    struct Prop {
      std::vector<double> val;  // nc values
      int lo, hi;               // nonzero corner range (inclusive), lo > hi if none
    };
    // idx(k, type, r) -> flat
    std::vector<int> base(levels + 1, 0);
    int total = 0;
    for (int k = 1; k <= levels; ++k) {
      base[k] = total;
      total += 2 * (n >> k);
    }
    std::vector<std::vector<double>> fun(total);
    for (int k = 1; k <= levels; ++k)
      for (int type = 0; type < 2; ++type)
        for (int r = 0; r < (n >> k); ++r) fun[base[k] + type * (n >> k) + r] = basis1d(n, k, type, r, m.h, m.g);
    std::vector<std::vector<Prop>> PY(G), PX(G);
    for (int gi = 0; gi < G; ++gi) {
      const GLTables& t = m.tab[gi][l];
      const int nc = m.wfs[gi].d.n_subap + 1;
      PY[gi].resize(total);
      PX[gi].resize(total);
      for (int f = 0; f < total; ++f) {
        for (int axis = 0; axis < 2; ++axis) {
          Prop& pr = axis ? PX[gi][f] : PY[gi][f];
          const std::vector<int>& q0 = axis ? t.q0x : t.q0y;
          const std::vector<double>& w = axis ? t.wx : t.wy;
          pr.val.assign(nc, 0.0);
          pr.lo = nc;
          pr.hi = -1;
          for (int j = 0; j < nc; ++j) {
            const double v = (1.0 - w[j]) * fun[f][q0[j]] + w[j] * fun[f][q0[j] + 1];
            pr.val[j] = v;
            if (v != 0.0) {
              pr.lo = std::min(pr.lo, j);
              pr.hi = std::max(pr.hi, j);
            }
          }
        }
      }
    }
    const double id2 = 1.0 / (lh.delta * lh.delta);
#pragma omp parallel for schedule(dynamic, 16)
    for (int R = 0; R < n; ++R) {
      for (int C = 0; C < n; ++C) {
        // level and types of Mallat position (R, C)
        int k = levels, ty = 0, tx = 0, ry = R, rx = C;
        for (int kk = 1; kk <= levels; ++kk) {
          const int half = n >> kk;
          if (R >= half || C >= half) {
            k = kk;
            ty = R >= half;
            tx = C >= half;
            ry = ty ? R - half : R;
            rx = tx ? C - half : C;
            break;
          }
        }
        const int fy = base[k] + ty * (n >> k) + ry;
        const int fx = base[k] + tx * (n >> k) + rx;
        double acc = 0.0;
        for (int gi = 0; gi < G; ++gi) {
          const WfsHost& w = m.wfs[gi];
          const int N = w.d.n_subap;
          const Prop& U = PY[gi][fy];
          const Prop& V = PX[gi][fx];
          if (U.lo > U.hi || V.lo > V.hi) continue;
          const int i0 = std::max(0, U.lo - 1), i1 = std::min(N - 1, U.hi);
          const int j0 = std::max(0, V.lo - 1), j1 = std::min(N - 1, V.hi);
          double Q = 0, Sx = 0, Sy = 0, SCx = 0, SCy = 0;
          for (int i = i0; i <= i1; ++i) {
            const double aU = 0.5 * (U.val[i] + U.val[i + 1]);
            const double dU = U.val[i + 1] - U.val[i];
            const uint8_t* mrow = &w.mask[i * N];
            const double* crow = &w.cinv[3 * i * N];
            for (int j = j0; j <= j1; ++j) {
              if (!mrow[j]) continue;
              const double sx = (V.val[j + 1] - V.val[j]) * aU;
              const double sy = dU * 0.5 * (V.val[j] + V.val[j + 1]);
              const double cx = crow[3 * j] * sx + crow[3 * j + 1] * sy;
              const double cy = crow[3 * j + 1] * sx + crow[3 * j + 2] * sy;
              Q += sx * cx + sy * cy;
              Sx += sx;
              Sy += sy;
              SCx += cx;
              SCy += cy;
            }
          }
          if (w.d.kind == FEWHA_LGS && w.d.tt_removal) {
            const double nM = (double)w.n_active;
            const double* S = w.sum_cinv;
            Q += -2.0 / nM * (Sx * SCx + Sy * SCy) +
                 (Sx * (S[0] * Sx + S[1] * Sy) + Sy * (S[2] * Sx + S[3] * Sy)) / (nM * nM);
          }
          acc += Q;
        }
        const long e = m.layer_off[l] + (long)R * n + C;
        m.J[e] = id2 * acc + m.alpha * std::max(m.Dprior[e], m.tau);
      }
    }
  }
  return FEWHA_OK;
}

}  // namespace fewha
