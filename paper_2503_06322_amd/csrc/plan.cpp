// Host plan: the level hierarchy and per-axis operator tables of one shape.
//
// Hierarchy (Algorithm 1 builds it from the input; the coarsening rule for
// sizes other than 2^k + 1 is not given in the paper): axis coordinates are
// the grid indices; a coarsening step keeps the even positions of a level and,
// when its node count is even, also its last node; all axes longer than 1
// coarsen together until the shortest has 2 nodes.
//
// Operators (Section IV-A: the data is the piecewise linear function through
// the nodal values; lerp, mass_trans and tridiag of Algorithm 1): P is the
// prolongation of coarse hat functions into the fine basis, M the mass matrix
// of the hats on one level.  Per coarse node j the restriction row of
// P^T M_l has five taps at fine positions p(j)-2 .. p(j)+2; the tridiagonal
// coarse mass matrix is pre-factored for the Thomas sweeps.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

#pragma clang fp contract(off)

namespace mgc {

namespace {

inline int64_t cpos(int64_t j, int64_t nf) { return std::min<int64_t>(2 * j, nf - 1); }
inline bool is_new(int64_t i, int64_t nf) { return (i & 1) && !(i == nf - 1); }

std::vector<double> coarse_coords(const std::vector<double>& x) {
  const int64_t n = (int64_t)x.size();
  std::vector<double> out;
  for (int64_t i = 0; i < n; i += 2) out.push_back(x[i]);
  if (n % 2 == 0) out.push_back(x[n - 1]);
  return out;
}

// Mass-matrix entry M(f, g) of the hats on nodes x.
double mass_entry(const std::vector<double>& x, int64_t f, int64_t g) {
  const int64_t n = (int64_t)x.size();
  if (g < 0 || g >= n) return 0.0;
  if (f == g) {
    double hl = f > 0 ? x[f] - x[f - 1] : 0.0;
    double hr = f < n - 1 ? x[f + 1] - x[f] : 0.0;
    return (hl + hr) / 3.0;
  }
  if (f - g == 1 || g - f == 1) return (x[std::max(f, g)] - x[std::min(f, g)]) / 6.0;
  return 0.0;
}

}  // namespace

Plan build_plan(int ndim, const uint64_t* shape) {
  Plan p;
  if (ndim < 1) fail(MGC_EINVAL, "ndim must be at least 1");
  if (ndim > 3) fail(MGC_EUNSUPPORTED, "ndim above 3 is not supported");
  if (!shape) fail(MGC_EINVAL, "null shape");
  p.ndim = ndim;
  unsigned __int128 N = 1;
  std::vector<int64_t> act;
  for (int d = 0; d < ndim; ++d) {
    p.shape[d] = shape[d];
    N *= shape[d];
    if (shape[d] > 1) act.push_back((int64_t)shape[d]);
  }
  if (N >= ((unsigned __int128)1 << 32)) fail(MGC_EUNSUPPORTED, "arrays of 2^32 or more values");
  p.N = (int64_t)N;
  if (p.N == 0) act.clear();
  p.D = (int)act.size();
  for (int k = 0; k < 3; ++k) {
    int d = k - (3 - p.D);
    p.n[k] = d >= 0 ? act[d] : 1;
    p.bit[k] = d >= 0 ? d : -1;
  }
  // hierarchy: collect levels finest first
  std::vector<std::array<int64_t, 3>> fine_first{{p.n[0], p.n[1], p.n[2]}};
  std::vector<std::array<std::vector<double>, 3>> coords(1);
  for (int k = 0; k < 3; ++k) {
    coords[0][k].resize(p.n[k]);
    for (int64_t i = 0; i < p.n[k]; ++i) coords[0][k][i] = (double)i;
  }
  if (p.D > 0 && p.N > 0) {
    while (true) {
      auto cur = fine_first.back();
      int64_t mn = INT64_MAX;
      for (int k = 0; k < 3; ++k)
        if (p.bit[k] >= 0) mn = std::min(mn, cur[k]);
      if (mn <= 2) break;
      std::array<int64_t, 3> nxt;
      std::array<std::vector<double>, 3> c;
      for (int k = 0; k < 3; ++k) {
        if (p.bit[k] >= 0) {
          c[k] = coarse_coords(coords.back()[k]);
          nxt[k] = (int64_t)c[k].size();
        } else {
          c[k] = coords.back()[k];
          nxt[k] = cur[k];
        }
      }
      fine_first.push_back(nxt);
      coords.push_back(c);
      if ((int)fine_first.size() > kMaxLevels) fail(MGC_EUNSUPPORTED, "too many levels");
    }
  }
  p.L = (int)fine_first.size() - 1;
  p.sizes.assign(fine_first.rbegin(), fine_first.rend());
  std::reverse(coords.begin(), coords.end());  // coords[l], l = 0..L

  p.lv.resize(p.L + 1);
  int64_t off = 0;
  for (int l = 0; l <= p.L; ++l) {
    PlanLevel& v = p.lv[l];
    for (int k = 0; k < 3; ++k) {
      v.nf[k] = p.sizes[l][k];
      v.nc[k] = l > 0 ? p.sizes[l - 1][k] : p.sizes[l][k];
      const auto& x = coords[l][k];
      double hm = 1.0;
      if (p.bit[k] >= 0 && x.size() > 1) {
        hm = 0.0;
        for (size_t i = 0; i + 1 < x.size(); ++i) hm = std::max(hm, x[i + 1] - x[i]);
      }
      v.hmax[k] = hm;
    }
    v.off = off;
    v.count = l == 0 ? p.points(0) : p.points(l) - p.points(l - 1);
    off += v.count;
    for (int m = 0; m < 8; ++m) v.sub_off[m] = 0;
    if (l >= 1) {
      int64_t acc = 0;
      for (int m = 1; m < (1 << p.D); ++m) {
        v.sub_off[m] = acc;
        int64_t sz = 1;
        for (int k = 0; k < 3; ++k) {
          bool nw = p.bit[k] >= 0 && ((m >> p.bit[k]) & 1);
          sz *= nw ? (v.nf[k] - v.nc[k]) : v.nc[k];
        }
        acc += sz;
      }
      // tables
      for (int k = 0; k < 3; ++k) {
        const int64_t nf = v.nf[k], nc = v.nc[k];
        const auto& xf = coords[l][k];
        const auto& xc = coords[l - 1][k];
        v.t_wl[k] = p.tab.size();
        p.tab.resize(p.tab.size() + nf, 0.0);
        v.t_wr[k] = p.tab.size();
        p.tab.resize(p.tab.size() + nf, 0.0);
        v.t_W[k] = p.tab.size();
        p.tab.resize(p.tab.size() + 5 * nc, 0.0);
        v.t_ta[k] = p.tab.size();
        p.tab.resize(p.tab.size() + nc, 0.0);
        v.t_tm[k] = p.tab.size();
        p.tab.resize(p.tab.size() + nc, 0.0);
        v.t_tc[k] = p.tab.size();
        p.tab.resize(p.tab.size() + nc, 0.0);
        v.t_WP[k] = p.tab.size();
        p.tab.resize(p.tab.size() + 5 * nc, 0.0);
        v.t_Mt[k] = p.tab.size();
        p.tab.resize(p.tab.size() + 3 * nf, 0.0);
        double* wl = &p.tab[v.t_wl[k]];
        double* wr = &p.tab[v.t_wr[k]];
        double* W = &p.tab[v.t_W[k]];
        double* ta = &p.tab[v.t_ta[k]];
        double* tm = &p.tab[v.t_tm[k]];
        double* tc = &p.tab[v.t_tc[k]];
        double* WP = &p.tab[v.t_WP[k]];
        double* Mt = &p.tab[v.t_Mt[k]];
        if (p.bit[k] < 0) {  // inactive axis: identity operators
          W[2] = 1.0;
          tm[0] = 1.0;
          WP[2] = 1.0;
          Mt[1] = 1.0;
          continue;
        }
        for (int64_t i = 0; i < nf; ++i) {
          if (!is_new(i, nf)) continue;
          const double xa = xf[i - 1], xb = xf[i + 1], xi = xf[i];
          wl[i] = (xb - xi) / (xb - xa);
          wr[i] = (xi - xa) / (xb - xa);
        }
        for (int64_t j = 0; j < nc; ++j) {
          const int64_t pj = cpos(j, nf);
          for (int d = -2; d <= 2; ++d) {
            double acc2 = 0.0;
            for (int64_t f = pj - 1; f <= pj + 1; ++f) {
              if (f < 0 || f >= nf) continue;
              double pf;
              if (f == pj) pf = 1.0;
              else if (is_new(f, nf) && f - 1 == pj) pf = wl[f];
              else if (is_new(f, nf) && f + 1 == pj) pf = wr[f];
              else pf = 0.0;
              if (pf != 0.0) acc2 += pf * mass_entry(xf, f, pj + d);
            }
            W[5 * j + d + 2] = acc2;
          }
        }
        // P^T row of coarse node j: its own fine node and the new nodes beside it
        for (int64_t j = 0; j < nc; ++j) {
          const int64_t pj = cpos(j, nf);
          WP[5 * j + 2] = 1.0;
          if (pj - 1 >= 0 && is_new(pj - 1, nf)) WP[5 * j + 1] = wr[pj - 1];
          if (pj + 1 < nf && is_new(pj + 1, nf)) WP[5 * j + 3] = wl[pj + 1];
        }
        // fine mass-matrix rows
        for (int64_t i = 0; i < nf; ++i) {
          Mt[3 * i + 0] = mass_entry(xf, i, i - 1);
          Mt[3 * i + 1] = mass_entry(xf, i, i);
          Mt[3 * i + 2] = mass_entry(xf, i, i + 1);
        }
        // Thomas factors of the coarse mass matrix
        double cprev = 0.0;
        for (int64_t j = 0; j < nc; ++j) {
          const double Hl = j > 0 ? xc[j] - xc[j - 1] : 0.0;
          const double Hr = j < nc - 1 ? xc[j + 1] - xc[j] : 0.0;
          const double a = Hl / 6.0, b = (Hl + Hr) / 3.0, s = Hr / 6.0;
          const double den = j > 0 ? b - a * cprev : b;
          const double mj = 1.0 / den;
          ta[j] = a * mj;  // zero at j = 0
          tm[j] = mj;
          tc[j] = s * mj;  // zero at j = nc - 1
          cprev = tc[j];
        }
      }
    }
  }
  return p;
}

// Device block: the operator tables, the bin factors K_l of both norms, then
// the per-level geometry records (whose table pointers point into the block).
std::vector<uint8_t> plan_device_image(Plan& p, void* base) {
  const size_t n_tab = p.tab.size();
  const size_t k_off = n_tab, k_len = (size_t)p.L + 1;
  const size_t geo_bytes = sizeof(LevelGeom) * ((size_t)p.L + 1);
  const size_t geo_off = ((n_tab + 2 * k_len) * sizeof(double) + 255) & ~size_t(255);
  const size_t total = geo_off + geo_bytes;
  p.d_tab = static_cast<double*>(base);
  std::vector<uint8_t> host(total, 0);
  if (n_tab) std::memcpy(host.data(), p.tab.data(), n_tab * sizeof(double));
  for (int nrm = 0; nrm < 2; ++nrm) {
    const std::vector<double> K = p.bin_factors(nrm == 0 ? MGC_LINF : MGC_L2);
    std::memcpy(host.data() + (k_off + nrm * k_len) * sizeof(double), K.data(),
                k_len * sizeof(double));
    p.d_K[nrm] = p.d_tab + k_off + nrm * k_len;
  }
  p.d_geo = reinterpret_cast<const LevelGeom*>(static_cast<uint8_t*>(base) + geo_off);
  for (int l = 0; l <= p.L; ++l) {
    const LevelGeom g = p.geom(l);
    std::memcpy(host.data() + geo_off + l * sizeof(LevelGeom), &g, sizeof(LevelGeom));
  }
  return host;
}

size_t plan_device_bytes(const Plan& p) {
  const size_t k_len = (size_t)p.L + 1;
  const size_t geo_off = ((p.tab.size() + 2 * k_len) * sizeof(double) + 255) & ~size_t(255);
  return geo_off + sizeof(LevelGeom) * k_len;
}

void upload_plan(Plan& p) {
  if (p.d_tab) return;
  void* mem = nullptr;
  MGC_HIP(hipMalloc(&mem, plan_device_bytes(p)));
  const std::vector<uint8_t> host = plan_device_image(p, mem);
  MGC_HIP(hipMemcpy(mem, host.data(), host.size(), hipMemcpyHostToDevice));
}

void free_plan(Plan& p) {
  if (p.d_tab) (void)hipFree(p.d_tab);
  p.d_tab = nullptr;
}

LevelGeom Plan::geom(int l) const {
  LevelGeom g{};
  const PlanLevel& v = lv[l];
  for (int k = 0; k < 3; ++k) {
    g.nf[k] = v.nf[k];
    g.nc[k] = v.nc[k];
    g.bit[k] = bit[k];
    if (l >= 1) {
      g.ax[k].wl = d_tab + v.t_wl[k];
      g.ax[k].wr = d_tab + v.t_wr[k];
      g.ax[k].W = d_tab + v.t_W[k];
      g.ax[k].ta = d_tab + v.t_ta[k];
      g.ax[k].tm = d_tab + v.t_tm[k];
      g.ax[k].tc = d_tab + v.t_tc[k];
      g.ax[k].WP = d_tab + v.t_WP[k];
      g.ax[k].Mt = d_tab + v.t_Mt[k];
    }
  }
  g.level_off = v.off;
  for (int m = 0; m < 8; ++m) g.sub_off[m] = v.sub_off[m];
  return g;
}

// kappa = ||M_c^{-1} P^T M_l||_inf of one axis of level l: the largest
// absolute row sum of the dense nc x nf matrix, formed one fine column at a
// time (column f of P^T M_l has at most three non-zeros, the restriction taps
// W of the coarse nodes within two fine positions; each column is solved
// with the Thomas factors of M_c), rounded up to a multiple of 2^-20.
double Plan::transfer_norm(int l, int k) const {
  const PlanLevel& v = lv[l];
  const int64_t nf = v.nf[k], nc = v.nc[k];
  const double* W = &tab[v.t_W[k]];
  const double* ta = &tab[v.t_ta[k]];
  const double* tm = &tab[v.t_tm[k]];
  const double* tc = &tab[v.t_tc[k]];
  std::vector<double> rows(nc, 0.0), y(nc), b(nc, 0.0);
  for (int64_t f = 0; f < nf; ++f) {
    // coarse nodes j with |p(j) - f| <= 2 (p(j) = min(2j, nf - 1))
    const int64_t j0 = std::max<int64_t>(0, (f - 2 + 1) / 2), j1 = std::min<int64_t>(nc - 1, (f + 2) / 2 + 1);
    int64_t lo = nc, hi = -1;
    for (int64_t j = j0; j <= j1; ++j) {
      const int64_t d = f - cpos(j, nf);
      if (d < -2 || d > 2) continue;
      b[j] = W[5 * j + d + 2];
      lo = std::min(lo, j);
      hi = std::max(hi, j);
    }
    if (hi < 0) continue;
    // forward sweep from the first non-zero (y is zero before it)
    for (int64_t j = lo; j < nc; ++j) y[j] = tm[j] * b[j] - (j > lo ? ta[j] * y[j - 1] : 0.0);
    double x = 0.0;
    for (int64_t j = nc - 1; j >= 0; --j) {
      x = (j >= lo ? y[j] : 0.0) - (j < nc - 1 ? tc[j] * x : 0.0);
      rows[j] += std::fabs(x);
    }
    for (int64_t j = lo; j <= hi; ++j) b[j] = 0.0;
  }
  double kappa = 0.0;
  for (int64_t j = 0; j < nc; ++j) kappa = std::max(kappa, rows[j]);
  return std::ceil(kappa * 1048576.0) / 1048576.0;
}

// q_l = tau' K_l.
// L-inf: reconstruction error <= sum_l A_l q_l / 2 with A_0 = 1 and
// A_l = 1 + prod over active axes of kappa (the transfer norm above).  The
// budget is split as K_l = 2 sqrt(m_l) / (A_l S), S = sum_j sqrt(m_j) (m_l
// coefficients on level l): the finest level gets the widest bins, and the
// small coarse levels keep their quantised values inside the dictionary
// (bins proportional to m_l / A_l, the split that minimises a log2(1/q)
// bit count, send most coarse-level values to the escape list).
// L2: every level gets an equal share of tau'^2 (see mgc.h).
std::vector<double> Plan::bin_factors(mgc_norm norm) const {
  std::vector<double> K(L + 1);
  int64_t pow6 = 1;
  for (int d = 0; d < D; ++d) pow6 *= 6;
  // L-inf: q_l = 2 tau' sqrt(m_l) / (A_l S), S = sum_j sqrt(m_j) (summed
  // from level 0 up)
  double S = 0.0;
  for (int l = 0; l <= L; ++l) S = S + std::sqrt((double)lv[l].count);
  for (int l = 0; l <= L; ++l) {
    if (norm == MGC_LINF) {
      double A = 1.0;
      if (l >= 1) {
        double prod = 1.0;
        for (int k = 0; k < 3; ++k)
          if (bit[k] >= 0) prod = prod * transfer_norm(l, k);
        A = 1.0 + prod;
      }
      K[l] = (2.0 * std::sqrt((double)lv[l].count)) / (S * A);
    } else {
      double den = (double)pow6 * (double)(L + 1);
      for (int k = 0; k < 3; ++k)
        if (bit[k] >= 0) den = den * lv[l].hmax[k];
      den = den * (double)lv[l].count;
      K[l] = 2.0 / std::sqrt(den);
    }
  }
  return K;
}

}  // namespace mgc
