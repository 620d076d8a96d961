// Host-side plan of one array shape: level hierarchy, per-axis operator
// tables, subband offsets and the quantisation-bin factors.
#pragma once

#include <array>
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace mgc {

struct PlanLevel {
  int64_t nf[3], nc[3];   // internal-axis sizes of level l and l-1 (l >= 1)
  int64_t off;            // stream offset of the level
  int64_t count;          // entries contributed (level 0: all nodes)
  int64_t sub_off[8];
  double hmax[3];         // largest spacing on each internal axis at level l
  size_t t_wl[3], t_wr[3], t_W[3], t_ta[3], t_tm[3], t_tc[3], t_WP[3], t_Mt[3];  // table offsets
};

struct Plan {
  int ndim = 0;
  uint64_t shape[3] = {0, 0, 0};   // user shape (unused entries 0)
  int64_t n[3] = {1, 1, 1};         // internal shape: squeezed axes first
  int D = 0;                         // active axes (length > 1)
  int L = 0;
  int64_t N = 0;
  int bit[3] = {-1, -1, -1};
  std::vector<std::array<int64_t, 3>> sizes;  // sizes[l], l = 0..L
  std::vector<PlanLevel> lv;                   // lv[l], l = 0..L
  std::vector<double> tab;                     // host copy of every table
  double* d_tab = nullptr;                     // device block (owned): tables, K, geometry
  const double* d_K[2] = {nullptr, nullptr};   // bin factors (L-inf, L2), L + 1 each
  const LevelGeom* d_geo = nullptr;            // d_geo[l], l = 0..L

  int64_t points(int l) const { return sizes[l][0] * sizes[l][1] * sizes[l][2]; }
  LevelGeom geom(int l) const;
  // q_l = tau_eff * K_l with K_l from the L-inf or L2 budget split.
  std::vector<double> bin_factors(mgc_norm norm) const;
  // ||M_{l-1}^{-1} P^T M_l||_inf of internal axis k (active) of level l >= 1,
  // rounded up to a multiple of 2^-20.
  double transfer_norm(int l, int k) const;
};

// Builds the plan (host tables only).  Throws Fail on invalid shapes.
Plan build_plan(int ndim, const uint64_t* shape);
void upload_plan(Plan& p);
// The plan's device block as host bytes, with every device pointer of the
// plan (tables, bin factors, geometry) set to point into a block at `base`;
// plan_device_bytes is its size.  upload_plan = allocate, image, copy.
std::vector<uint8_t> plan_device_image(Plan& p, void* base);
size_t plan_device_bytes(const Plan& p);
void free_plan(Plan& p);


}  // namespace mgc
