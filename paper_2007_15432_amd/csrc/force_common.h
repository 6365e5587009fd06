// force_common.h -- arguments of the force kernels and the exact neighbour
// test shared by the fused and the split force kernels.
#pragma once
#include "p3t_internal.h"

namespace p3t {

struct ForceArgs {
  const double *sx, *sy, *sz, *sm, *sinv, *sreach, *svx, *svy, *svz, *srs, *sro;
  const int32_t *sid;
  const WalkNode *wn;
  const CellMom *cm;
  const GroupList *gl;
  const int32_t *order;
  const int32_t *pool;
  DevCounters *cnt;
  int2 *pairs;
  int64_t pair_cap;
  int2 *cands;  // neighbour candidates (sorted indices), split form
  const uint8_t *slow;  // caller's order: pairs with a flagged member are not reported (nullable)
  int64_t cand_cap;
  int cand_slab;  // candidate slots a wavefront reserves at a time (0: exactly each tile's)
  double *acc;
  int64_t n;
  double G, gamma, inv1mg;
  double rsch2, rsch3, dt;  // neighbour-test parameters
  int persistent;
  int ngroups_bound;          // groups processed at most (the host's bound; the count itself is on the device)
  unsigned long long *queue;  // persistent-queue head of this launch
  uint8_t *close;             // caller's order: set for both members of a close neighbour pair (nullable)
  double close_k;             // G dt_soft^2 / CLOSE_RATIO^2
};

// Flags both members of the neighbour pair (i, j) (sorted indices) when
// its free-fall time scale is short against the soft step: (m_i + m_j)
// close_k >= r^3.  Steers only the dispatch order of the next hard part.
__device__ __forceinline__ void mark_close_pair(const ForceArgs &A, int i, int j) {
  if (!A.close) return;
  const double dx = A.sx[j] - A.sx[i], dy = A.sy[j] - A.sy[i], dz = A.sz[j] - A.sz[i];
  const double r2 = dx * dx + dy * dy + dz * dz;
  if ((A.sm[i] + A.sm[j]) * A.close_k >= r2 * sqrt(r2)) {
    A.close[A.sid[i]] = 1;
    A.close[A.sid[j]] = 1;
  }
}

// the split form (one kernel per interaction class), force_split.hip
hipError_t soft_force_split(p3t_ctx *c, const ForceArgs &A, unsigned nonpersistent_grid, double *acc3);

// Neighbour test of Section 2.3 (closest approach over the step compared
// with Rsearch2 r_out,ij, or slow pair), in a fixed division- and root-free
// FP64 operation order, contraction disabled, so that every decision is
// reproducible bit for bit.
__device__ __forceinline__ bool neighbour_test(double xi, double yi, double zi, double vxi, double vyi, double vzi,
                                               double mi, double roi, double rsi, double xj, double yj, double zj,
                                               double vxj, double vyj, double vzj, double mj, double roj, double rsj,
                                               double G, double rsch2, double rsch3, double dt) {
#pragma clang fp contract(off)
  const double dx = xi - xj, dy = yi - yj, dz = zi - zj;
  const double ux = vxi - vxj, uy = vyi - vyj, uz = vzi - vzj;
  const double rr = ((dx * dx) + (dy * dy)) + (dz * dz);
  const double rs = rsi > rsj ? rsi : rsj;
  if (!(rr < rs * rs)) return false;
  const double rv = ((dx * ux) + (dy * uy)) + (dz * uz);
  const double vv = ((ux * ux) + (uy * uy)) + (uz * uz);
  const double ro = roi > roj ? roi : roj;
  const double R2 = rsch2 * ro;
  const double RR = R2 * R2;
  bool close;
  if (vv == 0.0 || rv >= 0.0) {
    close = rr <= RR;
  } else if (-rv < dt * vv) {
    close = (rr * vv - rv * rv) <= RR * vv;
  } else {
    close = (rr + (2.0 * dt) * rv) + (dt * dt) * vv <= RR;
  }
  if (close) return true;
  const double A = (rsch3 * (G * (mi + mj))) * (0.5 * dt);
  return vv * (rr * rr) < A * A;
}

__device__ __forceinline__ void two_sum_acc(float &hi, float &lo, float v) {
  const float s = hi + v;
  const float bp = s - hi;
  const float err = (hi - (s - bp)) + (v - bp);
  hi = s;
  lo += err;
}

// the next group index of a persistent launch (every lane executes the
// atomic; lane 0's ticket is broadcast through a scalar register)
__device__ __forceinline__ int next_group(unsigned long long *queue, int lane) {
  return (int)wave_fetch_add(queue, 1ull);
}

}  // namespace p3t
