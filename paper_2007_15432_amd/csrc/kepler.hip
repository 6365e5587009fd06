// kepler.hip -- Kepler drift of particles without neighbours.
//
// Section 2.2 integrates the hard part of a particle that has no neighbour as
// its two-body orbit about the central star, found by Newton-Raphson on
// Kepler's equation.  Over a soft step dt the particle moves on the orbit of
// mu = G M_* (its own mass neglected against the star's).  Written in the
// difference dE of the eccentric anomaly, which needs neither the orbital
// elements nor the anomaly itself:
//
//   r0 = |x0|, 1/a = 2/r0 - |v0|^2/mu (bound: 1/a > 0 and finite),
//   n = sqrt(mu / a^3), ec = 1 - r0/a (= e cos E0), es = x0.v0 / sqrt(mu a) (= e sin E0),
//   Kepler's equation  dE - ec sin dE + es (1 - cos dE) = n dt, Newton from dE = n dt,
//   r = a (1 - ec cos dE + es sin dE),
//   f = 1 - (a/r0)(1 - cos dE),  g = dt + (sin dE - dE)/n,
//   fd = -a^2 n sin dE / (r r0),  gd = 1 - (a/r)(1 - cos dE),
//   x = f x0 + g v0,  v = fd x0 + gd v0.
//
// One thread per listed particle, FP64 throughout; the kernel reads and writes
// 48 B of state per particle (plus the 4 B index when a list is given), so it
// is bound by HBM, with a handful of sincos per particle on top.  Orbits that
// are not bound are left as they are, flagged -1 in the iteration output and
// counted in the device counters; so are list entries outside [0, n) (-2).
#include <algorithm>

#include "p3t_internal.h"

namespace p3t {

constexpr int KEPLER_MAX_ITER = 50;
constexpr double KEPLER_TOL = 1e-15;

// Drift particle i for dt about mu; returns the Newton iterations, or -1
// (state unchanged) when the orbit is not bound.
__device__ __forceinline__ int drift_one(int64_t n, int64_t i, double mu, double dt, double *__restrict__ pos,
                                         double *__restrict__ vel) {
  double x0[3], v0[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    x0[d] = pos[d * n + i];
    v0[d] = vel[d * n + i];
  }
  const double r0 = sqrt(x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2]);
  const double v2 = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2];
  const double inv_a = 2.0 / r0 - v2 / mu;
  if (!(inv_a > 0.0) || !(inv_a < INFINITY)) return -1;
  const double a = 1.0 / inv_a;
  const double nm = sqrt(mu / (a * a * a));
  const double ec = 1.0 - r0 / a;
  const double es = (x0[0] * v0[0] + x0[1] * v0[1] + x0[2] * v0[2]) / sqrt(mu * a);
  const double M = nm * dt;
  double dE = M, s, c;
  int it = 0;
  bool conv = false;
  while (it < KEPLER_MAX_ITER) {
    sincos(dE, &s, &c);
    const double F = dE - ec * s + es * (1.0 - c) - M;
    const double Fp = 1.0 - ec * c + es * s;
    const double step = F / Fp;
    dE -= step;
    ++it;
    if (!(fabs(step) > KEPLER_TOL * fmax(1.0, fabs(dE)))) {
      // the last step is below 1e-15 relative: rotate (s, c) by it instead of
      // a new sincos (the neglected terms are of order step^2)
      const double s1 = s - c * step;
      c += s * step;
      s = s1;
      conv = true;
      break;
    }
  }
  if (!conv) sincos(dE, &s, &c);
  const double r = a * (1.0 - ec * c + es * s);
  const double f = 1.0 - (a / r0) * (1.0 - c);
  const double g = dt + (s - dE) / nm;
  const double fd = -a * a * nm * s / (r * r0);
  const double gd = 1.0 - (a / r) * (1.0 - c);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    pos[d * n + i] = f * x0[d] + g * v0[d];
    vel[d * n + i] = fd * x0[d] + gd * v0[d];
  }
  return it;
}

__global__ __launch_bounds__(256) void k_kepler(int64_t n, int64_t n_list, const int32_t *__restrict__ list,
                                                double mu, double dt, double *__restrict__ pos,
                                                double *__restrict__ vel, int32_t *__restrict__ iters,
                                                DevCounters *__restrict__ cnt) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_list; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = list ? (int64_t)list[k] : k;
    if (i < 0 || i >= n) {  // a list entry out of range: skipped, counted
      if (iters) iters[k] = -2;
      atomicAdd(&cnt->n_bad_index, 1ull);
      continue;
    }
    const int it = drift_one(n, i, mu, dt, pos, vel);
    if (it < 0) atomicAdd(&cnt->n_unbound, 1ull);
    if (iters) iters[k] = it;
  }
}

// The clusters of one member inside the hard part: cluster ids from the
// size-bucket list, the member from the cluster CSR (both validated by the
// bucketing pass).  The carried hard step is cleared (a particle that joins a
// cluster later starts from the initial step criterion); the per-particle and
// per-cluster step counts read one step, the energy error zero.  An orbit
// that is not bound is left in place and flagged.
__global__ __launch_bounds__(256) void k_kepler_single(int64_t n, int32_t count, const int32_t *__restrict__ blist,
                                                       const int32_t *__restrict__ cl_ptr,
                                                       const int32_t *__restrict__ members, double mu, double dt,
                                                       double *__restrict__ pos, double *__restrict__ vel,
                                                       double *__restrict__ dt_hard, int32_t *__restrict__ msteps,
                                                       double *__restrict__ e_rel, int32_t *__restrict__ nsteps,
                                                       DevCounters *__restrict__ cnt) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) {
    const int cl = blist[k];
    const int64_t i = members[cl_ptr[cl]];
    const int it = drift_one(n, i, mu, dt, pos, vel);
    if (it < 0) set_flag(cnt, P3T_FLAG_UNBOUND);
    if (dt_hard) dt_hard[i] = 0.0;
    if (msteps) msteps[i] = 1;
    if (e_rel) e_rel[cl] = 0.0;
    if (nsteps) nsteps[cl] = 1;
  }
}

hipError_t kepler_singles(int64_t n, int32_t count, const int32_t *blist, const int32_t *cl_ptr,
                          const int32_t *members, double mu, double dt, double *pos3, double *vel3, double *dt_hard,
                          int32_t *msteps, double *e_rel, int32_t *nsteps, DevCounters *cnt, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int blocks = std::min(((int)count + 255) / 256, 65536);
  hipLaunchKernelGGL(k_kepler_single, dim3(blocks), dim3(256), 0, s, n, count, blist, cl_ptr, members, mu, dt, pos3,
                     vel3, dt_hard, msteps, e_rel, nsteps, cnt);
  return hipGetLastError();
}

hipError_t kepler_drift(int64_t n, int64_t n_list, const int32_t *list, double mu, double dt, double *pos3,
                        double *vel3, int32_t *iters, DevCounters *cnt, hipStream_t s) {
  if (n_list <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n_list + 255) / 256, 65536);
  hipLaunchKernelGGL(k_kepler, dim3((unsigned)blocks), dim3(256), 0, s, n, n_list, list, mu, dt, pos3, vel3, iters,
                     cnt);
  return hipGetLastError();
}

}  // namespace p3t
