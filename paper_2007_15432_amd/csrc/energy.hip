// energy.hip -- total energy of the planetesimals about the star, the
// quantity whose relative change over a run measures a P3T integration's
// error (Section 3.2.1).  eq. (soft) + eq. (hard) summed over all particles:
// the changeover weights of every pair add up to one (W + (1 - W)), so the
// sum is the Newtonian energy
//   E = sum_i [ m_i |v_i|^2 / 2 - G M_* m_i / |x_i| ] - sum_{i<j} G m_i m_j / r_ij.
// Direct O(N^2) in FP64 (a diagnostic for runs of modest N): each particle's
// share e_i = kinetic + star - (1/2) sum_{j != i} G m_i m_j / r_ij is summed
// over j tiles staged in LDS, then the shares are added in a fixed order.
// Every sum is compensated (Neumaier), so the result carries the rounding of
// a few operations rather than of N of them: relative changes down to
// 1e-15 of E stay visible.
#include "p3t_internal.h"

namespace p3t {

namespace {

constexpr int EN_T = 256;

// s + v with the rounding error kept in c (Neumaier's variant of Kahan's
// compensated summation)
__device__ __forceinline__ void csum(double &s, double &c, double v) {
  const double t = s + v;
  c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
  s = t;
}

__global__ __launch_bounds__(EN_T) void k_energy_share(int64_t n, const double *__restrict__ pos,
                                                       const double *__restrict__ vel, const double *__restrict__ m,
                                                       double G, double GM, double *__restrict__ share) {
  __shared__ double tx[EN_T], ty[EN_T], tz[EN_T], tm[EN_T];
  const int t = threadIdx.x;
  for (int64_t b0 = (int64_t)blockIdx.x * EN_T; b0 < n; b0 += (int64_t)gridDim.x * EN_T) {  // uniform per block
    const int64_t i = b0 + t;
    const bool act = i < n;
    const int64_t ic = act ? i : 0;
    const double xi = pos[ic], yi = pos[n + ic], zi = pos[2 * n + ic];
    double s = 0.0, c = 0.0;  // sum_j m_j / r_ij
    for (int64_t j0 = 0; j0 < n; j0 += EN_T) {
      const int64_t j = j0 + t;
      __syncthreads();
      if (j < n) {
        tx[t] = pos[j];
        ty[t] = pos[n + j];
        tz[t] = pos[2 * n + j];
        tm[t] = m[j];
      }
      __syncthreads();
      const int cnt = (int)(n - j0 < EN_T ? n - j0 : EN_T);
      if (act) {
        for (int k = 0; k < cnt; ++k) {
          if (j0 + k == i) continue;
          const double dx = tx[k] - xi, dy = ty[k] - yi, dz = tz[k] - zi;
          csum(s, c, tm[k] / sqrt(dx * dx + dy * dy + dz * dz));
        }
      }
    }
    if (act) {
      const double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i], mi = m[i];
      double e = 0.0, ec = 0.0;
      csum(e, ec, 0.5 * mi * (vx * vx + vy * vy + vz * vz));
      csum(e, ec, -GM * mi / sqrt(xi * xi + yi * yi + zi * zi));
      csum(e, ec, -0.5 * G * mi * s);
      csum(e, ec, -0.5 * G * mi * c);
      share[i] = e + ec;
    }
  }
}

// the shares added in a fixed order: thread t takes t, t + EN_T, ...; then the
// partials in thread order
__global__ __launch_bounds__(EN_T) void k_energy_sum(int64_t n, const double *__restrict__ share,
                                                     double *__restrict__ out) {
  __shared__ double ps[EN_T], pc[EN_T];
  const int t = threadIdx.x;
  double s = 0.0, c = 0.0;
  for (int64_t i = t; i < n; i += EN_T) csum(s, c, share[i]);
  ps[t] = s;
  pc[t] = c;
  __syncthreads();
  if (t == 0) {
    double S = 0.0, C = 0.0;
    for (int k = 0; k < EN_T; ++k) csum(S, C, ps[k]);
    for (int k = 0; k < EN_T; ++k) C += pc[k];
    out[0] = S + C;
  }
}

}  // namespace

hipError_t total_energy(int64_t n, const double *pos3, const double *vel3, const double *mass, double G, double GM,
                        double *share, double *out, hipStream_t s) {
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (n + EN_T - 1) / EN_T));
  hipLaunchKernelGGL(k_energy_share, dim3(g), dim3(EN_T), 0, s, n, pos3, vel3, mass, G, GM, share);
  hipLaunchKernelGGL(k_energy_sum, dim3(1), dim3(EN_T), 0, s, n, share, out);
  return hipGetLastError();
}

}  // namespace p3t
