// hermite.hip -- fourth-order Hermite integration of neighbour clusters over
// one soft step with block time steps (Section 2.1.1; step (5) of the
// procedure in Section 2.2; eta, eta_0 of Section 3.1).
//
// Per cluster: forces from the central star and every intra-cluster pair
// with (1 - K) (eq. (hardforce)), jerk including dK/dt; steps dt_soft 2^-k
// with integer time in ticks of dt_soft 2^-40; each block step predicts all
// members, evaluates the active ones, corrects once; new steps from Aarseth's
// criterion, quantised down, growing at most twofold and only on a multiple
// of the doubled step.  Energy of eq. (hard) restricted to the cluster before
// and after.
//
// Clusters are bucketed by size.  Sizes <= 64: SEG lanes per cluster
// (SEG = next power of two), 64/SEG clusters per wavefront, one member per
// lane, reductions by shuffles inside the segment.  Sizes 65..1024: one
// 256-thread workgroup per cluster, MPT members per thread, block reductions
// in LDS.  Predicted states are shared through LDS.
#include <climits>

#include "p3t_internal.h"

namespace p3t {

constexpr int TICK_BITS = 40;
constexpr int BIG_T = 256;
constexpr int N_BUCKETS = 11;  // SEG 1..64 (7), big MPT 1, 2, 4 (3), too big (1)

struct HermArgs {
  const int32_t *cl_ptr, *members, *blist;
  int nb;
  double *pos, *vel;
  const double *mass, *ro;
  double *dt_hard, *e_rel;
  int32_t *nsteps;
  int64_t n;
  double G, GM, gamma, inv1mg, eta, eta0, dt_soft, tick;
  int k_max, max_iter;
  double wc, wf1, wlog;
  double wp[8];  // f(y) = sum_k wp[k] y^k + wlog y ln y   (eq. (cutfuncW))
  DevCounters *cnt;
};

__device__ __forceinline__ double changeover_W(double y, const HermArgs &A) {
  if (y < A.gamma) return A.wc * y;
  if (y >= 1.0) return 1.0;
  double p = A.wp[7];
#pragma unroll
  for (int k = 6; k >= 0; --k) p = p * y + A.wp[k];
  return p + A.wlog * y * log(y) + (1.0 - A.wf1) * y;
}

// hard pair term on i from j: d = x_j - x_i, u = v_j - v_i
__device__ __forceinline__ void hard_pair(double dx, double dy, double dz, double ux, double uy, double uz, double gmj,
                                          double invR, const HermArgs &A, double *a, double *jk) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double rinv = rsqrt(r2);
  const double y = r2 * rinv * invR;
  const double x = fmin(fmax((y - A.gamma) * A.inv1mg, 0.0), 1.0);
  const double x2 = x * x, x3 = x2 * x;
  const double K = x2 * x2 * (35.0 + x * (-84.0 + x * (70.0 - 20.0 * x)));
  const double omx = 1.0 - x;
  const double Ky = (x > 0.0 && x < 1.0) ? 140.0 * x3 * omx * omx * omx * A.inv1mg : 0.0;
  const double s = dx * ux + dy * uy + dz * uz;
  const double rinv2 = rinv * rinv;
  const double rinv3 = rinv * rinv2;
  const double w = gmj * (1.0 - K) * rinv3;
  const double c1 = 3.0 * s * rinv2;
  const double c2 = gmj * Ky * s * rinv * invR * rinv3;
  a[0] += w * dx;
  a[1] += w * dy;
  a[2] += w * dz;
  jk[0] += w * (ux - c1 * dx) - c2 * dx;
  jk[1] += w * (uy - c1 * dy) - c2 * dy;
  jk[2] += w * (uz - c1 * dz) - c2 * dz;
}

__device__ __forceinline__ void star_term(const double *x, const double *v, double GM, double *a, double *jk) {
  const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  const double rinv = rsqrt(r2);
  const double rinv3 = rinv * rinv * rinv;
  const double xv = x[0] * v[0] + x[1] * v[1] + x[2] * v[2];
  const double c5 = 3.0 * xv * rinv * rinv;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    a[d] = -GM * x[d] * rinv3;
    jk[d] = -GM * (v[d] - c5 * x[d]) * rinv3;
  }
}

__device__ __forceinline__ int level_for(double dt_soft, double dtc, int kmax) {
  int k = 0;
  while (k <= kmax && ldexp(dt_soft, -k) > dtc) ++k;
  return k;
}

__device__ __forceinline__ double norm3(const double *a) { return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

// corrector + new level for one active member
__device__ __forceinline__ void correct(double *x, double *v, double *a0, double *j0, const double *xp, const double *vp,
                                        const double *a1, const double *j1, double h, int64_t tnew, int &lev,
                                        const HermArgs &A) {
  double a2[3], a3[3];
  const double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double da = a0[d] - a1[d];
    a2[d] = (-6.0 * da - h * (4.0 * j0[d] + 2.0 * j1[d])) / h2;
    a3[d] = (12.0 * da + 6.0 * h * (j0[d] + j1[d])) / h3;
    x[d] = xp[d] + a2[d] * h4 / 24.0 + a3[d] * h5 / 120.0;
    v[d] = vp[d] + a2[d] * h3 / 6.0 + a3[d] * h4 / 24.0;
    a0[d] = a1[d];
    j0[d] = j1[d];
  }
  const double a2e[3] = {a2[0] + a3[0] * h, a2[1] + a3[1] * h, a2[2] + a3[2] * h};
  const double an = norm3(a1), jn = norm3(j1), a2n = norm3(a2e), a3n = norm3(a3);
  const double den = jn * a3n + a2n * a2n;
  const double dtc = den > 0.0 ? sqrt(A.eta * (an * a2n + jn * jn) / den) : A.dt_soft;
  const int knew = level_for(A.dt_soft, dtc, A.k_max);
  int k = lev;
  if (knew < k) {
    const int64_t dbl = (int64_t)1 << (TICK_BITS - k + 1);
    if (k > 0 && (tnew % dbl) == 0) k = k - 1;
  } else {
    k = knew;
  }
  if (k > A.k_max) {
    set_flag(A.cnt, P3T_FLAG_KMAX);
    k = A.k_max;
  }
  lev = k;
}

template <typename T, int SEG>
__device__ __forceinline__ T seg_min(T v) {
#pragma unroll
  for (int o = SEG / 2; o > 0; o >>= 1) {
    T t = __shfl_xor(v, o, SEG);
    v = t < v ? t : v;
  }
  return v;
}
template <int SEG>
__device__ __forceinline__ double seg_sum(double v) {
#pragma unroll
  for (int o = SEG / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, SEG);
  return v;
}

// ---------------------------------------------------------------- small clusters
template <int SEG>
__global__ __launch_bounds__(WAVE) void k_herm_seg(HermArgs A) {
  __shared__ double px[WAVE], py[WAVE], pz[WAVE], pvx[WAVE], pvy[WAVE], pvz[WAVE], pgm[WAVE], pinv[WAVE];
  const int lane = threadIdx.x, seg = lane / SEG, sl = lane % SEG, sb = seg * SEG;
  const int ci = blockIdx.x * (WAVE / SEG) + seg;
  const int c = ci < A.nb ? A.blist[ci] : -1;
  const int b = c >= 0 ? A.cl_ptr[c] : 0;
  const int size = c >= 0 ? A.cl_ptr[c + 1] - b : 0;
  const bool mem = sl < size;
  const int gid = mem ? A.members[b + sl] : 0;
  const int64_t n = A.n;
  double x[3] = {1.0, 0.0, 0.0}, v[3] = {0.0, 1.0, 0.0}, a0[3], j0[3];
  double m = 0.0, ro = 1.0;
  if (mem) {
    x[0] = A.pos[gid];
    x[1] = A.pos[n + gid];
    x[2] = A.pos[2 * n + gid];
    v[0] = A.vel[gid];
    v[1] = A.vel[n + gid];
    v[2] = A.vel[2 * n + gid];
    m = A.mass[gid];
    ro = A.ro[gid];
  }
  pgm[lane] = A.G * m;
  pinv[lane] = 1.0 / ro;
  px[lane] = x[0];
  py[lane] = x[1];
  pz[lane] = x[2];
  pvx[lane] = v[0];
  pvy[lane] = v[1];
  pvz[lane] = v[2];
  __syncthreads();
  const double invi = 1.0 / ro;
  // forces at t = 0 and the initial energy
  star_term(x, v, A.GM, a0, j0);
  double e = mem ? 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - A.GM * m * rsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) : 0.0;
  for (int jj = 0; jj < size; ++jj) {
    if (jj == sl || !mem) continue;
    const int q = sb + jj;
    const double dx = px[q] - x[0], dy = py[q] - x[1], dz = pz[q] - x[2];
    const double invR = fmin(invi, pinv[q]);
    hard_pair(dx, dy, dz, pvx[q] - v[0], pvy[q] - v[1], pvz[q] - v[2], pgm[q], invR, A, a0, j0);
    if (jj > sl) {
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      e -= m * pgm[q] * (1.0 - changeover_W(r * invR, A)) / r;
    }
  }
  const double E0 = seg_sum<SEG>(e);
  int lev = 0;
  {
    double dtc = A.dt_soft;
    const double an = norm3(a0), jn = norm3(j0);
    if (jn > 0.0) dtc = A.eta0 * an / jn;
    if (mem && A.dt_hard && A.dt_hard[gid] > 0.0) dtc = A.dt_hard[gid];
    lev = level_for(A.dt_soft, dtc, A.k_max);
    if (lev > A.k_max) {
      if (mem) set_flag(A.cnt, P3T_FLAG_KMAX);
      lev = A.k_max;
    }
  }
  const int64_t T = (int64_t)1 << TICK_BITS;
  int64_t t = 0;
  int nst = 0;  // block steps of this lane's cluster
  for (int it = 0;; ++it) {
    const int64_t te = mem ? t + ((int64_t)1 << (TICK_BITS - lev)) : LLONG_MAX;
    const int64_t tn = seg_min<int64_t, SEG>(te);
    const int64_t tlow = seg_min<int64_t, SEG>(mem ? t : T);
    const bool done = (size == 0) || (tlow == T);
    if (__all(done)) break;
    if (it >= A.max_iter) {
      if (lane == 0) set_flag(A.cnt, P3T_FLAG_NSTEPS);
      break;
    }
    const bool active = mem && !done && te == tn;
    nst += done ? 0 : 1;
    double xp[3], vp[3];
    if (mem && !done) {
      const double dl = (double)(tn - t) * A.tick;
      const double d2 = dl * dl / 2.0, d3 = dl * dl * dl / 6.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        xp[d] = x[d] + v[d] * dl + a0[d] * d2 + j0[d] * d3;
        vp[d] = v[d] + a0[d] * dl + j0[d] * d2;
      }
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        xp[d] = x[d];
        vp[d] = v[d];
      }
    }
    __syncthreads();
    px[lane] = xp[0];
    py[lane] = xp[1];
    pz[lane] = xp[2];
    pvx[lane] = vp[0];
    pvy[lane] = vp[1];
    pvz[lane] = vp[2];
    __syncthreads();
    if (active) {
      double a1[3], j1[3];
      star_term(xp, vp, A.GM, a1, j1);
      for (int jj = 0; jj < size; ++jj) {
        if (jj == sl) continue;
        const int q = sb + jj;
        hard_pair(px[q] - xp[0], py[q] - xp[1], pz[q] - xp[2], pvx[q] - vp[0], pvy[q] - vp[1], pvz[q] - vp[2],
                  pgm[q], fmin(invi, pinv[q]), A, a1, j1);
      }
      const double h = (double)(tn - t) * A.tick;
      t = tn;
      correct(x, v, a0, j0, xp, vp, a1, j1, h, t, lev, A);
    }
  }
  // final energy
  __syncthreads();
  px[lane] = x[0];
  py[lane] = x[1];
  pz[lane] = x[2];
  pvx[lane] = v[0];
  pvy[lane] = v[1];
  pvz[lane] = v[2];
  __syncthreads();
  e = mem ? 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - A.GM * m * rsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) : 0.0;
  for (int jj = sl + 1; jj < size; ++jj) {
    if (!mem) break;
    const int q = sb + jj;
    const double dx = px[q] - x[0], dy = py[q] - x[1], dz = pz[q] - x[2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    e -= m * pgm[q] * (1.0 - changeover_W(r * fmin(invi, pinv[q]), A)) / r;
  }
  const double E1 = seg_sum<SEG>(e);
  if (mem) {
    A.pos[gid] = x[0];
    A.pos[n + gid] = x[1];
    A.pos[2 * n + gid] = x[2];
    A.vel[gid] = v[0];
    A.vel[n + gid] = v[1];
    A.vel[2 * n + gid] = v[2];
    if (A.dt_hard) A.dt_hard[gid] = ldexp(A.dt_soft, -lev);
    if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))) set_flag(A.cnt, P3T_FLAG_NAN);
  }
  if (sl == 0 && c >= 0 && A.e_rel) A.e_rel[c] = fabs(E1 - E0) / fabs(E0);
  if (sl == 0 && c >= 0 && A.nsteps) A.nsteps[c] = nst;
}

// ---------------------------------------------------------------- big clusters
__device__ __forceinline__ int64_t block_min_i64(int64_t v, int64_t *sh) {
  v = wave_min(v);
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[w] = v;
  __syncthreads();
  int64_t r = sh[0];
  for (int q = 1; q < BIG_T / WAVE; ++q) r = sh[q] < r ? sh[q] : r;
  return r;
}
__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int q = 0; q < BIG_T / WAVE; ++q) r += sh[q];
  return r;
}

template <int MPT>
__global__ __launch_bounds__(BIG_T) void k_herm_big(HermArgs A) {
  constexpr int CAP = BIG_T * MPT;
  __shared__ double px[CAP], py[CAP], pz[CAP], pvx[CAP], pvy[CAP], pvz[CAP], pgm[CAP], pinv[CAP];
  __shared__ int64_t shi[BIG_T / WAVE];
  __shared__ double shd[BIG_T / WAVE];
  const int tid = threadIdx.x;
  const int c = blockIdx.x < (unsigned)A.nb ? A.blist[blockIdx.x] : -1;
  if (c < 0) return;  // whole block uniform
  const int b = A.cl_ptr[c];
  const int size = A.cl_ptr[c + 1] - b;
  const int64_t n = A.n;
  double x[MPT][3], v[MPT][3], a0[MPT][3], j0[MPT][3], m[MPT], invi[MPT];
  int64_t t[MPT];
  int lev[MPT], gid[MPT];
  bool mem[MPT];
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int k = tid + BIG_T * u;
    mem[u] = k < size;
    gid[u] = mem[u] ? A.members[b + k] : 0;
    x[u][0] = 1.0;
    x[u][1] = x[u][2] = 0.0;
    v[u][0] = v[u][2] = 0.0;
    v[u][1] = 1.0;
    m[u] = 0.0;
    double ro = 1.0;
    if (mem[u]) {
      for (int d = 0; d < 3; ++d) {
        x[u][d] = A.pos[d * n + gid[u]];
        v[u][d] = A.vel[d * n + gid[u]];
      }
      m[u] = A.mass[gid[u]];
      ro = A.ro[gid[u]];
    }
    invi[u] = 1.0 / ro;
    px[k] = x[u][0];
    py[k] = x[u][1];
    pz[k] = x[u][2];
    pvx[k] = v[u][0];
    pvy[k] = v[u][1];
    pvz[k] = v[u][2];
    pgm[k] = A.G * m[u];
    pinv[k] = invi[u];
    t[u] = 0;
  }
  __syncthreads();
  double e = 0.0;
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int k = tid + BIG_T * u;
    star_term(x[u], v[u], A.GM, a0[u], j0[u]);
    if (!mem[u]) continue;
    e += 0.5 * m[u] * (v[u][0] * v[u][0] + v[u][1] * v[u][1] + v[u][2] * v[u][2]) -
         A.GM * m[u] * rsqrt(x[u][0] * x[u][0] + x[u][1] * x[u][1] + x[u][2] * x[u][2]);
    for (int q = 0; q < size; ++q) {
      if (q == k) continue;
      const double dx = px[q] - x[u][0], dy = py[q] - x[u][1], dz = pz[q] - x[u][2];
      const double invR = fmin(invi[u], pinv[q]);
      hard_pair(dx, dy, dz, pvx[q] - v[u][0], pvy[q] - v[u][1], pvz[q] - v[u][2], pgm[q], invR, A, a0[u], j0[u]);
      if (q > k) {
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        e -= m[u] * pgm[q] * (1.0 - changeover_W(r * invR, A)) / r;
      }
    }
    double dtc = A.dt_soft;
    const double an = norm3(a0[u]), jn = norm3(j0[u]);
    if (jn > 0.0) dtc = A.eta0 * an / jn;
    if (A.dt_hard && A.dt_hard[gid[u]] > 0.0) dtc = A.dt_hard[gid[u]];
    lev[u] = level_for(A.dt_soft, dtc, A.k_max);
    if (lev[u] > A.k_max) {
      set_flag(A.cnt, P3T_FLAG_KMAX);
      lev[u] = A.k_max;
    }
  }
#pragma unroll
  for (int u = 0; u < MPT; ++u)
    if (!mem[u]) lev[u] = 0;
  const double E0 = block_sum(e, shd);
  const int64_t T = (int64_t)1 << TICK_BITS;
  int it = 0;  // block steps taken
  for (;; ++it) {
    int64_t tel = LLONG_MAX, tlow = T;
#pragma unroll
    for (int u = 0; u < MPT; ++u)
      if (mem[u]) {
        const int64_t te = t[u] + ((int64_t)1 << (TICK_BITS - lev[u]));
        tel = te < tel ? te : tel;
        tlow = t[u] < tlow ? t[u] : tlow;
      }
    const int64_t tn = uniform_first64(block_min_i64(tel, shi));
    const int64_t tl = uniform_first64(block_min_i64(tlow, shi));
    if (tl == T) break;
    if (it >= A.max_iter) {
      if (tid == 0) set_flag(A.cnt, P3T_FLAG_NSTEPS);
      break;
    }
    double xp[MPT][3], vp[MPT][3];
#pragma unroll
    for (int u = 0; u < MPT; ++u) {
      const double dl = mem[u] ? (double)(tn - t[u]) * A.tick : 0.0;
      const double d2 = dl * dl / 2.0, d3 = dl * dl * dl / 6.0;
      for (int d = 0; d < 3; ++d) {
        xp[u][d] = x[u][d] + v[u][d] * dl + a0[u][d] * d2 + j0[u][d] * d3;
        vp[u][d] = v[u][d] + a0[u][d] * dl + j0[u][d] * d2;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MPT; ++u) {
      const int k = tid + BIG_T * u;
      px[k] = xp[u][0];
      py[k] = xp[u][1];
      pz[k] = xp[u][2];
      pvx[k] = vp[u][0];
      pvy[k] = vp[u][1];
      pvz[k] = vp[u][2];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MPT; ++u) {
      const int k = tid + BIG_T * u;
      if (!mem[u] || t[u] + ((int64_t)1 << (TICK_BITS - lev[u])) != tn) continue;
      double a1[3], j1[3];
      star_term(xp[u], vp[u], A.GM, a1, j1);
      for (int q = 0; q < size; ++q) {
        if (q == k) continue;
        hard_pair(px[q] - xp[u][0], py[q] - xp[u][1], pz[q] - xp[u][2], pvx[q] - vp[u][0], pvy[q] - vp[u][1],
                  pvz[q] - vp[u][2], pgm[q], fmin(invi[u], pinv[q]), A, a1, j1);
      }
      const double h = (double)(tn - t[u]) * A.tick;
      t[u] = tn;
      correct(x[u], v[u], a0[u], j0[u], xp[u], vp[u], a1, j1, h, t[u], lev[u], A);
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int k = tid + BIG_T * u;
    px[k] = x[u][0];
    py[k] = x[u][1];
    pz[k] = x[u][2];
    pvx[k] = v[u][0];
    pvy[k] = v[u][1];
    pvz[k] = v[u][2];
  }
  __syncthreads();
  e = 0.0;
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int k = tid + BIG_T * u;
    if (!mem[u]) continue;
    e += 0.5 * m[u] * (v[u][0] * v[u][0] + v[u][1] * v[u][1] + v[u][2] * v[u][2]) -
         A.GM * m[u] * rsqrt(x[u][0] * x[u][0] + x[u][1] * x[u][1] + x[u][2] * x[u][2]);
    for (int q = k + 1; q < size; ++q) {
      const double dx = px[q] - x[u][0], dy = py[q] - x[u][1], dz = pz[q] - x[u][2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      e -= m[u] * pgm[q] * (1.0 - changeover_W(r * fmin(invi[u], pinv[q]), A)) / r;
    }
  }
  const double E1 = block_sum(e, shd);
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    if (!mem[u]) continue;
    for (int d = 0; d < 3; ++d) {
      A.pos[d * n + gid[u]] = x[u][d];
      A.vel[d * n + gid[u]] = v[u][d];
    }
    if (A.dt_hard) A.dt_hard[gid[u]] = ldexp(A.dt_soft, -lev[u]);
    if (!(isfinite(x[u][0]) && isfinite(x[u][1]) && isfinite(x[u][2]))) set_flag(A.cnt, P3T_FLAG_NAN);
  }
  if (tid == 0 && A.e_rel) A.e_rel[c] = fabs(E1 - E0) / fabs(E0);
  if (tid == 0 && A.nsteps) A.nsteps[c] = it;
}

// ---------------------------------------------------------------- bucketing
__device__ __forceinline__ int bucket_of(int size) {
  if (size <= 1) return 0;
  if (size <= 2) return 1;
  if (size <= 4) return 2;
  if (size <= 8) return 3;
  if (size <= 16) return 4;
  if (size <= 32) return 5;
  if (size <= 64) return 6;
  if (size <= 256) return 7;
  if (size <= 512) return 8;
  if (size <= 1024) return 9;
  return 10;
}

// Bucket the clusters by size; also validate the caller's cluster arrays
// (offsets non-decreasing from >= 0, members in [0, n)); any violation sets
// bcount[15] and nothing is integrated.
__global__ void k_herm_bucket(int64_t nc, int64_t n, const int32_t *__restrict__ cl_ptr,
                              const int32_t *__restrict__ members, int32_t *__restrict__ bcount,
                              int32_t *__restrict__ blists) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
    const int a = cl_ptr[c], b = cl_ptr[c + 1];
    if (a < 0 || b < a) {
      atomicOr(&bcount[15], 1);
      continue;
    }
    bool ok = true;
    for (int k = a; k < b; ++k) {
      const int g = members[k];
      ok &= (g >= 0 && (int64_t)g < n);
    }
    if (!ok) {
      atomicOr(&bcount[15], 1);
      continue;
    }
    const int size = b - a;
    if (size <= 0) continue;
    const int bk = bucket_of(size);
    const int p = atomicAdd(&bcount[bk], 1);
    blists[(int64_t)bk * nc + p] = (int32_t)c;
  }
}

static void host_changeover_coeffs(double g, HermArgs &A) {
  // c and f(y) of eq. (cutfuncW), expanded in powers of y (plus y ln y)
  const double g2 = g * g, g3 = g2 * g, g4 = g3 * g, g5 = g4 * g, g6 = g5 * g, g7 = g6 * g;
  const double gm = g - 1.0, gm7 = gm * gm * gm * gm * gm * gm * gm;
  A.wc = 7.0 * (g6 - 9.0 * g5 + 45.0 * g4 - 60.0 * g3 * std::log(g) - 45.0 * g2 + 9.0 * g - 1.0) / (3.0 * gm7);
  A.wp[7] = (-10.0 / 3.0) / gm7;
  A.wp[6] = 14.0 * (g + 1.0) / gm7;
  A.wp[5] = -21.0 * (g2 + 3.0 * g + 1.0) / gm7;
  A.wp[4] = 35.0 * (g3 + 9.0 * g2 + 9.0 * g + 1.0) / 3.0 / gm7;
  A.wp[3] = -70.0 * (g3 + 3.0 * g2 + g) / gm7;
  A.wp[2] = 210.0 * (g3 + g2) / gm7;
  A.wp[1] = 0.0;
  A.wp[0] = (g7 - 7.0 * g6 + 21.0 * g5 - 35.0 * g4) / gm7;
  A.wlog = -140.0 * g3 / gm7;
  double f1 = 0.0;
  for (int k = 0; k < 8; ++k) f1 += A.wp[k];  // y = 1, ln 1 = 0
  A.wf1 = f1;
}

hipError_t hermite_clusters(p3t_ctx *c, int64_t n, int64_t nc, const int32_t *cl_ptr, const int32_t *cl_members,
                            double *pos3, double *vel3, const double *mass, const double *r_out, double *dt_hard,
                            double *e_rel_err, int32_t *n_steps) {
  hipStream_t s = c->stream;
  hipError_t e;
  if (nc <= 0) return hipSuccess;
  int32_t *bcount = c->herm_bcount;
  int32_t *blists = c->herm_blists;
  if ((e = fill_i32(bcount, 0, 16, s)) != hipSuccess) return e;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, (nc + 255) / 256));
  hipLaunchKernelGGL(k_herm_bucket, dim3(g), dim3(256), 0, s, nc, n, cl_ptr, cl_members, bcount, blists);
  int32_t hc[16];
  if ((e = hipMemcpyAsync(hc, bcount, sizeof(hc), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  if (hc[15]) return hipErrorInvalidDevicePointer;  // malformed cluster arrays
  if (hc[10] > 0) return hipErrorInvalidValue;       // cluster above the largest supported size
  const p3t_params &P = c->P;
  HermArgs A;
  A.cl_ptr = cl_ptr;
  A.members = cl_members;
  A.pos = pos3;
  A.vel = vel3;
  A.mass = mass;
  A.ro = r_out;
  A.dt_hard = dt_hard;
  A.e_rel = e_rel_err;
  A.nsteps = n_steps;
  A.n = n;
  A.G = P.G;
  A.GM = P.G * P.m_star;
  A.gamma = P.gamma;
  A.inv1mg = 1.0 / (1.0 - P.gamma);
  A.eta = P.eta;
  A.eta0 = P.eta0;
  A.dt_soft = P.dt_soft;
  A.tick = std::ldexp(P.dt_soft, -TICK_BITS);
  A.k_max = P.k_max;
  A.max_iter = 1 << 22;
  A.cnt = c->cnt;
  host_changeover_coeffs(P.gamma, A);
  for (int bk = 0; bk < 10; ++bk) {
    if (hc[bk] == 0) continue;
    A.blist = blists + (int64_t)bk * nc;
    A.nb = hc[bk];
    if (bk < 7) {
      const int seg = 1 << bk;
      const unsigned grid = (unsigned)((hc[bk] + (WAVE / seg) - 1) / (WAVE / seg));
      switch (seg) {
        case 1: hipLaunchKernelGGL(k_herm_seg<1>, dim3(grid), dim3(WAVE), 0, s, A); break;
        case 2: hipLaunchKernelGGL(k_herm_seg<2>, dim3(grid), dim3(WAVE), 0, s, A); break;
        case 4: hipLaunchKernelGGL(k_herm_seg<4>, dim3(grid), dim3(WAVE), 0, s, A); break;
        case 8: hipLaunchKernelGGL(k_herm_seg<8>, dim3(grid), dim3(WAVE), 0, s, A); break;
        case 16: hipLaunchKernelGGL(k_herm_seg<16>, dim3(grid), dim3(WAVE), 0, s, A); break;
        case 32: hipLaunchKernelGGL(k_herm_seg<32>, dim3(grid), dim3(WAVE), 0, s, A); break;
        default: hipLaunchKernelGGL(k_herm_seg<64>, dim3(grid), dim3(WAVE), 0, s, A); break;
      }
    } else if (bk == 7) {
      hipLaunchKernelGGL(k_herm_big<1>, dim3(hc[bk]), dim3(BIG_T), 0, s, A);
    } else if (bk == 8) {
      hipLaunchKernelGGL(k_herm_big<2>, dim3(hc[bk]), dim3(BIG_T), 0, s, A);
    } else {
      hipLaunchKernelGGL(k_herm_big<4>, dim3(hc[bk]), dim3(BIG_T), 0, s, A);
    }
  }
  return hipGetLastError();
}

}  // namespace p3t
