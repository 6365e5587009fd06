// slow.hip -- the soft interactions of the members of parked clusters.
//
// p3t_hard_evaluate parks the clusters still running after a block-step
// budget (the set S of their members) and resumes them on a second stream,
// while the main stream builds, walks and evaluates the tree of everyone
// else at the post-drift state, with the members of S massless (their
// pre-drift positions only shape the boxes) and no neighbour pair involving
// them reported.  On the second stream, after the resume, with S's final
// state read from the park buffers:
//   - every particle i outside S gets sum_{s in S} of the soft pair term of
//     Section 2.2 (changeover K at the larger cut-off, eq. (rout2)), and
//     every (i, s) that passes the neighbour test of Section 2.3 is reported
//     in both directions;
//   - every s in S gets sum_{j != s} over all particles (partial sums over
//     SLOW_CHUNKS ranges of j, added in a fixed order), and the pairs
//     (s, s') with s' in S are reported from both sides;
//   - in mixed precision the pairs beyond the larger cut-off (K = 1) take
//     the Newtonian term in FP32 from an FP64 offset, like the far-particle
//     kernel; everything else is FP64.
// These go into a force buffer and a pair buffer of their own.  After the
// join the main stream adds them to the tree's force (members of S take the
// direct sum alone), appends the pairs behind the force kernels' pairs and
// copies S's final state into pos / vel.  Sums are accumulated in FP64 in a
// fixed order, so the result is reproducible; the pairs arrive in any order
// (the CSR build sorts every row).
#include "force_common.h"

namespace p3t {

namespace {

constexpr double kTinyR2s = 1e-150;  // r = 0 gives y ~ 0 < gamma: K = 0, the term vanishes

struct SoftPair {
  double G, gamma, inv1mg;
};

// soft pair term: G m_j K(r / max(r_out,i, r_out,j)) (x_j - x_i) / r^3
__device__ __forceinline__ void soft_term(const SoftPair &P, double dx, double dy, double dz, double gm, double invi,
                                          double invj, double &ax, double &ay, double &az) {
  const double r2s = fmax(dx * dx + dy * dy + dz * dz, kTinyR2s);
  const double rinv = rsqrt(r2s);
  const double y = r2s * rinv * fmin(invi, invj);
  const double x = fmin(fmax((y - P.gamma) * P.inv1mg, 0.0), 1.0);
  const double x2 = x * x;
  const double K = x2 * x2 * (35.0 + x * (-84.0 + x * (70.0 - 20.0 * x)));
  const double f = gm * K * rinv * rinv * rinv;
  ax += f * dx;
  ay += f * dy;
  az += f * dz;
}

// MIXED: a pair beyond the larger cut-off (y = r / max(r_out) >= 1, so
// K = 1) takes the Newtonian term in FP32 from its FP64 offset, as in the
// far-particle kernel; inside it, and always without MIXED, the FP64 soft
// term.  The pair is screened on the FP32 square of its offset against
// the squares of both sides' r_out and r_search, widened by margins far
// above that square's rounding (a few units in 2^-24): every pair inside
// the changeover goes to the FP64 term (K = 1 for the few within the
// margin), and every pair within a search reach to the exact test.  The
// squares are compared as the bit patterns of non-negative floats, which
// order as the floats do.
constexpr double kMixMargin = 1e-5, kReachMargin = 1e-4;

__device__ __forceinline__ int widened_sq(double r, double margin) {
  return __float_as_int((float)(r * r * (1.0 + margin)));
}

// the K = 1 test and the FP32 term of a MIXED pair: returns true (and adds
// nothing) for a pair that needs the FP64 soft term
__device__ __forceinline__ bool mixed_far_term(float ex, float ey, float ez, int r2q, int ro2a, int ro2b, float gm,
                                               float &fx, float &fy, float &fz) {
  const bool chg = (r2q < ro2a) | (r2q < ro2b);
  const float ri = __frsqrt_rn(__int_as_float(r2q));
  const float f = chg ? 0.0f : gm * ri * ri * ri;
  fx += f * ex;
  fy += f * ey;
  fz += f * ez;
  return chg;
}

// reach of the neighbour test without MIXED: no pair beyond the larger
// search radius passes
__device__ __forceinline__ bool may_neighbour64(double dx, double dy, double dz, double rsi, double rsj) {
  const double rs = fmax(rsi, rsj);
  return dx * dx + dy * dy + dz * dz < rs * rs * (1.0 + 1e-12);
}

// Slots beyond the capacity are counted but not written: the host compares
// the count with the capacity after the join (no status bit is set here,
// because the main stream's evaluation reads and clears the shared status
// word while these kernels run).
__device__ __forceinline__ void push_pair(unsigned long long *n_pairs, int2 *pairs, int64_t cap, int a, int b) {
  const unsigned long long q = atomicAdd(n_pairs, 1ull);
  if ((int64_t)q < cap) pairs[q] = make_int2(a, b);
}

struct SlowArgs {
  const double *pos, *vel, *mass, *ro, *rs;
  const double *spos, *svel;  // final state of the members of S (indexed like pos / vel)
  const uint8_t *slow;
  const int32_t *list;
  int ns;
  int64_t n;
  double *acc;
  double *part;
  DevCounters *cnt;
  unsigned *status;             // status bits of this stream (DevCounters::status_d)
  unsigned long long *n_pairs;  // counter of `pairs`
  int2 *pairs;
  int64_t pair_cap;
  SoftPair P;
  double rsch2, rsch3, dt;
};


constexpr int ST = 256;  // threads per block of the direct kernels

// bitonic sort of the slow list (n <= w entries, w = blockDim.x a power of
// two <= SLOW_CAP) in one workgroup, so that the direct sums run in
// ascending member order
__global__ __launch_bounds__(SLOW_CAP) void k_sort_list(int32_t *a, int n) {
  __shared__ int32_t v[SLOW_CAP];
  const int t = threadIdx.x, w = blockDim.x;
  v[t] = t < n ? a[t] : 0x7fffffff;
  __syncthreads();
  for (int k = 2; k <= w; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int p = t ^ j;
      if (p > t) {
        const bool up = (t & k) == 0;
        const int x = v[t], y = v[p];
        if ((x > y) == up) {
          v[t] = y;
          v[p] = x;
        }
      }
      __syncthreads();
    }
  }
  if (t < n) a[t] = v[t];
}

__global__ void k_mask_mass(int64_t n, const double *__restrict__ mass, const uint8_t *__restrict__ slow,
                            double *__restrict__ m_eff) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m_eff[i] = slow[i] ? 0.0 : mass[i];
}

__global__ void k_slow_scatter(int64_t n, int ns, const int32_t *__restrict__ list, const double *__restrict__ sp,
                               const double *__restrict__ sv, double *__restrict__ pos, double *__restrict__ vel) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < ns; s += gridDim.x * blockDim.x) {
    const int64_t i = list[s];
    for (int d = 0; d < 3; ++d) {
      pos[d * n + i] = sp[d * n + i];
      vel[d * n + i] = sv[d * n + i];
    }
  }
}

// every particle outside S: add the terms of S, report its pairs with S
template <bool MIXED>
__global__ __launch_bounds__(ST) void k_slow_into(SlowArgs A) {
  __shared__ double tx[ST], ty[ST], tz[ST], tvx[ST], tvy[ST], tvz[ST], tm[ST], tro[ST], trs[ST], tinv[ST];
  __shared__ int4 tq[ST];  // MIXED: widened r_out^2 and r_search^2 (bit patterns), G m in FP32
  __shared__ int32_t tid_[ST];
  const int t = threadIdx.x;
  const int64_t n = A.n;
  for (int64_t b0 = (int64_t)blockIdx.x * ST; b0 < n; b0 += (int64_t)gridDim.x * ST) {  // uniform per block
    const int64_t i = b0 + t;
    const bool act = i < n && !A.slow[i];
    const int64_t ic = act ? i : 0;
    const double xi = A.pos[ic], yi = A.pos[n + ic], zi = A.pos[2 * n + ic];
    const double vxi = A.vel[ic], vyi = A.vel[n + ic], vzi = A.vel[2 * n + ic];
    const double mi = A.mass[ic], roi = A.ro[ic], rsi = A.rs[ic], invi = 1.0 / roi;
    const int ro2i = MIXED ? widened_sq(roi, kMixMargin) : 0, rs2i = MIXED ? widened_sq(rsi, kReachMargin) : 0;
    double ax = 0.0, ay = 0.0, az = 0.0;
    bool coincident = false;
    for (int s0 = 0; s0 < A.ns; s0 += ST) {
      const int m = min(ST, A.ns - s0);
      __syncthreads();
      if (t < m) {
        const int64_t j = A.list[s0 + t];
        tx[t] = A.spos[j];
        ty[t] = A.spos[n + j];
        tz[t] = A.spos[2 * n + j];
        tvx[t] = A.svel[j];
        tvy[t] = A.svel[n + j];
        tvz[t] = A.svel[2 * n + j];
        tm[t] = A.mass[j];
        tro[t] = A.ro[j];
        tinv[t] = 1.0 / A.ro[j];
        trs[t] = A.rs[j];
        tid_[t] = (int32_t)j;
        if (MIXED)
          tq[t] = make_int4(widened_sq(A.ro[j], kMixMargin), widened_sq(A.rs[j], kReachMargin),
                            __float_as_int((float)(A.P.G * A.mass[j])), 0);
      }
      __syncthreads();
      if (act) {
        float fx = 0.0f, fy = 0.0f, fz = 0.0f;  // MIXED: this tile's K = 1 terms
        for (int k = 0; k < m; ++k) {
          const double dx = tx[k] - xi, dy = ty[k] - yi, dz = tz[k] - zi;
          bool reach;
          if (MIXED) {
            const int4 q = tq[k];
            const float ex = (float)dx, ey = (float)dy, ez = (float)dz;
            const int r2q = __float_as_int(ex * ex + ey * ey + ez * ez);
            if (mixed_far_term(ex, ey, ez, r2q, ro2i, q.x, __int_as_float(q.z), fx, fy, fz))
              soft_term(A.P, dx, dy, dz, A.P.G * tm[k], invi, tinv[k], ax, ay, az);
            reach = (r2q <= rs2i) | (r2q <= q.y);
          } else {
            soft_term(A.P, dx, dy, dz, A.P.G * tm[k], invi, tinv[k], ax, ay, az);
            reach = may_neighbour64(dx, dy, dz, rsi, trs[k]);
          }
          if (!reach) continue;
          if (tx[k] == xi && ty[k] == yi && tz[k] == zi) coincident = true;
          if (neighbour_test(xi, yi, zi, vxi, vyi, vzi, mi, roi, rsi, tx[k], ty[k], tz[k], tvx[k], tvy[k], tvz[k],
                             tm[k], tro[k], trs[k], A.P.G, A.rsch2, A.rsch3, A.dt)) {
            push_pair(A.n_pairs, A.pairs, A.pair_cap, (int32_t)i, tid_[k]);
            push_pair(A.n_pairs, A.pairs, A.pair_cap, tid_[k], (int32_t)i);
          }
        }
        if (MIXED) {
          ax += (double)fx;
          ay += (double)fy;
          az += (double)fz;
        }
      }
    }
    if (act) {  // the terms of S alone; added to the tree's force after the join
      A.acc[i] = ax;
      A.acc[n + i] = ay;
      A.acc[2 * n + i] = az;
      if (coincident) atomicOr(A.status, P3T_FLAG_COINCIDENT);
    }
  }
}

// Members of S in lanes (SM per workgroup, s = SM blockIdx.y + lane)
// against the particles of chunk blockIdx.x, which pass through LDS in
// tiles of SJ and are read back as broadcasts, so each particle is read
// once per SM members: the partial sum of each member over the chunk, and
// the pairs (s, s') with s' in S.
constexpr int SM = 128, SJ = 256;

template <bool MIXED>
__global__ __launch_bounds__(SM) void k_slow_from(SlowArgs A) {
  __shared__ double4 ja[SJ];  // x, y, z (final state for members of S), G m
  __shared__ double jinv[SJ];  // 1 / r_out
  __shared__ int4 jc[SJ];      // widened r_out^2 (bit pattern), G m in FP32 (bit pattern), member of S
  const int t = threadIdx.x;
  const int slot = blockIdx.y * SM + t;
  const bool act = slot < A.ns;
  const int64_t n = A.n;
  const int64_t i = A.list[act ? slot : 0];
  const double xi = A.spos[i], yi = A.spos[n + i], zi = A.spos[2 * n + i];
  const double invi = 1.0 / A.ro[i];
  const int ro2i = widened_sq(A.ro[i], kMixMargin);
  double ax = 0.0, ay = 0.0, az = 0.0;
  bool coincident = false;
  const int64_t chunk = (n + SLOW_CHUNKS - 1) / SLOW_CHUNKS;
  const int64_t j0 = (int64_t)blockIdx.x * chunk, j1 = j0 + chunk < n ? j0 + chunk : n;
  for (int64_t b = j0; b < j1; b += SJ) {
    const int m = (int)(j1 - b < SJ ? j1 - b : SJ);
    __syncthreads();
    for (int k = t; k < m; k += SM) {
      const int64_t j = b + k;
      const bool sj = A.slow[j];
      const double *pj = sj ? A.spos : A.pos;  // members of S: their final state
      const double roj = A.ro[j], gmj = A.P.G * A.mass[j];
      ja[k] = make_double4(pj[j], pj[n + j], pj[2 * n + j], gmj);
      jinv[k] = 1.0 / roj;
      jc[k] = make_int4(widened_sq(roj, kMixMargin), __float_as_int((float)gmj), sj ? 1 : 0, 0);
    }
    __syncthreads();
    if (!act) continue;
    // j = s itself gives r = 0, hence K = 0 (FP64 term) and an exact zero
    for (int k = 0; k < m; ++k) {
      const double4 q = ja[k];
      const int4 c = jc[k];
      const double dx = q.x - xi, dy = q.y - yi, dz = q.z - zi;
      if (MIXED) {
        const float ex = (float)dx, ey = (float)dy, ez = (float)dz;
        float fx = 0.0f, fy = 0.0f, fz = 0.0f;
        if (mixed_far_term(ex, ey, ez, __float_as_int(ex * ex + ey * ey + ez * ez), ro2i, c.x, __int_as_float(c.y), fx,
                           fy, fz))
          soft_term(A.P, dx, dy, dz, q.w, invi, jinv[k], ax, ay, az);
        ax += (double)fx;
        ay += (double)fy;
        az += (double)fz;
      } else {
        soft_term(A.P, dx, dy, dz, q.w, invi, jinv[k], ax, ay, az);
      }
      if (c.z) {  // a pair within S (rare; uniform over the wavefront)
        const int64_t j = b + k;
        if (j == i) continue;
        if (q.x == xi && q.y == yi && q.z == zi) coincident = true;
        if (neighbour_test(xi, yi, zi, A.svel[i], A.svel[n + i], A.svel[2 * n + i], A.mass[i], A.ro[i], A.rs[i], q.x,
                           q.y, q.z, A.svel[j], A.svel[n + j], A.svel[2 * n + j], A.mass[j], A.ro[j], A.rs[j], A.P.G,
                           A.rsch2, A.rsch3, A.dt))
          push_pair(A.n_pairs, A.pairs, A.pair_cap, (int32_t)i, (int32_t)j);
      }
    }
  }
  if (!act) return;
  if (coincident) atomicOr(A.status, P3T_FLAG_COINCIDENT);
  double *pp = A.part + ((int64_t)slot * SLOW_CHUNKS + blockIdx.x) * 3;
  pp[0] = ax;
  pp[1] = ay;
  pp[2] = az;
}

// one workgroup of RT threads per member s (blockIdx.x): thread t adds the
// chunks t, t + RT, ... in order, then the RT sums are combined pairwise in
// a fixed tree, so the order never changes
constexpr int RT = 256;

__global__ __launch_bounds__(RT) void k_slow_reduce(SlowArgs A) {
  __shared__ double red[3][RT];
  const int s = blockIdx.x, t = threadIdx.x;
  const double *part = A.part + (int64_t)s * SLOW_CHUNKS * 3;
  double a[3] = {0.0, 0.0, 0.0};
  for (int p = t; p < SLOW_CHUNKS; p += RT)
    for (int d = 0; d < 3; ++d) a[d] += part[p * 3 + d];
  for (int d = 0; d < 3; ++d) red[d][t] = a[d];
  for (int w = RT / 2; w > 0; w >>= 1) {
    __syncthreads();
    if (t < w)
      for (int d = 0; d < 3; ++d) red[d][t] += red[d][t + w];
  }
  if (t == 0) {
    const int64_t i = A.list[s];
    for (int d = 0; d < 3; ++d) A.acc[d * A.n + i] = red[d][0];
    if (!(isfinite(red[0][0]) && isfinite(red[1][0]) && isfinite(red[2][0]))) atomicOr(A.status, P3T_FLAG_NAN);
  }
}

// after the join: the tree's force plus the terms of S (members of S: the
// direct sum alone), and the state of S into pos / vel
__global__ void k_slow_merge(int64_t n, const uint8_t *__restrict__ slow, const double *__restrict__ acc_d,
                             double *__restrict__ acc, DevCounters *cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const bool s = slow[i];
    double a[3];
    for (int d = 0; d < 3; ++d) {
      a[d] = s ? acc_d[d * n + i] : acc[d * n + i] + acc_d[d * n + i];
      acc[d * n + i] = a[d];
    }
    if (!(isfinite(a[0]) && isfinite(a[1]) && isfinite(a[2]))) set_flag(cnt, P3T_FLAG_NAN);
  }
}

// the pairs of the direct terms go behind those of the force kernels; a
// second launch moves the counter (every thread of the first reads it).
// Only the slots that were written are moved (at most cap_d); a count above
// cap_d makes the host redo the evaluation.
__global__ void k_slow_pairs(const int2 *__restrict__ pd, int64_t cap_d, int2 *__restrict__ pairs, int64_t cap,
                             DevCounters *cnt) {
  const unsigned long long nd = cnt->n_pairs_d, base = cnt->n_pairs;
  const unsigned long long m = nd < (unsigned long long)cap_d ? nd : (unsigned long long)cap_d;
  for (unsigned long long k = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; k < m;
       k += (unsigned long long)gridDim.x * blockDim.x) {
    if (base + k < (unsigned long long)cap)
      pairs[base + k] = pd[k];
    else
      set_flag(cnt, P3T_FLAG_PAIR_OVERFLOW);
  }
}

__global__ void k_slow_pairs_count(DevCounters *cnt, int64_t cap_d) {
  const unsigned long long nd = cnt->n_pairs_d;
  cnt->n_pairs += nd < (unsigned long long)cap_d ? nd : (unsigned long long)cap_d;
}

}  // namespace

hipError_t slow_prepare(p3t_ctx *c, const double *mass, int ns) {
  hipStream_t s = c->stream;
  const int64_t n = c->n;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, (n + 255) / 256));
  hipLaunchKernelGGL(k_mask_mass, dim3(g), dim3(256), 0, s, n, mass, (const uint8_t *)c->slow_flag, c->m_eff);
  (void)ns;
  return hipGetLastError();
}

// The parked members in ascending order (the list is complete when the
// budgeted launch ends; the resume does not read it), in a workgroup of the
// next power of two threads, at least one wavefront.
hipError_t slow_sort(p3t_ctx *c, int ns, hipStream_t s) {
  if (ns <= 1 || ns > SLOW_CAP) return hipSuccess;
  int w = WAVE;
  while (w < ns) w <<= 1;
  hipLaunchKernelGGL(k_sort_list, dim3(1), dim3(w), 0, s, c->slow_list, ns);
  return hipGetLastError();
}

hipError_t slow_direct(p3t_ctx *c, const double *pos3, const double *vel3, const double *mass, const double *r_out,
                       const double *r_search, int ns, hipStream_t s) {
  const int64_t n = c->n;
  SlowArgs A;
  A.pos = pos3;
  A.vel = vel3;
  A.spos = c->pk_x;
  A.svel = c->pk_v;
  A.mass = mass;
  A.ro = r_out;
  A.rs = r_search;
  A.slow = c->slow_flag;
  A.list = c->slow_list;
  A.ns = ns;
  A.n = n;
  A.acc = c->acc_d;
  A.part = c->slow_part;
  A.cnt = c->cnt;
  A.status = &c->cnt->status_d;
  A.n_pairs = &c->cnt->n_pairs_d;
  A.pairs = c->pairs_d;
  A.pair_cap = c->pairs_d_cap;
  A.P.G = c->P.G;
  A.P.gamma = c->P.gamma;
  A.P.inv1mg = 1.0 / (1.0 - c->P.gamma);
  A.rsch2 = c->P.r_search2;
  A.rsch3 = c->P.r_search3;
  A.dt = c->P.dt_soft;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, (n + ST - 1) / ST));
  const dim3 gf(SLOW_CHUNKS, (ns + SM - 1) / SM);
  if (c->P.precision == 1) {
    hipLaunchKernelGGL(k_slow_into<true>, dim3(g), dim3(ST), 0, s, A);
    hipLaunchKernelGGL(k_slow_from<true>, gf, dim3(SM), 0, s, A);
  } else {
    hipLaunchKernelGGL(k_slow_into<false>, dim3(g), dim3(ST), 0, s, A);
    hipLaunchKernelGGL(k_slow_from<false>, gf, dim3(SM), 0, s, A);
  }
  hipLaunchKernelGGL(k_slow_reduce, dim3(ns), dim3(RT), 0, s, A);
  return hipGetLastError();
}

hipError_t slow_merge(p3t_ctx *c, double *pos3, double *vel3, double *acc3, int ns) {
  hipStream_t s = c->stream;
  const int64_t n = c->n;
  const unsigned gs = (unsigned)std::min<int64_t>(65536, (ns + 255) / 256);
  hipLaunchKernelGGL(k_slow_scatter, dim3(gs), dim3(256), 0, s, n, ns, (const int32_t *)c->slow_list,
                     (const double *)c->pk_x, (const double *)c->pk_v, pos3, vel3);
  if (!acc3) return hipGetLastError();  // state only
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, (n + 255) / 256));
  hipLaunchKernelGGL(k_slow_merge, dim3(g), dim3(256), 0, s, n, (const uint8_t *)c->slow_flag,
                     (const double *)c->acc_d, acc3, c->cnt);
  const unsigned gp = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (c->pairs_d_cap + 255) / 256));
  hipLaunchKernelGGL(k_slow_pairs, dim3(gp), dim3(256), 0, s, (const int2 *)c->pairs_d, c->pairs_d_cap, c->pairs,
                     c->pair_cap, c->cnt);
  hipLaunchKernelGGL(k_slow_pairs_count, dim3(1), dim3(1), 0, s, c->cnt, c->pairs_d_cap);
  return hipGetLastError();
}

}  // namespace p3t
