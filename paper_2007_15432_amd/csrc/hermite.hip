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
// Clusters are bucketed by size; the buckets up to 64 members run in ONE
// launch, so the long-running clusters of different sizes overlap instead
// of queueing:
//   sizes <= 4: SEG = next power of two lanes per cluster, 64/SEG clusters
//     per wavefront, one member per lane (seg_body);
//   sizes 5..64: one wavefront per cluster, one member per lane, the due
//     members' partner sums spread over the wavefront (wave_body);
//   each wavefront runs its own block steps and synchronises only with
//   itself (LDS is private per wave);
//   sizes 65..1024: one 256-thread workgroup per cluster with 1, 2 or 4
//     members per thread, in launches of their own beside the fused one;
//   larger: the percolated-cluster path (device-wide, below).
// Predicted states are shared through LDS.
#include <algorithm>
#include <climits>
#include <vector>

#include "p3t_internal.h"

// No automatic contraction in this file: the fused multiply-adds of the
// step are written out (fmad), so that the plain, parking and resuming
// launches, which compile the same formulas into different kernels, round
// every operation identically (a parked and resumed cluster ends bit for
// bit where an uninterrupted one does).
#pragma clang fp contract(off)

namespace p3t {

constexpr int TICK_BITS = 40;
constexpr int BIG_T = 256;
constexpr int N_BUCKETS = HERM_N_BUCKETS;  // SEG 1..64 (7), 256-thread MPT 1, 2, 4 (3), too big (1)
constexpr int BC_NC = HERM_BC_NC, BC_BAD = HERM_BC_BAD, BC_WORDS = HERM_BC_WORDS;
constexpr int PK_MEM = HERM_BC_PARKED - HERM_BC_PARK0;  // parked-member word, relative to the park counts
constexpr int WAVE_BK0 = 3;  // buckets 3..6 (5..64 members): one wavefront per cluster (wave_body)
// Regions of the fused launch: buckets 0..6, then the clusters of buckets
// 1..3 that hold a close pair (regions 7..9); dispatched from the last
// region to the first.
constexpr int FUSED_REGIONS = 10;

struct HermArgs {
  const int32_t *cl_ptr, *members, *blists;
  int64_t nc;                      // clusters (stride of the bucket lists)
  int bcount[N_BUCKETS];           // clusters per bucket (the close ones of buckets 1..3 not counted)
  int ccount[4];                   // [1..3]: clusters of buckets 1..3 with a close pair
  int boff[N_BUCKETS + 1];         // first block of each region of the fused launch (FUSED_REGIONS + 1 used)
  double *pos, *vel;
  const double *mass, *ro;
  double *dt_hard, *e_rel;
  int32_t *nsteps;
  int32_t *msteps;  // per particle: block steps of its cluster (nullable)
  // Parking: in the parking launches (k_herm_fused<1>, k_herm_big<., 1>) a
  // cluster still running after `budget` block steps saves its state to pk
  // and stops; the resume launches (mode 2) continue parked clusters from pk
  // and write their final state to pos / vel (the park buffers).
  int budget;
  struct {
    double *x, *v, *a, *j;  // per member (3n each), at the member's own time
    int64_t *t;             // per member: its time in ticks
    int32_t *lev;           // per member: its block level
    int32_t *nst;           // per cluster: block steps so far
    double *e0;             // per cluster: energy at the start
    int32_t *count;         // [0, 10) parked clusters per bucket, [PK_MEM] parked members
    int32_t *lists;         // parked clusters, 10 lists of n
    int32_t *members;       // parked members (n)
    uint8_t *flag;          // per particle: 1 if parked (cleared by the caller)
  } pk;
  // perfect-accretion collisions (wave path, k_herm_fused<0, true>): two
  // bodies merge when r < coll_f (R_i + R_j), R = cbrt(coll_r3 m)
  double coll_f, coll_r3;
  int32_t *merged;  // per particle: index of its composite's lowest member (nullable)
  double *ceps;     // per cluster: six dissipation sums (nullable)
  int64_t n;
  double G, GM, gamma, inv1mg, eta, eta0, dt_soft, tick;
  // powers of dt_soft for the corrector (scaled per level by exact powers of two)
  double inv_dt2, inv_dt3, dt3_6, dt4_24, dt5_120, dt_soft2;
  int k_max, max_iter;
  double wc, wf1, wlog;
  double wp[8];  // f(y) = sum_k wp[k] y^k + wlog y ln y   (eq. (cutfuncW))
  DevCounters *cnt;
};

__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// x + v dl + a dl^2/2 + j dl^3/6 and v + a dl + j dl^2/2 (d2 = dl^2/2,
// d3 = dl^3/6), Horner-ordered fused multiply-adds
__device__ __forceinline__ void predict(const double *x, const double *v, const double *a, const double *j, double dl,
                                        double d2, double d3, double *xp, double *vp) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    xp[d] = fmad(j[d], d3, fmad(a[d], d2, fmad(v[d], dl, x[d])));
    vp[d] = fmad(j[d], d2, fmad(a[d], dl, v[d]));
  }
}

__device__ __forceinline__ double changeover_W(double y, const HermArgs &A) {
  if (y < A.gamma) return A.wc * y;
  if (y >= 1.0) return 1.0;
  double p = A.wp[7];
#pragma unroll
  for (int k = 6; k >= 0; --k) p = fmad(p, y, A.wp[k]);
  return fmad(1.0 - A.wf1, y, fmad(A.wlog * y, log(y), p));
}

// hard pair term on i from j: d = x_j - x_i, u = v_j - v_i
__device__ __forceinline__ void hard_pair(double dx, double dy, double dz, double ux, double uy, double uz, double gmj,
                                          double invR, const HermArgs &A, double *a, double *jk) {
  const double r2 = fmad(dz, dz, fmad(dy, dy, dx * dx));
  const double rinv = rsqrt_pos(r2);  // distinct members (coincident ones are flagged before)
  const double y = r2 * rinv * invR;
  const double x = fmin(fmax((y - A.gamma) * A.inv1mg, 0.0), 1.0);
  const double x2 = x * x, x3 = x2 * x;
  const double K = x2 * x2 * fmad(x, fmad(x, fmad(-20.0, x, 70.0), -84.0), 35.0);
  const double omx = 1.0 - x;
  const double Ky = (x > 0.0 && x < 1.0) ? 140.0 * x3 * omx * omx * omx * A.inv1mg : 0.0;
  const double s = fmad(dz, uz, fmad(dy, uy, dx * ux));
  const double rinv2 = rinv * rinv;
  const double rinv3 = rinv * rinv2;
  const double w = gmj * (1.0 - K) * rinv3;
  const double c1 = 3.0 * s * rinv2;
  const double c2 = gmj * Ky * s * rinv * invR * rinv3;
  a[0] = fmad(w, dx, a[0]);
  a[1] = fmad(w, dy, a[1]);
  a[2] = fmad(w, dz, a[2]);
  jk[0] = fmad(-c2, dx, fmad(w, fmad(-c1, dx, ux), jk[0]));
  jk[1] = fmad(-c2, dy, fmad(w, fmad(-c1, dy, uy), jk[1]));
  jk[2] = fmad(-c2, dz, fmad(w, fmad(-c1, dz, uz), jk[2]));
}

__device__ __forceinline__ void star_term(const double *x, const double *v, double GM, double *a, double *jk) {
  const double r2 = fmad(x[2], x[2], fmad(x[1], x[1], x[0] * x[0]));
  const double rinv = rsqrt_pos(r2);  // a particle away from the star
  const double rinv3 = rinv * rinv * rinv;
  const double xv = fmad(x[2], v[2], fmad(x[1], v[1], x[0] * v[0]));
  const double c5 = 3.0 * xv * rinv * rinv;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    a[d] = -GM * x[d] * rinv3;
    jk[d] = -GM * fmad(-c5, x[d], v[d]) * rinv3;
  }
}

// Smallest k >= 0 with dt_soft 2^-k <= dtc (k_max + 1 if none): the same
// decision as a linear search from k = 0, started two levels below the
// exponent difference (every comparison is exact: ldexp scales by 2^-k).
__device__ __forceinline__ int level_for(double dt_soft, double dtc, int kmax) {
  if (!(dtc < dt_soft)) return 0;
  if (!(dtc > 0.0)) return kmax + 1;
  int k = ilogb(dt_soft) - ilogb(dtc) - 1;
  k = k < 0 ? 0 : k;
  while (k <= kmax && ldexp(dt_soft, -k) > dtc) ++k;
  return k;
}

__device__ __forceinline__ double dot3(const double *a, const double *b) {
  return fmad(a[2], b[2], fmad(a[1], b[1], a[0] * b[0]));
}
__device__ __forceinline__ double norm3(const double *a) { return sqrt(dot3(a, a)); }

// The square roots of the Aarseth sums, which only decide the level: x
// times the corrected hardware reciprocal root (within about an ulp of the
// rounded root), zero for x = 0.  A non-finite x gives a NaN, which the
// level search maps to level 0 like any other non-finite criterion.
__device__ __forceinline__ double root_level(double x) { return x > 0.0 ? x * rsqrt_pos(x) : 0.0; }

// Smallest k >= 0 with P 4^-k <= L (k_max + 1 if none), P = dt_soft^2 den,
// L = eta num >= 0: the level whose squared step does not exceed the
// squared Aarseth step.  P = 0 (den = 0) gives level 0, as a step of dt_soft.
// Closed form, without a search loop: for P > L > 0 let e = ilogb(P) -
// ilogb(L) >= 0; P 4^-k <= L holds for 2k >= e + 1 and fails for 2k <= e - 1,
// and at 2k = e one exact comparison of the scaled P decides.
__device__ __forceinline__ int level_for_sq(double P, double L, int kmax) {
  const bool ok = P > L && L > 0.0;
  // ilogb(inf) is INT_MAX: bounded first; then e >= 2 k_max + 2 already
  // gives k_max + 1
  int eP = ilogb(ok ? P : 2.0);
  eP = eP < 1100 ? eP : 1100;
  int e = eP - ilogb(ok ? L : 1.0);
  e = e < 2 * kmax + 2 ? e : 2 * kmax + 2;
  int k = (e + 1) >> 1;
  k += ((e & 1) == 0 && ldexp(P, -e) > L) ? 1 : 0;
  k = k > kmax ? kmax + 1 : k;
  k = (L > 0.0) ? k : kmax + 1;
  return (P > L) ? k : 0;
}

// corrector + new level for one active member; its step is h = dt_soft 2^-lev
// (h, 1/h^2, 1/h^3, h^3/6, ... are the level-0 powers scaled by exact
// powers of two, so no division sits on the step's dependency chain)
__device__ __forceinline__ void correct(double *x, double *v, double *a0, double *j0, const double *xp, const double *vp,
                                        const double *a1, const double *j1, double h, int64_t tnew, int &lev,
                                        const HermArgs &A) {
  double a2[3], a3[3];
  const int l = lev, l2 = l + l, l3 = l2 + l, l4 = l2 + l2, l5 = l4 + l;  // shifts and adds, no multiply
  const double ih2 = ldexp(A.inv_dt2, l2), ih3 = ldexp(A.inv_dt3, l3);
  const double h3_6 = ldexp(A.dt3_6, -l3), h4_24 = ldexp(A.dt4_24, -l4), h5_120 = ldexp(A.dt5_120, -l5);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double da = a0[d] - a1[d];
    a2[d] = fmad(-h, fmad(4.0, j0[d], 2.0 * j1[d]), -6.0 * da) * ih2;
    a3[d] = fmad(6.0 * h, j0[d] + j1[d], 12.0 * da) * ih3;
    x[d] = fmad(a3[d], h5_120, fmad(a2[d], h4_24, xp[d]));
    v[d] = fmad(a3[d], h4_24, fmad(a2[d], h3_6, vp[d]));
    a0[d] = a1[d];
    j0[d] = j1[d];
  }
  // Aarseth: dt^2 = eta (|a||a2| + |j|^2) / (|j||a3| + |a2|^2), a2 at the
  // step's end.  The level is the smallest k with (dt_soft 2^-k)^2 <= dt^2,
  // found without the division and the outer root: dt_soft^2 den 4^-k <=
  // eta num, with |a||a2| = sqrt(|a|^2 |a2|^2) (two roots instead of four).
  const double a2e[3] = {fmad(a3[0], h, a2[0]), fmad(a3[1], h, a2[1]), fmad(a3[2], h, a2[2])};
  const double an2 = dot3(a1, a1), jn2 = dot3(j1, j1), a2n2 = dot3(a2e, a2e), a3n2 = dot3(a3, a3);
  const double num = A.eta * (root_level(an2 * a2n2) + jn2);
  const double den = root_level(jn2 * a3n2) + a2n2;
  const int knew = level_for_sq(A.dt_soft2 * den, num, A.k_max);
  // grow by at most a factor two, and only on a multiple of the doubled
  // step (lev <= k_max <= 40, so the shift stays below 64)
  const int64_t dbl_mask = ((int64_t)1 << (TICK_BITS - lev + 1)) - 1;
  const bool grow = lev > 0 && (tnew & dbl_mask) == 0;
  int k = knew < lev ? (grow ? lev - 1 : lev) : knew;
  if (k > A.k_max) {
    set_flag(A.cnt, P3T_FLAG_KMAX);
    k = A.k_max;
  }
  lev = k;
}

__device__ __forceinline__ int initial_level(const double *a0, const double *j0, bool mem, int gid, const HermArgs &A) {
  double dtc = A.dt_soft;
  const double an = norm3(a0), jn = norm3(j0);
  if (jn > 0.0) dtc = A.eta0 * an / jn;
  if (mem && A.dt_hard && A.dt_hard[gid] > 0.0) dtc = A.dt_hard[gid];  // step carried from the last soft step
  int lev = level_for(A.dt_soft, dtc, A.k_max);
  if (lev > A.k_max) {
    if (mem) set_flag(A.cnt, P3T_FLAG_KMAX);
    lev = A.k_max;
  }
  return lev;
}

// DPP lane permutations inside a row of 16 lanes (no LDS round trip):
// quad_perm [1,0,3,2] and [2,3,0,1] exchange with lane^1 and lane^2;
// row_half_mirror and row_mirror reflect 8- and 16-lane blocks, which after
// the quad steps brings the other half's minimum to every lane.
template <int CTRL>
__device__ __forceinline__ int64_t dpp_i64(int64_t v) {
  // every lane is written (the permutations stay inside each row), so no
  // "old" value is needed
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)(uint64_t)v, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)((uint64_t)v >> 32), CTRL, 0xF, 0xF, true);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140;

// minimum over aligned segments of 2^sl2 lanes (sl2 wave-uniform); every
// lane of the wave must be active
__device__ __forceinline__ int64_t seg_min(int64_t v, int sl2) {
  int64_t t;
  if (sl2 >= 1) { t = dpp_i64<DPP_XOR1>(v); v = t < v ? t : v; }
  if (sl2 >= 2) { t = dpp_i64<DPP_XOR2>(v); v = t < v ? t : v; }
  if (sl2 >= 3) { t = dpp_i64<DPP_HALF_MIRROR>(v); v = t < v ? t : v; }
  if (sl2 >= 4) { t = dpp_i64<DPP_MIRROR>(v); v = t < v ? t : v; }
  if (sl2 >= 5) { t = __shfl_xor(v, 16, WAVE); v = t < v ? t : v; }
  if (sl2 >= 6) { t = __shfl_xor(v, 32, WAVE); v = t < v ? t : v; }
  return v;
}
// sum over aligned segments of 2^sl2 lanes
__device__ __forceinline__ double seg_sum(double v, int sl2) {
  for (int o = 1; o < (1 << sl2); o <<= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// LDS ordering inside one wavefront: a wave's LDS operations execute in
// order, so a compiler fence at wavefront scope is enough between a write by
// one lane and a read by another.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Work counters: n_eval evaluations of a member of a cluster of `size`
// (each sums size - 1 partners), summed over the wavefront, one atomic.
// Every lane of the wavefront must call it.
__device__ __forceinline__ void count_work(const HermArgs &A, int n_eval, int size) {
  unsigned long long e = (unsigned long long)n_eval, p = (unsigned long long)n_eval * (unsigned long long)(size - 1);
  if (size <= 0) e = p = 0;
  e = wave_sum(e);
  p = wave_sum(p);
  if ((threadIdx.x & (WAVE - 1)) == 0 && e > 0) {
    atomicAdd(&A.cnt->n_heval, e);
    atomicAdd(&A.cnt->n_hpair, p);
  }
}

struct Lds {
  double *px, *py, *pz, *pvx, *pvy, *pvz, *pgm, *pinv;
  int *act;     // big clusters: active members of the step (BIG_ACT)
  double *res;  // big clusters: their reduced partner sums (6 BIG_ACT)
  // collisions (wave path): composite of each slot (its lowest slot), the
  // composite's radius, the slot's mass
  int *cid;
  double *rad, *pm;
};
constexpr int BIG_ACT = 128;  // most active members handled lane-parallel

// ---------------------------------------------------------------- small clusters
// One wavefront (lanes [wbase, wbase + 64) of the LDS arrays) runs 64/SEG
// clusters; cluster index ci of bucket bk.
// Lanes of a size bucket bk <= 6: SEG = 2^bk member slots per cluster and
// LPM = 2^ll2 lanes per member that share the member's pair loop, so a
// cluster spans 2^(bk + ll2) lanes.  Small clusters (bk <= 1) keep one lane
// per member and pack many clusters per wavefront; from four members on,
// the pair loop, which grows with the cluster, is split over up to eight
// lanes per member (clusters then fill a whole wavefront or a quarter).
__host__ __device__ constexpr int lanes_per_member_log2(int bk) {
  return bk < 2 ? 0 : (bk < 6 - bk ? bk : 6 - bk);
}

// DPP exchange of a double with a fixed lane permutation
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int64_t t = dpp_i64<CTRL>(__double_as_longlong(v));
  return __longlong_as_double(t);
}
// sum over aligned groups of 2^ll2 <= 8 lanes (all lanes active)
__device__ __forceinline__ double lpm_sum(double v, int ll2) {
  if (ll2 >= 1) v += dpp_f64<DPP_XOR1>(v);
  if (ll2 >= 2) v += dpp_f64<DPP_XOR2>(v);
  if (ll2 >= 3) v += dpp_f64<DPP_HALF_MIRROR>(v);
  return v;
}

// One wavefront (lanes [wbase, wbase + 64) of the LDS arrays) runs the
// clusters ci0, ci0 + 1, ... of bucket bk; one body serves every bucket (a
// template per bucket would multiply the kernel's code, and all buckets run
// side by side in the fused launch, sharing the instruction cache).  The
// LPM lanes of a member hold identical copies of its state; each evaluates
// every LPM-th partner and the partial sums are added across them.
// MODE 0: plain; 1: park clusters still running after A.budget steps;
// 2: resume parked clusters
template <int MODE, int SL2 = -1>
__device__ __forceinline__ void seg_body(const HermArgs &A, const int32_t *blist, int count, int ci0, const Lds &L,
                                         int wbase, int sl2_rt) {
  const int sl2 = SL2 >= 0 ? SL2 : sl2_rt;
  constexpr bool RESUME = MODE == 2, PARK = MODE == 1;
  const int ll2 = lanes_per_member_log2(sl2), cl2 = sl2 + ll2;
  const int SEG = 1 << sl2, LPM = 1 << ll2;
  const int lane = threadIdx.x & (WAVE - 1), cseg = lane >> cl2, lic = lane & ((1 << cl2) - 1);
  const int sl = lic >> ll2, sub = lic & (LPM - 1);
  const int sb = wbase + cseg * SEG;  // LDS slot of the cluster's first member
  const int ci = ci0 + cseg;
  const int c = ci < count ? blist[ci] : -1;
  const int b = c >= 0 ? A.cl_ptr[c] : 0;
  const int size = c >= 0 ? A.cl_ptr[c + 1] - b : 0;
  const bool mem = sl < size;
  const bool lead = mem && sub == 0;  // the copy that reads and writes memory
  const int gid = mem ? A.members[b + sl] : 0;
  const int64_t n = A.n;
  const int me = sb + sl;
  double x[3] = {1.0, 0.0, 0.0}, v[3] = {0.0, 1.0, 0.0}, a0[3], j0[3];
  double m = 0.0, ro = 1.0;
  const double *src_x = RESUME ? A.pk.x : A.pos, *src_v = RESUME ? A.pk.v : A.vel;
  if (mem) {
    x[0] = src_x[gid];
    x[1] = src_x[n + gid];
    x[2] = src_x[2 * n + gid];
    v[0] = src_v[gid];
    v[1] = src_v[n + gid];
    v[2] = src_v[2 * n + gid];
    m = A.mass[gid];
    ro = A.ro[gid];
  }
  const double invi = 1.0 / ro;
  wave_sync();
  if (lead) {
    L.pgm[me] = A.G * m;
    L.pinv[me] = invi;
    L.px[me] = x[0];
    L.py[me] = x[1];
    L.pz[me] = x[2];
    L.pvx[me] = v[0];
    L.pvy[me] = v[1];
    L.pvz[me] = v[2];
  }
  wave_sync();
  // forces at t = 0 and the initial energy (a resumed cluster reads them)
  double pa[3] = {0.0, 0.0, 0.0}, pj[3] = {0.0, 0.0, 0.0};
  double e = lead ? 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) -
                        A.GM * m * rsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2])
                  : 0.0;
  if (mem && !RESUME) {
    for (int jj = sub; jj < size; jj += LPM) {
      if (jj == sl) continue;
      const int q = sb + jj;
      const double dx = L.px[q] - x[0], dy = L.py[q] - x[1], dz = L.pz[q] - x[2];
      const double invR = fmin(invi, L.pinv[q]);
      hard_pair(dx, dy, dz, L.pvx[q] - v[0], L.pvy[q] - v[1], L.pvz[q] - v[2], L.pgm[q], invR, A, pa, pj);
      if (jj > sl) {
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        e -= m * L.pgm[q] * (1.0 - changeover_W(r * invR, A)) / r;
      }
    }
  }
  star_term(x, v, A.GM, a0, j0);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    a0[d] += lpm_sum(pa[d], ll2);
    j0[d] += lpm_sum(pj[d], ll2);
  }
  double E0 = seg_sum(e, cl2);
  int lev = initial_level(a0, j0, mem, gid, A);  // every copy reads the carried step
  // two-member clusters: the partner's G m and 1 / r_out (lane ^ 1), and
  // the pair's 1 / max(r_out) as the LDS path forms it
  double pgm_q = 0.0, pinv_q = 0.0;
  if constexpr (SL2 == 1) {
    pgm_q = dpp_f64<DPP_XOR1>(A.G * m);
    pinv_q = fmin(invi, dpp_f64<DPP_XOR1>(invi));
  }
  const int64_t T = (int64_t)1 << TICK_BITS;
  const int max_iter = A.max_iter;
  const double tick = A.tick, GM = A.GM;
  int64_t t = 0;
  int nst = 0;  // block steps of this lane's cluster
  if (RESUME && mem) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      a0[d] = A.pk.a[d * n + gid];
      j0[d] = A.pk.j[d * n + gid];
    }
    t = A.pk.t[gid];
    lev = A.pk.lev[gid];
  }
  if (RESUME && c >= 0) {
    nst = A.pk.nst[c];
    E0 = A.pk.e0[c];
  }
  bool parked = false;
  const int budget = PARK ? A.budget : INT_MAX;
  int n_eval = 0;  // block steps in which this lane's member was due (lead copies only)
  for (int it = 0;; ++it) {
    const int64_t te = mem ? t + ((int64_t)1 << (TICK_BITS - lev)) : LLONG_MAX;
    // every step divides T and each member's time is a multiple of its
    // step, so a cluster is finished exactly when its earliest next time
    // lies beyond T
    const int64_t tn = seg_min(te, cl2);
    const bool done = (size == 0) || (tn > T) || parked;
    if (__all(done)) break;
    if (it == budget) break;  // uniform
    if (it >= max_iter) {
      if (lane == 0) set_flag(A.cnt, P3T_FLAG_NSTEPS);
      break;
    }
    const bool active = mem && !done && te == tn;
    nst += done ? 0 : 1;
    double xp[3], vp[3];
    // every lane predicts (a lane whose cluster is done, or that holds no
    // member, computes a value nobody reads), so no branch is taken here
    {
      const double dl = (double)(tn - t) * tick;
      const double d2 = dl * dl * 0.5, d3 = dl * dl * dl * (1.0 / 6.0);
      predict(x, v, a0, j0, dl, d2, d3, xp, vp);
    }
    double a1[3], j1[3];
    if constexpr (SL2 == 1) {
      // two members in adjacent lanes: the partner's predicted state comes
      // over DPP (every lane is active here), no LDS round trip, and its
      // term adds straight onto the star's; lanes that are not due compute
      // sums nobody reads
      star_term(xp, vp, GM, a1, j1);
      const double qx = dpp_f64<DPP_XOR1>(xp[0]), qy = dpp_f64<DPP_XOR1>(xp[1]), qz = dpp_f64<DPP_XOR1>(xp[2]);
      const double qvx = dpp_f64<DPP_XOR1>(vp[0]), qvy = dpp_f64<DPP_XOR1>(vp[1]), qvz = dpp_f64<DPP_XOR1>(vp[2]);
      hard_pair(qx - xp[0], qy - xp[1], qz - xp[2], qvx - vp[0], qvy - vp[1], qvz - vp[2], pgm_q, pinv_q, A, a1, j1);
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) pa[d] = pj[d] = 0.0;
      wave_sync();
      if (lead) {
        L.px[me] = xp[0];
        L.py[me] = xp[1];
        L.pz[me] = xp[2];
        L.pvx[me] = vp[0];
        L.pvy[me] = vp[1];
        L.pvz[me] = vp[2];
      }
      // the star's term needs only the own predicted state: computed while
      // the exchange through LDS is in flight (one wavefront runs this chain
      // alone, so independent work is what hides the FP64 latency)
      star_term(xp, vp, GM, a1, j1);
      wave_sync();
      if (active) {
        for (int jj = sub; jj < size; jj += LPM) {
          if (jj == sl) continue;
          const int q = sb + jj;
          hard_pair(L.px[q] - xp[0], L.py[q] - xp[1], L.pz[q] - xp[2], L.pvx[q] - vp[0], L.pvy[q] - vp[1],
                    L.pvz[q] - vp[2], L.pgm[q], fmin(invi, L.pinv[q]), A, pa, pj);
        }
      }
    }
    if (ll2 > 0) {  // partial sums of the member's copies (all lanes take part)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        pa[d] = lpm_sum(pa[d], ll2);
        pj[d] = lpm_sum(pj[d], ll2);
      }
    }
    if (active) {
      if constexpr (SL2 != 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          a1[d] += pa[d];
          j1[d] += pj[d];
        }
      }
      const double h = (double)(tn - t) * tick;
      t = tn;
      correct(x, v, a0, j0, xp, vp, a1, j1, h, t, lev, A);
      n_eval += sub == 0 ? 1 : 0;
    }
  }
  count_work(A, n_eval, size);
  if (PARK) {
    // park the clusters still running: their first lane takes the slots
    const int64_t te = mem ? t + ((int64_t)1 << (TICK_BITS - lev)) : LLONG_MAX;
    const int64_t tmin = seg_min(te, cl2);  // every lane takes part
    const bool fin = (size == 0) || (tmin > T);
    int64_t slot = LLONG_MAX;
    if (!fin && lic == 0) {
      const int k = atomicAdd(&A.pk.count[sl2], 1);
      A.pk.lists[(int64_t)sl2 * A.n + k] = c;
      A.pk.nst[c] = nst;
      A.pk.e0[c] = E0;
      slot = atomicAdd(&A.pk.count[PK_MEM], size);
    }
    slot = seg_min(slot, cl2);
    parked = slot != LLONG_MAX;
    if (parked && lead) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        A.pk.x[d * n + gid] = x[d];
        A.pk.v[d * n + gid] = v[d];
        A.pk.a[d * n + gid] = a0[d];
        A.pk.j[d * n + gid] = j0[d];
      }
      A.pk.t[gid] = t;
      A.pk.lev[gid] = lev;
      A.pk.members[slot + sl] = gid;
      A.pk.flag[gid] = 1;
    }
  }
  // final energy
  wave_sync();
  if (lead) {
    L.px[me] = x[0];
    L.py[me] = x[1];
    L.pz[me] = x[2];
    L.pvx[me] = v[0];
    L.pvy[me] = v[1];
    L.pvz[me] = v[2];
  }
  wave_sync();
  e = lead ? 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) -
                 A.GM * m * rsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2])
           : 0.0;
  if (mem) {
    for (int jj = sl + 1 + sub; jj < size; jj += LPM) {
      const int q = sb + jj;
      const double dx = L.px[q] - x[0], dy = L.py[q] - x[1], dz = L.pz[q] - x[2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      e -= m * L.pgm[q] * (1.0 - changeover_W(r * fmin(invi, L.pinv[q]), A)) / r;
    }
  }
  const double E1 = seg_sum(e, cl2);
  if (PARK && parked) return;  // finished by the resume launch
  if (lead) {
    A.pos[gid] = x[0];
    A.pos[n + gid] = x[1];
    A.pos[2 * n + gid] = x[2];
    A.vel[gid] = v[0];
    A.vel[n + gid] = v[1];
    A.vel[2 * n + gid] = v[2];
    if (A.dt_hard) A.dt_hard[gid] = ldexp(A.dt_soft, -lev);
    if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))) set_flag(A.cnt, P3T_FLAG_NAN);
  }
  if (lic == 0 && c >= 0 && A.e_rel) A.e_rel[c] = fabs(E1 - E0) / fabs(E0);
  if (lic == 0 && c >= 0 && A.nsteps) A.nsteps[c] = nst;
  if (lead && A.msteps) A.msteps[gid] = nst;
}

// ---------------------------------------------------------------- mid-size clusters
// one butterfly stage (a DPP lane permutation inside rows of 16 lanes)
// added to six sums; every lane of the wavefront takes part
template <int CTRL>
__device__ __forceinline__ void red6(double *pa, double *pj) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    pa[d] += dpp_f64<CTRL>(pa[d]);
    pj[d] += dpp_f64<CTRL>(pj[d]);
  }
}

// minimum over the wavefront, as a wave-uniform value: DPP inside each row
// of 16 lanes, then the four row minima read into scalar registers (no LDS
// round trip)
__device__ __forceinline__ int64_t wave_min_uniform(int64_t v) {
  v = seg_min(v, 4);
  const int64_t r0 = uniform_lane64(v, 0), r1 = uniform_lane64(v, 16);
  const int64_t r2 = uniform_lane64(v, 32), r3 = uniform_lane64(v, 48);
  const int64_t m01 = r0 < r1 ? r0 : r1, m23 = r2 < r3 ? r2 : r3;
  return m01 < m23 ? m01 : m23;
}

// ceil(log2(v)) for 1 <= v <= 64
__device__ __forceinline__ int ceil_log2(int v) { return v <= 1 ? 0 : 32 - __clz(v - 1); }

// the same minimum when only lanes [0, size) hold values (the others hold
// the maximum): a cluster of at most 16 members needs the DPP stages of
// its own power of two and lane 0 alone (uniform branch on size)
__device__ __forceinline__ int64_t wave_min_members(int64_t v, int size) {
  if (size <= 16) return uniform_lane64(seg_min(v, ceil_log2(size)), 0);
  return wave_min_uniform(v);
}

// Partner sums (star excluded) of the members listed in L.act[wbase, +n_act)
// from the states in the LDS slots [wbase, wbase + size): each listed member
// gets 2^lg lanes, 2^lg = the largest power of two with n_act 2^lg <= 64 and
// 2^lg <= the cluster's power of two; a lane sums every 2^lg-th partner and
// DPP adds the partial sums inside each row of 16 lanes.  The sums land in
// L.res, six doubles per slot: the member at list position a owns the slots
// [a P, a P + P), P = 2^lg / 16 row partials (1 if 2^lg <= 16), which its
// own lane adds in order (res_slots gives P).  Every lane of the wavefront
// must call it.
__device__ __forceinline__ int res_parts_log2(int lg) { return lg > 4 ? lg - 4 : 0; }

__device__ __forceinline__ int spread_lg(int size, int n_act) { return min(6 - ceil_log2(n_act), ceil_log2(size)); }

// COLL: the two parts of a composite exchange no term, and every evaluated
// pair of distinct bodies closer than coll_f (R_k + R_q) is a collision;
// returns the first of them as (lower slot) * 64 + higher slot, or -1
// (wave-uniform).  Without COLL returns -1.
template <bool COLL>
__device__ __forceinline__ int spread_sums(const HermArgs &A, const Lds &L, int wbase, int size, int n_act, int lane,
                                           unsigned long long amask) {
  const int lg = spread_lg(size, n_act);
  const int grp = lane >> lg, sub = lane & ((1 << lg) - 1);
  int k;
  if (n_act <= 2) {  // the usual case: the members from the due mask, in scalar registers
    const int k0 = __ffsll((long long)amask) - 1;
    const int k1 = __ffsll((long long)(amask & (amask - 1))) - 1;
    k = grp == 0 ? k0 : (grp == 1 ? k1 : -1);
  } else {
    k = grp < n_act ? L.act[wbase + grp] : -1;
  }
  double pa[3] = {0.0, 0.0, 0.0}, pj[3] = {0.0, 0.0, 0.0};
  int key = INT_MAX;  // COLL: first colliding pair seen by this lane
  if (k >= 0) {
    const int sk = wbase + k;
    const double xk = L.px[sk], yk = L.py[sk], zk = L.pz[sk], vxk = L.pvx[sk], vyk = L.pvy[sk], vzk = L.pvz[sk];
    const double ik = L.pinv[sk];
    const int ck = COLL ? L.cid[sk] : 0;
    const double rk = COLL ? L.rad[sk] : 0.0;
    for (int q = sub; q < size; q += 1 << lg) {
      if (q == k) continue;
      const int sq = wbase + q;
      if (COLL) {
        if (L.cid[sq] == ck) continue;  // parts of one composite
        const double dx = L.px[sq] - xk, dy = L.py[sq] - yk, dz = L.pz[sq] - zk;
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double rs = A.coll_f * (rk + L.rad[sq]);
        if (r2 < rs * rs) key = min(key, min(k, q) * WAVE + max(k, q));
      }
      hard_pair(L.px[sq] - xk, L.py[sq] - yk, L.pz[sq] - zk, L.pvx[sq] - vxk, L.pvy[sq] - vyk, L.pvz[sq] - vzk,
                L.pgm[sq], fmin(ik, L.pinv[sq]), A, pa, pj);
    }
  }
  // one uniform branch per stage for all six sums
  const int rl = lg < 4 ? lg : 4;
  if (rl >= 1) red6<DPP_XOR1>(pa, pj);
  if (rl >= 2) red6<DPP_XOR2>(pa, pj);
  if (rl >= 3) red6<DPP_HALF_MIRROR>(pa, pj);
  if (rl >= 4) red6<DPP_MIRROR>(pa, pj);
  if (k >= 0 && (sub & ((1 << rl) - 1)) == 0) {
    const int slot = (grp << res_parts_log2(lg)) + (sub >> 4);
    double *r = L.res + 6 * (wbase + slot);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      r[d] = pa[d];
      r[3 + d] = pj[d];
    }
  }
  if (!COLL || __ballot(key != INT_MAX) == 0ull) return -1;
  return uniform_first(wave_min(key));
}

// adds the partner sums of the member at list position a (after spread_sums)
__device__ __forceinline__ void add_spread(const Lds &L, int wbase, int a, int lg, double *a1, double *j1) {
  const int pl = res_parts_log2(lg);
  for (int p = 0; p < (1 << pl); ++p) {
    const double *r = L.res + 6 * (wbase + (a << pl) + p);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      a1[d] += r[d];
      j1[d] += r[3 + d];
    }
  }
}

// One wavefront per cluster of 5..64 members (buckets 3..6), one member per
// lane.  In a block step usually only a few members are due; their partner
// sums are spread over the whole wavefront (spread_sums), so a step costs a
// few pair evaluations per lane instead of size - 1 in the due members'
// lanes.  The wavefront synchronises only with itself.  Same arithmetic per
// member as the other paths (hard_pair, star_term, correct, initial_level).
// MODE 0: plain; 1: park after A.budget block steps; 2: resume parked.
//
// COLL (MODE 0 only; clusters of 2..64 members): perfect-accretion
// collisions (Section 2.5.1).  Each slot belongs to a composite (its lowest
// slot, initially itself); the parts of a composite exchange no term and
// move with the mass-weighted mean of their accelerations and jerks.  The
// first colliding pair of a block step (lowest (slot, slot) order, found on
// the predicted states among the evaluated pairs) merges after the
// corrector, from the states at the block time (corrected for due members,
// predicted for the others): centre of mass and momentum, the dissipations
// eq. (e0) ... eq. (e3) (with W, with one and with 1 - W), acceleration and
// jerk of the composite at the block time, a new step from eta_0 refined
// until the block time is a multiple of it.  One merger per block step.
__device__ __forceinline__ double body_radius(double m, const HermArgs &A) { return cbrt(A.coll_r3 * m); }

// composite mean of q (three components) over the slots of composite cq:
// sum over its slots in slot order of m q, divided by the summed mass; the
// values m q of every slot are in L.res (three doubles per slot, at 6 slot)
__device__ __forceinline__ void composite_mean3(const Lds &L, int wbase, int size, int cq, int off, double *q) {
  double M = 0.0, s[3] = {0.0, 0.0, 0.0};
  for (int l = 0; l < size; ++l) {
    if (L.cid[wbase + l] != cq) continue;
    M += L.pm[wbase + l];
#pragma unroll
    for (int d = 0; d < 3; ++d) s[d] += L.res[6 * (wbase + l) + off + d];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) q[d] = s[d] / M;
}

template <int MODE, bool COLL>
__device__ __forceinline__ void wave_body(const HermArgs &A, const int32_t *blist, int count, int ci, const Lds &L,
                                          int wbase, int bk) {
  constexpr bool RESUME = MODE == 2, PARK = MODE == 1;
  static_assert(!COLL || MODE == 0, "collisions run without parking");
  const int lane = threadIdx.x & (WAVE - 1);
  if (ci >= count) return;  // uniform per wavefront; no workgroup barrier follows
  const int c = blist[ci];
  const int b = A.cl_ptr[c];
  const int size = uniform_first(A.cl_ptr[c + 1] - b);
  const bool mem = lane < size;
  const int gid = mem ? A.members[b + lane] : 0;
  const int64_t n = A.n;
  const int me = wbase + lane;
  double x[3] = {1.0, 0.0, 0.0}, v[3] = {0.0, 1.0, 0.0}, a0[3], j0[3];
  double m = 0.0, ro = 1.0;
  const double *src_x = RESUME ? A.pk.x : A.pos, *src_v = RESUME ? A.pk.v : A.vel;
  if (mem) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      x[d] = src_x[d * n + gid];
      v[d] = src_v[d * n + gid];
    }
    m = A.mass[gid];
    ro = A.ro[gid];
  }
  const double invi = 1.0 / ro;
  const double GM = A.GM, tick = A.tick;
  int mycid = lane;                                        // COLL: composite of this slot
  double eps[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};          // COLL: dissipations (summed on every lane)
  int ncoll = 0;
  wave_sync();
  L.pgm[me] = A.G * m;
  L.pinv[me] = invi;
  L.px[me] = x[0];
  L.py[me] = x[1];
  L.pz[me] = x[2];
  L.pvx[me] = v[0];
  L.pvy[me] = v[1];
  L.pvz[me] = v[2];
  if (COLL) {
    L.cid[me] = lane;
    L.rad[me] = mem ? body_radius(m, A) : 0.0;
    L.pm[me] = m;
  }
  if (mem) L.act[wbase + lane] = lane;  // every member: the forces at t = 0
  wave_sync();
  double E0 = 0.0;
  int lev = 0;
  int64_t t = 0;
  int nst = 0;
  star_term(x, v, GM, a0, j0);
  if (!RESUME) {
    spread_sums<COLL>(A, L, wbase, size, size, lane, __ballot(mem));
    double e = mem ? 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) -
                         GM * m * rsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2])
                   : 0.0;
    if (mem)
      for (int q = lane + 1; q < size; ++q) {
        const int sq = wbase + q;
        const double dx = L.px[sq] - x[0], dy = L.py[sq] - x[1], dz = L.pz[sq] - x[2];
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        e -= m * L.pgm[sq] * (1.0 - changeover_W(r * fmin(invi, L.pinv[sq]), A)) / r;
      }
    E0 = seg_sum(e, 6);
    wave_sync();
    if (mem) add_spread(L, wbase, lane, spread_lg(size, size), a0, j0);  // list position = lane
    lev = initial_level(a0, j0, mem, gid, A);
  } else {
    if (mem) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        a0[d] = A.pk.a[d * n + gid];
        j0[d] = A.pk.j[d * n + gid];
      }
      t = A.pk.t[gid];
      lev = A.pk.lev[gid];
    }
    nst = A.pk.nst[c];
    E0 = A.pk.e0[c];
  }
  const int64_t T = (int64_t)1 << TICK_BITS;
  const int budget = PARK ? A.budget : INT_MAX;
  const int max_iter = A.max_iter;
  int n_eval = 0;  // block steps in which this lane's member was due
  bool parked = false;
  for (int it = 0;; ++it) {
    const int64_t te = mem ? t + ((int64_t)1 << (TICK_BITS - lev)) : LLONG_MAX;
    const int64_t tn = wave_min_members(te, size);
    if (tn > T) break;  // every member has reached T (see seg_body)
    if (it == budget) {
      parked = true;
      break;
    }
    if (nst >= max_iter) {
      if (lane == 0) set_flag(A.cnt, P3T_FLAG_NSTEPS);
      break;
    }
    const bool active = mem && te == tn;
    const unsigned long long amask = __ballot(active);
    const int n_act = __popcll(amask);
    ++nst;
    double xp[3], vp[3];
    {
      const double dl = mem ? (double)(tn - t) * tick : 0.0;
      const double d2 = dl * dl * 0.5, d3 = dl * dl * dl * (1.0 / 6.0);
      predict(x, v, a0, j0, dl, d2, d3, xp, vp);
    }
    wave_sync();
    L.px[me] = xp[0];
    L.py[me] = xp[1];
    L.pz[me] = xp[2];
    L.pvx[me] = vp[0];
    L.pvy[me] = vp[1];
    L.pvz[me] = vp[2];
    const int apos = popc_below(amask);  // position among the due members
    if (active && n_act > 2) L.act[wbase + apos] = lane;
    double a1[3], j1[3];
    star_term(xp, vp, GM, a1, j1);  // while the LDS writes are in flight
    wave_sync();
    const int ckey = spread_sums<COLL>(A, L, wbase, size, n_act, lane, amask);
    wave_sync();
    if (active) add_spread(L, wbase, apos, spread_lg(size, n_act), a1, j1);
    if (COLL && __ballot(mem && mycid != lane) != 0ull) {
      // composites: every part moves with the mass-weighted mean
      wave_sync();
      if (active) {
        double *r = L.res + 6 * me;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          r[d] = m * a1[d];
          r[3 + d] = m * j1[d];
        }
      }
      wave_sync();
      if (active) {
        composite_mean3(L, wbase, size, mycid, 0, a1);
        composite_mean3(L, wbase, size, mycid, 3, j1);
      }
    }
    if (active) {
      const double h = (double)(tn - t) * tick;
      t = tn;
      correct(x, v, a0, j0, xp, vp, a1, j1, h, t, lev, A);
      ++n_eval;
    }
    if (COLL && ckey >= 0) {
      // ---- merger of the composites of slots ci_ < cj_ at tn
      const int ci_ = ckey / WAVE, cj_ = ckey % WAVE;
      double sx[3], sv[3];  // state at tn
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        sx[d] = active ? x[d] : xp[d];
        sv[d] = active ? v[d] : vp[d];
      }
      wave_sync();
      L.px[me] = sx[0];
      L.py[me] = sx[1];
      L.pz[me] = sx[2];
      L.pvx[me] = sv[0];
      L.pvy[me] = sv[1];
      L.pvz[me] = sv[2];
      wave_sync();
      const int CA = L.cid[wbase + ci_], CB = L.cid[wbase + cj_];
      const bool inA = mem && mycid == CA, inB = mem && mycid == CB;
      const double MA = wave_sum(inA ? m : 0.0), MB = wave_sum(inB ? m : 0.0), M = MA + MB;
      double xa[3], xb[3], va[3], vb[3], xn[3], vn[3];
      xa[0] = L.px[wbase + ci_], xa[1] = L.py[wbase + ci_], xa[2] = L.pz[wbase + ci_];
      xb[0] = L.px[wbase + cj_], xb[1] = L.py[wbase + cj_], xb[2] = L.pz[wbase + cj_];
      va[0] = L.pvx[wbase + ci_], va[1] = L.pvy[wbase + ci_], va[2] = L.pvz[wbase + ci_];
      vb[0] = L.pvx[wbase + cj_], vb[1] = L.pvy[wbase + cj_], vb[2] = L.pvz[wbase + cj_];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        xn[d] = (MA * xa[d] + MB * xb[d]) / M;
        vn[d] = (MA * va[d] + MB * vb[d]) / M;
      }
      const double dvx = va[0] - vb[0], dvy = va[1] - vb[1], dvz = va[2] - vb[2];
      const double e0 = 0.5 * (MA * MB / M) * (dvx * dvx + dvy * dvy + dvz * dvz);  // eq. (e0)
      const double rab = sqrt((xb[0] - xa[0]) * (xb[0] - xa[0]) + (xb[1] - xa[1]) * (xb[1] - xa[1]) +
                              (xb[2] - xa[2]) * (xb[2] - xa[2]));
      double e1 = 0.0, e1u = 0.0, e1h = 0.0, e3 = 0.0, e3u = 0.0, e3h = 0.0;
      if (inA)  // eq. (e1): every part of A with every part of B
        for (int l = 0; l < size; ++l) {
          if (L.cid[wbase + l] != CB) continue;
          const double W = changeover_W(rab * fmin(invi, L.pinv[wbase + l]), A);
          const double mm = m * L.pm[wbase + l];
          e1 -= mm * W / rab;
          e1u -= mm / rab;
          e1h -= mm * (1.0 - W) / rab;
        }
      if (inA || inB) {  // eq. (e3): the parts of A and B with the other members
        const double *xo = inA ? xa : xb;
        for (int l = 0; l < size; ++l) {
          const int cl = L.cid[wbase + l];
          if (cl == CA || cl == CB) continue;
          const int sl = wbase + l;
          const double iR = fmin(invi, L.pinv[sl]);
          const double ox = L.px[sl] - xo[0], oy = L.py[sl] - xo[1], oz = L.pz[sl] - xo[2];
          const double nx = L.px[sl] - xn[0], ny = L.py[sl] - xn[1], nz = L.pz[sl] - xn[2];
          const double r_o = sqrt(ox * ox + oy * oy + oz * oz), r_n = sqrt(nx * nx + ny * ny + nz * nz);
          const double Wo = changeover_W(r_o * iR, A), Wn = changeover_W(r_n * iR, A);
          const double mm = m * L.pm[sl];
          e3 -= mm * (Wo / r_o - Wn / r_n);
          e3u -= mm * (1.0 / r_o - 1.0 / r_n);
          e3h -= mm * ((1.0 - Wo) / r_o - (1.0 - Wn) / r_n);
        }
      }
      const double G = A.G;
      e1 = G * wave_sum(e1);
      e1u = G * wave_sum(e1u);
      e1h = G * wave_sum(e1h);
      e3 = G * wave_sum(e3);
      e3u = G * wave_sum(e3u);
      e3h = G * wave_sum(e3h);
      const double e2 = -GM * (MA / sqrt(xa[0] * xa[0] + xa[1] * xa[1] + xa[2] * xa[2]) +
                               MB / sqrt(xb[0] * xb[0] + xb[1] * xb[1] + xb[2] * xb[2]) -
                               M / sqrt(xn[0] * xn[0] + xn[1] * xn[1] + xn[2] * xn[2]));  // eq. (e2)
      eps[0] += e0;
      eps[1] += e1;
      eps[2] += e2;
      eps[3] += e3;
      eps[4] += e0 + e1u + e2 + e3u;
      eps[5] += e0 + e1h + e2 + e3h;
      ++ncoll;
      // the composite takes the merged state at tn
      const bool inC = inA || inB;
      const int cn = min(CA, CB);
      if (inC) {
        mycid = cn;
        t = tn;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          x[d] = sx[d] = xn[d];
          v[d] = sv[d] = vn[d];
        }
      }
      wave_sync();
      if (inC) {
        L.cid[me] = cn;
        L.rad[me] = body_radius(M, A);
        L.px[me] = xn[0];
        L.py[me] = xn[1];
        L.pz[me] = xn[2];
        L.pvx[me] = vn[0];
        L.pvy[me] = vn[1];
        L.pvz[me] = vn[2];
      }
      wave_sync();
      // its acceleration and jerk at tn from everyone's state at tn
      double an[3], jn[3];
      star_term(sx, sv, GM, an, jn);
      if (inC) {
        double pa[3] = {0.0, 0.0, 0.0}, pj[3] = {0.0, 0.0, 0.0};
        for (int l = 0; l < size; ++l) {
          const int sl = wbase + l;
          if (L.cid[sl] == cn) continue;
          hard_pair(L.px[sl] - sx[0], L.py[sl] - sx[1], L.pz[sl] - sx[2], L.pvx[sl] - sv[0], L.pvy[sl] - sv[1],
                    L.pvz[sl] - sv[2], L.pgm[sl], fmin(invi, L.pinv[sl]), A, pa, pj);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          an[d] += pa[d];
          jn[d] += pj[d];
        }
        double *r = L.res + 6 * me;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          r[d] = m * an[d];
          r[3 + d] = m * jn[d];
        }
      }
      wave_sync();
      if (inC) {
        composite_mean3(L, wbase, size, cn, 0, an);
        composite_mean3(L, wbase, size, cn, 3, jn);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          a0[d] = an[d];
          j0[d] = jn[d];
        }
        // first step after the merger: eta_0 criterion, on a multiple of the step
        const double anr = norm3(an), jnr = norm3(jn);
        const double dtc = jnr > 0.0 ? A.eta0 * anr / jnr : A.dt_soft;
        int kl = level_for(A.dt_soft, dtc, A.k_max);
        if (kl > A.k_max) {
          set_flag(A.cnt, P3T_FLAG_KMAX);
          kl = A.k_max;
        }
        while (kl < A.k_max && (tn & (((int64_t)1 << (TICK_BITS - kl)) - 1)) != 0) ++kl;
        lev = kl;
      }
    }
  }
  count_work(A, n_eval, size);
  if (PARK && parked) {
    int slot = 0;
    if (lane == 0) {
      const int k = atomicAdd(&A.pk.count[bk], 1);
      A.pk.lists[(int64_t)bk * A.n + k] = c;
      A.pk.nst[c] = nst;
      A.pk.e0[c] = E0;
      slot = atomicAdd(&A.pk.count[PK_MEM], size);
    }
    slot = __shfl(slot, 0, WAVE);
    if (mem) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        A.pk.x[d * n + gid] = x[d];
        A.pk.v[d * n + gid] = v[d];
        A.pk.a[d * n + gid] = a0[d];
        A.pk.j[d * n + gid] = j0[d];
      }
      A.pk.t[gid] = t;
      A.pk.lev[gid] = lev;
      A.pk.members[slot + lane] = gid;
      A.pk.flag[gid] = 1;
    }
    return;  // finished by the resume launch
  }
  // final energy (the pairs inside a composite left out)
  wave_sync();
  L.px[me] = x[0];
  L.py[me] = x[1];
  L.pz[me] = x[2];
  L.pvx[me] = v[0];
  L.pvy[me] = v[1];
  L.pvz[me] = v[2];
  wave_sync();
  double e = mem ? 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) -
                       GM * m * rsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2])
                 : 0.0;
  if (mem)
    for (int q = lane + 1; q < size; ++q) {
      const int sq = wbase + q;
      if (COLL && L.cid[sq] == mycid) continue;
      const double dx = L.px[sq] - x[0], dy = L.py[sq] - x[1], dz = L.pz[sq] - x[2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      e -= m * L.pgm[sq] * (1.0 - changeover_W(r * fmin(invi, L.pinv[sq]), A)) / r;
    }
  const double E1 = seg_sum(e, 6);
  if (mem) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      A.pos[d * n + gid] = x[d];
      A.vel[d * n + gid] = v[d];
    }
    if (A.dt_hard) A.dt_hard[gid] = ldexp(A.dt_soft, -lev);
    if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))) set_flag(A.cnt, P3T_FLAG_NAN);
    if (A.msteps) A.msteps[gid] = nst;
    if (COLL && A.merged) A.merged[gid] = A.members[b + mycid];
  }
  // with mergers the cluster's energy check adds the hard-energy dissipation
  if (lane == 0 && A.e_rel) A.e_rel[c] = fabs(E1 + eps[5] - E0) / fabs(E0);
  if (lane == 0 && A.nsteps) A.nsteps[c] = nst;
  if (COLL && lane == 0) {
    if (A.ceps)
      for (int q = 0; q < 6; ++q) A.ceps[6 * (int64_t)c + q] = eps[q];
    if (ncoll > 0) atomicAdd(&A.cnt->n_coll, (unsigned long long)ncoll);
  }
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

// exclusive scan of one int per thread over the workgroup; returns the total
__device__ __forceinline__ int block_excl_scan_i32(int v, int &excl, int64_t *sh) {
  const int w = threadIdx.x / WAVE, l = threadIdx.x & (WAVE - 1);
  const int incl = wave_incl_scan(v);
  __syncthreads();
  if (l == WAVE - 1) sh[w] = incl;
  __syncthreads();
  int off = 0, tot = 0;
  for (int q = 0; q < BIG_T / WAVE; ++q) {
    const int s = (int)sh[q];
    off += q < w ? s : 0;
    tot += s;
  }
  excl = off + incl - v;
  return tot;
}

// One 256-thread workgroup per cluster c, MPT members per thread.
template <int MPT, int MODE>
__device__ __forceinline__ void big_body(const HermArgs &A, int c, int bk, const Lds &L, int64_t *shi, double *shd) {
  constexpr bool RESUME = MODE == 2, PARK = MODE == 1;
  const int tid = threadIdx.x;
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
      const double *sx = RESUME ? A.pk.x : A.pos, *sv = RESUME ? A.pk.v : A.vel;
      for (int d = 0; d < 3; ++d) {
        x[u][d] = sx[d * n + gid[u]];
        v[u][d] = sv[d * n + gid[u]];
      }
      m[u] = A.mass[gid[u]];
      ro = A.ro[gid[u]];
    }
    invi[u] = 1.0 / ro;
    L.px[k] = x[u][0];
    L.py[k] = x[u][1];
    L.pz[k] = x[u][2];
    L.pvx[k] = v[u][0];
    L.pvy[k] = v[u][1];
    L.pvz[k] = v[u][2];
    L.pgm[k] = A.G * m[u];
    L.pinv[k] = invi[u];
    t[u] = 0;
  }
  __syncthreads();
  double e = 0.0;
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int k = tid + BIG_T * u;
    star_term(x[u], v[u], A.GM, a0[u], j0[u]);
    lev[u] = 0;
    if (!mem[u]) continue;
    if (RESUME) {  // a parked cluster continues from its saved state
      for (int d = 0; d < 3; ++d) {
        a0[u][d] = A.pk.a[d * n + gid[u]];
        j0[u][d] = A.pk.j[d * n + gid[u]];
      }
      t[u] = A.pk.t[gid[u]];
      lev[u] = A.pk.lev[gid[u]];
      continue;
    }
    e += 0.5 * m[u] * (v[u][0] * v[u][0] + v[u][1] * v[u][1] + v[u][2] * v[u][2]) -
         A.GM * m[u] * rsqrt(x[u][0] * x[u][0] + x[u][1] * x[u][1] + x[u][2] * x[u][2]);
    for (int q = 0; q < size; ++q) {
      if (q == k) continue;
      const double dx = L.px[q] - x[u][0], dy = L.py[q] - x[u][1], dz = L.pz[q] - x[u][2];
      const double invR = fmin(invi[u], L.pinv[q]);
      hard_pair(dx, dy, dz, L.pvx[q] - v[u][0], L.pvy[q] - v[u][1], L.pvz[q] - v[u][2], L.pgm[q], invR, A, a0[u],
                j0[u]);
      if (q > k) {
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        e -= m[u] * L.pgm[q] * (1.0 - changeover_W(r * invR, A)) / r;
      }
    }
    lev[u] = initial_level(a0[u], j0[u], true, gid[u], A);
  }
  double E0 = block_sum(e, shd);
  const int64_t T = (int64_t)1 << TICK_BITS;
  int it = 0;  // block steps taken
  if (RESUME) {
    E0 = A.pk.e0[c];
    it = A.pk.nst[c];
  }
  const int budget = PARK ? A.budget : INT_MAX;
  int n_ev = 0;  // evaluations of this thread's members
  for (int its = 0;; ++it, ++its) {
    int64_t tel = LLONG_MAX;
#pragma unroll
    for (int u = 0; u < MPT; ++u)
      if (mem[u]) {
        const int64_t te = t[u] + ((int64_t)1 << (TICK_BITS - lev[u]));
        tel = te < tel ? te : tel;
      }
    const int64_t tn = uniform_first64(block_min_i64(tel, shi));
    if (tn > T) break;  // every member has reached T (see seg_body)
    if (its == budget) {  // uniform: park the cluster and stop
      __shared__ int pslot;
      if (tid == 0) {
        const int k = atomicAdd(&A.pk.count[bk], 1);
        A.pk.lists[(int64_t)bk * n + k] = c;
        A.pk.nst[c] = it;
        A.pk.e0[c] = E0;
        pslot = atomicAdd(&A.pk.count[PK_MEM], size);
      }
      __syncthreads();
      const int slot = pslot;
#pragma unroll
      for (int u = 0; u < MPT; ++u) {
        if (!mem[u]) continue;
        for (int d = 0; d < 3; ++d) {
          A.pk.x[d * n + gid[u]] = x[u][d];
          A.pk.v[d * n + gid[u]] = v[u][d];
          A.pk.a[d * n + gid[u]] = a0[u][d];
          A.pk.j[d * n + gid[u]] = j0[u][d];
        }
        A.pk.t[gid[u]] = t[u];
        A.pk.lev[gid[u]] = lev[u];
        A.pk.members[slot + tid + BIG_T * u] = gid[u];
        A.pk.flag[gid[u]] = 1;
      }
      count_work(A, n_ev, size);
      return;  // the whole workgroup: finished by the resume launch
    }
    if (it >= A.max_iter) {
      if (tid == 0) set_flag(A.cnt, P3T_FLAG_NSTEPS);
      break;
    }
    double xp[MPT][3], vp[MPT][3];
#pragma unroll
    for (int u = 0; u < MPT; ++u) {
      const double dl = mem[u] ? (double)(tn - t[u]) * A.tick : 0.0;
      const double d2 = dl * dl * 0.5, d3 = dl * dl * dl * (1.0 / 6.0);
      predict(x[u], v[u], a0[u], j0[u], dl, d2, d3, xp[u], vp[u]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MPT; ++u) {
      const int k = tid + BIG_T * u;
      L.px[k] = xp[u][0];
      L.py[k] = xp[u][1];
      L.pz[k] = xp[u][2];
      L.pvx[k] = vp[u][0];
      L.pvy[k] = vp[u][1];
      L.pvz[k] = vp[u][2];
    }
    __syncthreads();
    // Active members (due at tn).  With few of them, each active member's
    // partner loop is spread over the 64 lanes of a wavefront (wavefronts
    // take active members in turn) and reduced; otherwise every thread
    // loops over all partners of its own members.
    bool act[MPT];
    int slot[MPT];
    int na_me = 0;
#pragma unroll
    for (int u = 0; u < MPT; ++u) {
      act[u] = mem[u] && t[u] + ((int64_t)1 << (TICK_BITS - lev[u])) == tn;
      na_me += act[u] ? 1 : 0;
    }
    int base_me = 0;
    const int na = block_excl_scan_i32(na_me, base_me, shi);
    const bool spread = L.act != nullptr && na <= BIG_ACT && 2 * na <= size;
    if (spread) {
      int q = base_me;
#pragma unroll
      for (int u = 0; u < MPT; ++u) {
        slot[u] = act[u] ? q : -1;
        if (act[u]) L.act[q++] = tid + BIG_T * u;
      }
      __syncthreads();
      const int w = tid / WAVE, lane = tid & (WAVE - 1);
      for (int a = w; a < na; a += BIG_T / WAVE) {  // uniform per wavefront
        const int k = L.act[a];
        const double xk = L.px[k], yk = L.py[k], zk = L.pz[k], vxk = L.pvx[k], vyk = L.pvy[k], vzk = L.pvz[k];
        const double ik = L.pinv[k];
        double pa[3] = {0.0, 0.0, 0.0}, pj[3] = {0.0, 0.0, 0.0};
        for (int qq = lane; qq < size; qq += WAVE) {
          if (qq == k) continue;
          hard_pair(L.px[qq] - xk, L.py[qq] - yk, L.pz[qq] - zk, L.pvx[qq] - vxk, L.pvy[qq] - vyk, L.pvz[qq] - vzk,
                    L.pgm[qq], fmin(ik, L.pinv[qq]), A, pa, pj);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          pa[d] = wave_sum(pa[d]);
          pj[d] = wave_sum(pj[d]);
        }
        if (lane == 0) {
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            L.res[6 * a + d] = pa[d];
            L.res[6 * a + 3 + d] = pj[d];
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < MPT; ++u) {
      const int k = tid + BIG_T * u;
      if (!act[u]) continue;
      double a1[3], j1[3];
      star_term(xp[u], vp[u], A.GM, a1, j1);
      if (spread) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          a1[d] += L.res[6 * slot[u] + d];
          j1[d] += L.res[6 * slot[u] + 3 + d];
        }
      } else {
        for (int q = 0; q < size; ++q) {
          if (q == k) continue;
          hard_pair(L.px[q] - xp[u][0], L.py[q] - xp[u][1], L.pz[q] - xp[u][2], L.pvx[q] - vp[u][0],
                    L.pvy[q] - vp[u][1], L.pvz[q] - vp[u][2], L.pgm[q], fmin(invi[u], L.pinv[q]), A, a1, j1);
        }
      }
      const double h = (double)(tn - t[u]) * A.tick;
      t[u] = tn;
      correct(x[u], v[u], a0[u], j0[u], xp[u], vp[u], a1, j1, h, t[u], lev[u], A);
      ++n_ev;
    }
  }
  count_work(A, n_ev, size);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int k = tid + BIG_T * u;
    L.px[k] = x[u][0];
    L.py[k] = x[u][1];
    L.pz[k] = x[u][2];
    L.pvx[k] = v[u][0];
    L.pvy[k] = v[u][1];
    L.pvz[k] = v[u][2];
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
      const double dx = L.px[q] - x[u][0], dy = L.py[q] - x[u][1], dz = L.pz[q] - x[u][2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      e -= m[u] * L.pgm[q] * (1.0 - changeover_W(r * fmin(invi[u], L.pinv[q]), A)) / r;
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
  if (A.msteps)
    for (int u = 0; u < MPT; ++u)
      if (mem[u]) A.msteps[gid[u]] = it;
}

// Buckets 0..6 (sizes 1..64) in one launch of 256-thread workgroups; the
// block index selects the bucket (uniform per workgroup).  COLL: every
// cluster of 2..64 members takes the wavefront path with collisions.
__host__ __device__ constexpr int clusters_per_wave(int bk, bool coll) {
  return (coll && bk >= 1) || bk >= WAVE_BK0 ? 1 : WAVE >> (bk + lanes_per_member_log2(bk));
}

template <int MODE, bool COLL = false>
__global__ __launch_bounds__(BIG_T) void k_herm_fused(HermArgs A) {
  __shared__ double lds[8][BIG_T];
  __shared__ int act[BIG_T];
  __shared__ double res[6 * BIG_T];
  constexpr int NC = COLL ? BIG_T : 1;
  __shared__ int cid[NC];
  __shared__ double rad[NC], pm[NC];
  const Lds L = {lds[0], lds[1], lds[2], lds[3], lds[4], lds[5], lds[6], lds[7], act, res, cid, rad, pm};
  // workgroups are dispatched roughly in index order: the buckets of the
  // larger clusters (fewer, longer chains) take the first indices, the
  // singletons the last, so the long chains start first
  const int blk = gridDim.x - 1 - blockIdx.x;
  // bucket of this workgroup (boff is non-decreasing).  Only constant
  // indices into the argument struct: a run-time index would make the
  // compiler copy the whole struct to per-lane scratch memory.
  int rg = 0, first = 0;
#pragma unroll
  for (int q = 1; q < FUSED_REGIONS; ++q)
    if (A.boff[q] <= blk) {
      rg = q;
      first = A.boff[q];
    }
  const int local = blk - first;
  const bool close = rg >= 7;  // the clusters of bucket rg - 6 with a close pair
  const int bk = close ? rg - 6 : rg;
  const int w = threadIdx.x / WAVE;
  const int wbase = w * WAVE;
  const int ci0 = (local * (BIG_T / WAVE) + w) * clusters_per_wave(bk, COLL);
  int count = 0;
#pragma unroll
  for (int q = 0; q < 7; ++q)
    if (q == bk) count = A.bcount[q];  // constant indices only (see above)
#pragma unroll
  for (int q = 1; q < 4; ++q)
    if (close && q == bk) count = A.ccount[q];
  // the close clusters sit at the end of their bucket's list
  const int32_t *blist = A.blists + (int64_t)bk * A.nc + (close ? A.nc - count : 0);
  if (bk >= (COLL ? 1 : WAVE_BK0))
    wave_body<MODE, COLL>(A, blist, count, ci0, L, wbase, bk);
  else if (bk == 1)
    seg_body<MODE, 1>(A, blist, count, ci0, L, wbase, bk);
  else
    seg_body<MODE>(A, blist, count, ci0, L, wbase, bk);
}

template <int MPT, int MODE>
__global__ __launch_bounds__(BIG_T) void k_herm_big(HermArgs A, int bk) {
  __shared__ double lds[8][BIG_T * MPT];
  __shared__ int64_t shi[BIG_T / WAVE];
  __shared__ double shd[BIG_T / WAVE];
  // the lane-parallel partner loop needs 6.6 KB more LDS, which the
  // 1024-member variant does not have within 64 KB per workgroup
  constexpr int NACT = MPT <= 2 ? BIG_ACT : 1;
  __shared__ int act[NACT];
  __shared__ double res[6 * NACT];
  const Lds L = {lds[0], lds[1], lds[2], lds[3], lds[4], lds[5], lds[6], lds[7], MPT <= 2 ? act : nullptr, res};
  big_body<MPT, MODE>(A, A.blists[(int64_t)bk * A.nc + blockIdx.x], bk, L, shi, shd);
}

// ---------------------------------------------------------------- bucketing
// Buckets: 0..2 the packed wavefront segments (1, 2, 3-4 members), 3..6 one
// wavefront per cluster (5-8, 9-16, 17-32, 33-64), 7..9 one workgroup per
// cluster (65-256, 257-512, 513-1024), 10 the percolated-cluster path.
__device__ __forceinline__ int bucket_of(int size, int cap) {
  if (size > cap) return 10;  // the percolated-cluster path
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

// Bucket the clusters by size with one atomic per bucket per wavefront; also
// validate the caller's cluster arrays (offsets non-decreasing from >= 0,
// members in [0, n)); a violation sets bcount[BC_BAD] and nothing is integrated.
// Bucket lists.  Each workgroup owns a contiguous range of clusters: it
// counts its clusters per bucket in LDS, reserves its share of every bucket
// with one global atomic per bucket, then writes the entries in cluster
// order.  (One atomic per wavefront and bucket contended on the same eleven
// counters across the whole grid.)
__device__ __forceinline__ int cluster_bucket(int64_t c, int64_t n, int cap, const int32_t *__restrict__ cl_ptr,
                                              const int32_t *__restrict__ members, int32_t *__restrict__ bcount) {
  const int a = cl_ptr[c], b = cl_ptr[c + 1];
  bool ok = a >= 0 && b >= a;
  for (int k = a; ok && k < b; ++k) {
    const int g = members[k];
    ok = g >= 0 && (int64_t)g < n;
  }
  if (!ok) {
    atomicOr(&bcount[BC_BAD], 1);
    return -1;
  }
  return b > a ? bucket_of(b - a, cap) : -1;
}

struct BucketArgs {
  int64_t nc_host;
  const int64_t *nc_dev;
  int64_t stride, n;
  int cap;  // clusters above this many members take the percolated-cluster path
  const int32_t *cl_ptr, *members;
  int32_t *bcount, *blists;
  int32_t *cl_bk;  // category chosen per cluster (between the sweeps)
  DevCounters *cnt;
  int reset_work;  // zero the Hermite work counters
  CloseSrc close;  // member flags that make a cluster of buckets 1..3 close
  int32_t *wgc;    // per-chunk category counts, then their offsets (N_CATS rows)
};

__device__ bool cluster_close(int a, int b, const BucketArgs &B) {
  for (int p = a; p < b; ++p) {
    const int g = B.members[p];
    if ((B.close.a && B.close.a[g]) || (B.close.b && B.close.b[g])) return true;
  }
  return false;
}

// Categories: the buckets 0..10, and N_BUCKETS + k - 1 for the clusters of
// bucket k = 1..3 with a close pair.  The close ones are written from the
// end of their bucket's list backwards (count in bcount[HERM_BC_CLOSE0 + k
// - 1]), the others from its start.  Three launches, each over one
// 256-cluster chunk per workgroup: the category counts of every chunk
// (k_bucket_count), their exclusive scan over the chunks per category
// (k_bucket_scan, one workgroup per category), and the entries in cluster
// order (k_bucket_write).  B.wgc holds N_CATS rows of nchunk counts.
constexpr int N_CATS = N_BUCKETS + 3;
constexpr int BK_T = 256;

__device__ __forceinline__ int64_t bucket_nc(const BucketArgs &B) {
  return B.nc_dev ? *B.nc_dev : B.nc_host;  // clusters (at most stride)
}

// category of cluster c (-1: empty or beyond the count)
__device__ __forceinline__ int cluster_category(const BucketArgs &B, int64_t c, int64_t nc) {
  if (c >= nc) return -1;
  int cat = cluster_bucket(c, B.n, B.cap, B.cl_ptr, B.members, B.bcount);
  if (cat >= 1 && cat <= 3 && (B.close.a || B.close.b) && cluster_close(B.cl_ptr[c], B.cl_ptr[c + 1], B))
    cat += N_BUCKETS - 1;
  return cat;
}

// per wavefront: the mask of its lanes in category q, for every q (all lanes
// take part); returns this lane's mask
__device__ __forceinline__ unsigned long long cat_masks(int cat, int *wcount, int lane) {
  unsigned long long mine = 0ull;
  for (int q = 0; q < N_CATS; ++q) {
    const unsigned long long mask = __ballot(cat == q);
    if (lane == 0) wcount[q] = (int)__popcll(mask);
    if (q == cat) mine = mask;
  }
  return mine;
}

__global__ __launch_bounds__(BK_T) void k_bucket_count(BucketArgs B, int nchunk) {
  __shared__ int wc[BK_T / WAVE][N_CATS];
  const int t = threadIdx.x, lane = t & (WAVE - 1), w = t / WAVE;
  const int64_t nc = bucket_nc(B);
  if (blockIdx.x == 0 && t == 0) {
    B.bcount[BC_NC] = (int32_t)nc;
    if (B.reset_work) {  // the work counters of this hard part
      B.cnt->n_heval = 0;
      B.cnt->n_hpair = 0;
      B.cnt->n_coll = 0;
    }
  }
  const int64_t c = (int64_t)blockIdx.x * BK_T + t;
  const int cat = cluster_category(B, c, nc);
  if (c < nc) B.cl_bk[c] = cat;
  cat_masks(cat, wc[w], lane);
  __syncthreads();
  if (t < N_CATS) {
    int tot = 0;
    for (int u = 0; u < BK_T / WAVE; ++u) tot += wc[u][t];
    B.wgc[(int64_t)t * nchunk + blockIdx.x] = tot;
  }
}

// row q of wgc becomes its exclusive scan over the chunks; the row total is
// the category's count
__global__ __launch_bounds__(BK_T) void k_bucket_scan(BucketArgs B, int nchunk) {
  __shared__ int ws[BK_T / WAVE];
  const int q = blockIdx.x, t = threadIdx.x, lane = t & (WAVE - 1), w = t / WAVE;
  int32_t *row = B.wgc + (int64_t)q * nchunk;
  int carry = 0;
  for (int c0 = 0; c0 < nchunk; c0 += BK_T) {  // uniform
    const int i = c0 + t;
    const int v = i < nchunk ? row[i] : 0;
    const int incl = wave_incl_scan(v);
    if (lane == WAVE - 1) ws[w] = incl;
    __syncthreads();
    int before = 0, chunk = 0;
    for (int u = 0; u < BK_T / WAVE; ++u) {
      before += u < w ? ws[u] : 0;
      chunk += ws[u];
    }
    if (i < nchunk) row[i] = carry + before + incl - v;
    carry += chunk;
    __syncthreads();  // ws is rewritten by the next chunk
  }
  if (t == 0) {
    if (q < N_BUCKETS)
      B.bcount[q] = carry;
    else
      B.bcount[HERM_BC_CLOSE0 + q - N_BUCKETS] = carry;
  }
}

__global__ __launch_bounds__(BK_T) void k_bucket_write(BucketArgs B, int nchunk) {
  __shared__ int wc[BK_T / WAVE][N_CATS];
  const int t = threadIdx.x, lane = t & (WAVE - 1), w = t / WAVE;
  const int64_t nc = bucket_nc(B);
  const int64_t c = (int64_t)blockIdx.x * BK_T + t;
  const int cat = c < nc ? B.cl_bk[c] : -1;  // as decided by k_bucket_count
  const unsigned long long mine = cat_masks(cat, wc[w], lane);
  __syncthreads();
  if (cat >= 0) {
    int off = 0;
    for (int u = 0; u < w; ++u) off += wc[u][cat];  // wavefronts take their slots in order
    const int64_t k = (int64_t)B.wgc[(int64_t)cat * nchunk + blockIdx.x] + off + popc_below(mine);
    if (cat < N_BUCKETS)
      B.blists[(int64_t)cat * B.stride + k] = (int32_t)c;
    else
      B.blists[(int64_t)(cat - N_BUCKETS + 1) * B.stride + B.stride - 1 - k] = (int32_t)c;
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

// Bucket lists and counts (one host synchronisation); hc receives the
// BC_WORDS words (the park counts are zero).
hipError_t herm_bucket(p3t_ctx *c, int64_t n, int64_t nc, const int32_t *cl_ptr, const int32_t *cl_members,
                       const int64_t *nc_dev, int32_t *hc, const CloseSrc &close) {
  hipError_t e = herm_bucket_enqueue(c, c->stream, n, nc, cl_ptr, cl_members, nc_dev, hc, true, close);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
  if (hc[BC_BAD]) return hipErrorInvalidDevicePointer;  // malformed cluster arrays
  return hipSuccess;
}

// The bucket kernel and the copy of the bucket words to hc (host memory) on
// stream s, without waiting.
hipError_t herm_bucket_enqueue(p3t_ctx *c, hipStream_t s, int64_t n, int64_t nc, const int32_t *cl_ptr,
                               const int32_t *cl_members, const int64_t *nc_dev, int32_t *hc, bool reset_work,
                               const CloseSrc &close) {
  hipError_t e;
  if ((e = fill_i32(c->herm_bcount, 0, BC_WORDS, s)) != hipSuccess) return e;
  BucketArgs B;
  B.nc_host = nc;
  B.nc_dev = nc_dev;
  B.stride = nc;
  B.n = n;
  B.cap = std::min(c->P.cluster_cap, 1024);
  B.cl_ptr = cl_ptr;
  B.members = cl_members;
  B.bcount = c->herm_bcount;
  B.blists = c->herm_blists;
  B.cl_bk = c->herm_clbk;
  B.cnt = c->cnt;
  B.reset_work = reset_work ? 1 : 0;
  B.close = close;
  // the per-chunk counts use the radix sort's histogram buffer, which is
  // free here (it holds 256 entries per 2048 keys, these N_CATS per 256)
  const int64_t nchunk = std::max<int64_t>(1, (nc + BK_T - 1) / BK_T);
  if (nchunk * N_CATS > c->radix_hist_cap || nchunk > INT32_MAX) return hipErrorInvalidValue;
  B.wgc = reinterpret_cast<int32_t *>(c->radix_hist);
  hipLaunchKernelGGL(k_bucket_count, dim3((unsigned)nchunk), dim3(BK_T), 0, s, B, (int)nchunk);
  hipLaunchKernelGGL(k_bucket_scan, dim3(N_CATS), dim3(BK_T), 0, s, B, (int)nchunk);
  hipLaunchKernelGGL(k_bucket_write, dim3((unsigned)nchunk), dim3(BK_T), 0, s, B, (int)nchunk);
  return hipMemcpyAsync(hc, c->herm_bcount, sizeof(int32_t) * BC_WORDS, hipMemcpyDeviceToHost, s);
}

__global__ void k_herm_reset_work(DevCounters *cnt) {
  cnt->n_heval = 0;
  cnt->n_hpair = 0;
  cnt->n_coll = 0;
}

// The Hermite work counters zeroed on stream s (a kernel, not a memset: the
// caller may be capturing).
hipError_t herm_reset_work(p3t_ctx *c, hipStream_t s) {
  hipLaunchKernelGGL(k_herm_reset_work, dim3(1), dim3(1), 0, s, c->cnt);
  return hipGetLastError();
}

__global__ void k_huge_flag(DevCounters *cnt, unsigned bits) { set_flag(cnt, bits); }

namespace {
hipError_t huge_clusters(p3t_ctx *c, const HermArgs &A, int count, hipStream_t s);
}

// Integrates the clusters of the buckets (counts in hc[0, 11)) on stream s;
// clusters of 65 members and more go to stream s_big (which may be s),
// joined back into s at the end.  budget > 0 parks the clusters still
// running after `budget` block steps (their counts land in
// the park words of herm_bcount).  resume = 1 continues the parked clusters
// (counts in hc[HERM_BC_PARK0, + 10)) and writes their final state into the
// park buffers' x and v.
hipError_t herm_launch(p3t_ctx *c, int64_t n, int64_t stride, const int32_t *cl_ptr, const int32_t *cl_members,
                       double *pos3, double *vel3, const double *mass, const double *r_out, double *dt_hard,
                       double *e_rel_err, int32_t *n_steps, int32_t *steps_out, const int32_t *hc, int budget,
                       int resume, hipStream_t s, hipStream_t s_big, hipEvent_t ev_fork, hipEvent_t ev_join,
                       const HermColl *coll) {
  hipError_t e;
  const bool collide = coll != nullptr;
  if (collide && (resume || budget > 0)) return hipErrorInvalidValue;  // collisions run without parking
  const p3t_params &P = c->P;
  HermArgs A;
  A.cl_ptr = cl_ptr;
  A.members = cl_members;
  A.blists = resume ? c->pk_lists : c->herm_blists;
  A.nc = resume ? n : stride;
  A.pos = resume ? c->pk_x : pos3;
  A.vel = resume ? c->pk_v : vel3;
  A.mass = mass;
  A.ro = r_out;
  A.dt_hard = dt_hard;
  A.e_rel = e_rel_err;
  A.nsteps = n_steps;
  A.msteps = steps_out;
  A.budget = budget;
  A.pk.x = c->pk_x;
  A.pk.v = c->pk_v;
  A.pk.a = c->pk_a;
  A.pk.j = c->pk_j;
  A.pk.t = c->pk_t;
  A.pk.lev = c->pk_lev;
  A.pk.nst = c->pk_nst;
  A.pk.e0 = c->pk_e0;
  A.pk.count = c->herm_bcount + HERM_BC_PARK0;
  A.pk.lists = c->pk_lists;
  A.pk.members = c->slow_list;
  A.pk.flag = c->slow_flag;
  if ((budget > 0 || resume) && !c->pk_x) return hipErrorInvalidValue;  // park buffers not allocated
  A.n = n;
  A.G = P.G;
  A.GM = P.G * P.m_star;
  A.gamma = P.gamma;
  A.inv1mg = 1.0 / (1.0 - P.gamma);
  A.eta = P.eta;
  A.eta0 = P.eta0;
  A.dt_soft = P.dt_soft;
  A.tick = std::ldexp(P.dt_soft, -TICK_BITS);
  {
    const double h = P.dt_soft, h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
    A.inv_dt2 = 1.0 / h2;
    A.inv_dt3 = 1.0 / h3;
    A.dt3_6 = h3 / 6.0;
    A.dt4_24 = h4 / 24.0;
    A.dt5_120 = h5 / 120.0;
    A.dt_soft2 = h2;
  }
  A.k_max = P.k_max;
  A.max_iter = 1 << 22;
  A.coll_f = collide ? coll->f : 0.0;
  A.coll_r3 = collide ? coll->r3 : 0.0;
  A.merged = collide ? coll->merged : nullptr;
  A.ceps = collide ? coll->ceps : nullptr;
  A.cnt = c->cnt;
  host_changeover_coeffs(P.gamma, A);
  for (int bk = 0; bk < N_BUCKETS; ++bk) A.bcount[bk] = resume ? (bk < 10 ? hc[HERM_BC_PARK0 + bk] : 0) : hc[bk];
  A.ccount[0] = 0;
  for (int k = 1; k < 4; ++k) A.ccount[k] = resume ? 0 : hc[HERM_BC_CLOSE0 + k - 1];
  // clusters of one member: their two-body orbits, exactly (they never
  // park); launched beside the big clusters below when there are any
  const int32_t n_single = (P.isolated == 1 && !resume) ? A.bcount[0] : 0;
  if (n_single > 0) A.bcount[0] = 0;
  // fused launch: buckets 0..6 (clusters per 256-thread block = 4 * 64 / SEG /
  // lanes per member); the clusters of 65 members and more run at the same
  // time in their own launches (one workgroup each)
  // regions 0..6 the buckets, 7..9 the close clusters of buckets 1..3
  // (dispatched first)
  int blocks = 0;
  for (int rg = 0; rg < FUSED_REGIONS; ++rg) {
    A.boff[rg] = blocks;
    const int bk = rg < 7 ? rg : rg - 6;
    const int per_block = (BIG_T / WAVE) * clusters_per_wave(bk, collide);
    const int cnt = rg < 7 ? A.bcount[bk] : A.ccount[bk];
    blocks += (cnt + per_block - 1) / per_block;
  }
  for (int rg = FUSED_REGIONS; rg <= N_BUCKETS; ++rg) A.boff[rg] = blocks;
  // clusters above 1024 members (never parked): the percolated-cluster path
  const int n_huge = resume ? 0 : A.bcount[10];
  const bool big = A.bcount[7] > 0 || A.bcount[8] > 0 || A.bcount[9] > 0 || n_huge > 0;
  hipStream_t s2 = s;
  if (big && blocks > 0 && s_big != s) {
    s2 = s_big;
    if ((e = hipEventRecord(ev_fork, s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s2, ev_fork, 0)) != hipSuccess) return e;
  }
  if (n_single > 0 && (e = kepler_singles(n, n_single, A.blists, cl_ptr, cl_members, A.GM, P.dt_soft, pos3, vel3,
                                           dt_hard, steps_out, e_rel_err, n_steps, c->cnt, s2)) != hipSuccess)
    return e;
  const int mode = resume ? 2 : (budget > 0 ? 1 : 0);
#define P3T_LAUNCH_BIG(MPT, BK)                                                                         \
  if (A.bcount[BK] > 0) {                                                                               \
    if (mode == 2)                                                                                      \
      hipLaunchKernelGGL((k_herm_big<MPT, 2>), dim3(A.bcount[BK]), dim3(BIG_T), 0, s2, A, BK);          \
    else if (mode == 1)                                                                                 \
      hipLaunchKernelGGL((k_herm_big<MPT, 1>), dim3(A.bcount[BK]), dim3(BIG_T), 0, s2, A, BK);          \
    else                                                                                                \
      hipLaunchKernelGGL((k_herm_big<MPT, 0>), dim3(A.bcount[BK]), dim3(BIG_T), 0, s2, A, BK);          \
  }
  P3T_LAUNCH_BIG(1, 7)
  P3T_LAUNCH_BIG(2, 8)
  P3T_LAUNCH_BIG(4, 9)
#undef P3T_LAUNCH_BIG
  if (blocks > 0) {
    if (resume)
      hipLaunchKernelGGL(k_herm_fused<2>, dim3(blocks), dim3(BIG_T), 0, s, A);
    else if (budget > 0)
      hipLaunchKernelGGL(k_herm_fused<1>, dim3(blocks), dim3(BIG_T), 0, s, A);
    else if (collide)
      hipLaunchKernelGGL((k_herm_fused<0, true>), dim3(blocks), dim3(BIG_T), 0, s, A);
    else
      hipLaunchKernelGGL(k_herm_fused<0>, dim3(blocks), dim3(BIG_T), 0, s, A);
  }
  // collisions are looked for in clusters of up to 64 members only
  if (collide && big)
    hipLaunchKernelGGL(k_huge_flag, dim3(1), dim3(1), 0, s, c->cnt, (unsigned)P3T_FLAG_COLL_UNCHECKED);
  if (n_huge > 0) {
    // issued after the fused launch, so that it runs beside them; the host
    // waits here until the percolated clusters are done
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = huge_clusters(c, A, n_huge, s2)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_huge_flag, dim3(1), dim3(1), 0, s2, c->cnt, (unsigned)P3T_FLAG_BIG_CLUSTER);
  }
  if (s2 != s) {  // join
    if ((e = hipEventRecord(ev_join, s2)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, ev_join, 0)) != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t aux_streams(p3t_ctx *c) {
  hipError_t e;
  if (!c->aux_stream && (e = hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking)) != hipSuccess) return e;
  if (!c->slow_stream && (e = hipStreamCreateWithFlags(&c->slow_stream, hipStreamNonBlocking)) != hipSuccess)
    return e;
  if (!c->aux_ev[0])
    for (auto &ev : c->aux_ev)
      if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t hermite_clusters(p3t_ctx *c, int64_t n, int64_t nc, const int32_t *cl_ptr, const int32_t *cl_members,
                            double *pos3, double *vel3, const double *mass, const double *r_out, double *dt_hard,
                            double *e_rel_err, int32_t *n_steps, const int64_t *nc_dev, int64_t *nc_out,
                            int32_t *steps_out, const HermColl *coll) {
  if (nc_out) *nc_out = 0;
  if (nc <= 0) return hipSuccess;  // with nc_dev, nc is an upper bound (the particle count)
  int32_t hc[BC_WORDS];
  hipError_t e = herm_bucket(c, n, nc, cl_ptr, cl_members, nc_dev, hc);
  if (nc_out) *nc_out = hc[BC_NC];
  if (e != hipSuccess) return e;
  if ((e = aux_streams(c)) != hipSuccess) return e;
  return herm_launch(c, n, nc, cl_ptr, cl_members, pos3, vel3, mass, r_out, dt_hard, e_rel_err, n_steps, steps_out, hc,
                     0, 0, c->stream, c->aux_stream, c->aux_ev[0], c->aux_ev[1], coll);
}

// ---------------------------------------------------------------- percolated clusters
// Clusters above 1024 members: the neighbour graph has percolated (Section
// 3.2.3 of the paper integrates such a cluster directly, with Hermite, on
// one process).  Here the cluster is spread over the whole chip with its
// member states in device memory, and each block step is two launches:
//   k_huge_predict  every member predicted to the block time tn (the
//                   minimum next time of the previous step), the active
//                   members (due at tn) listed and flagged;
//   k_huge_step     one wavefront per active member sums its partners
//                   lane-parallel over all members' predicted states, then
//                   corrects it and takes its new level; every member's
//                   next time goes into an atomic minimum, the next tn.
// The host issues the launches in batches and reads a done word after each
// batch (no grid-wide barrier inside a kernel).  Same arithmetic per member
// as the other paths (hard_pair, star_term, correct, initial_level), with
// the partner sums added in wave-reduction order.
struct HugeArgs {
  int c, M;                          // cluster index, members
  const int32_t *mem;                // the cluster's members (cl_members + cl_ptr[c])
  double *x, *v, *a, *j, *xp, *vp;   // 3M each, component d of member k at d * M + k
  double *m, *gm, *inv, *e;          // M each: mass, G m, 1 / r_out, energy partials
  int64_t *t;                        // M: time in ticks
  int32_t *lev, *act, *aflag;        // M: level, active list, active flag
  unsigned long long *tn;            // [2] next block time (double-buffered by step parity)
  int32_t *nact;                     // [2] active members of the step
  int32_t *nst;                      // block steps so far
  int32_t *done;                     // 1 once every member reached dt_soft
  double *E;                         // [0] energy before, [1] after
};
constexpr int HUGE_T = 256;

__global__ __launch_bounds__(HUGE_T) void k_huge_load(HermArgs A, HugeArgs H) {
  const int64_t n = A.n;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    H.tn[0] = H.tn[1] = ~0ull;
    H.nact[0] = H.nact[1] = 0;
    *H.nst = 0;
    *H.done = 0;
  }
  for (int k = blockIdx.x * HUGE_T + threadIdx.x; k < H.M; k += gridDim.x * HUGE_T) {
    const int64_t g = H.mem[k];
    double x[3], v[3];
    for (int d = 0; d < 3; ++d) {
      x[d] = A.pos[d * n + g];
      v[d] = A.vel[d * n + g];
      H.x[d * H.M + k] = x[d];
      H.v[d * H.M + k] = v[d];
    }
    const double m = A.mass[g];
    H.m[k] = m;
    H.gm[k] = A.G * m;
    H.inv[k] = 1.0 / A.ro[g];
    H.t[k] = 0;
    H.e[k] = 0.5 * m * dot3(v, v) - A.GM * m * rsqrt(dot3(x, x));
  }
}

// One wavefront per member: INIT forms the forces at t = 0, the initial
// level and the first next time, and adds the pair energies (eq. (hard),
// partners above the member); otherwise only the energy of the final state.
template <bool INIT>
__global__ __launch_bounds__(HUGE_T) void k_huge_eval(HermArgs A, HugeArgs H) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wave = (blockIdx.x * HUGE_T + threadIdx.x) / WAVE, n_waves = gridDim.x * (HUGE_T / WAVE);
  const int M = H.M;
  for (int k = wave; k < M; k += n_waves) {  // uniform per wavefront
    const double xk[3] = {H.x[k], H.x[M + k], H.x[2 * M + k]};
    const double vk[3] = {H.v[k], H.v[M + k], H.v[2 * M + k]};
    const double ik = H.inv[k], mk = H.m[k];
    double pa[3] = {0.0, 0.0, 0.0}, pj[3] = {0.0, 0.0, 0.0}, e = 0.0;
    for (int q = lane; q < M; q += WAVE) {
      if (q == k) continue;
      const double dx = H.x[q] - xk[0], dy = H.x[M + q] - xk[1], dz = H.x[2 * M + q] - xk[2];
      const double invR = fmin(ik, H.inv[q]);
      if (INIT)
        hard_pair(dx, dy, dz, H.v[q] - vk[0], H.v[M + q] - vk[1], H.v[2 * M + q] - vk[2], H.gm[q], invR, A, pa, pj);
      if (q > k) {
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        e -= mk * H.gm[q] * (1.0 - changeover_W(r * invR, A)) / r;
      }
    }
    e = wave_sum(e);
    if (INIT) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        pa[d] = wave_sum(pa[d]);
        pj[d] = wave_sum(pj[d]);
      }
    }
    if (lane == 0) {
      if (INIT) {
        double a0[3], j0[3];
        star_term(xk, vk, A.GM, a0, j0);
        for (int d = 0; d < 3; ++d) {
          a0[d] += pa[d];
          j0[d] += pj[d];
          H.a[d * M + k] = a0[d];
          H.j[d * M + k] = j0[d];
        }
        const int lev = initial_level(a0, j0, true, H.mem[k], A);
        H.lev[k] = lev;
        atomicMin(&H.tn[0], (unsigned long long)1 << (TICK_BITS - lev));
        H.e[k] += e;
      } else {
        H.e[k] = 0.5 * mk * dot3(vk, vk) - A.GM * mk * rsqrt(dot3(xk, xk)) + e;
      }
    }
  }
}

// E[which] = sum of the energy partials, in a fixed order
__global__ __launch_bounds__(HUGE_T) void k_huge_esum(HugeArgs H, int which) {
  __shared__ double sh[HUGE_T];
  double s = 0.0;
  for (int k = threadIdx.x; k < H.M; k += HUGE_T) s += H.e[k];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = HUGE_T / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) H.E[which] = sh[0];
}

__global__ __launch_bounds__(HUGE_T) void k_huge_predict(HermArgs A, HugeArgs H, int s) {
  if (*H.done) return;
  const unsigned long long T = 1ull << TICK_BITS;
  const unsigned long long tnu = H.tn[s & 1];
  if (tnu > T) {  // every member has reached dt_soft (see seg_body)
    if (blockIdx.x == 0 && threadIdx.x == 0) *H.done = 1;
    return;
  }
  const int64_t tn = (int64_t)tnu;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    H.tn[(s + 1) & 1] = ~0ull;  // filled by this step's k_huge_step
    H.nact[(s + 1) & 1] = 0;
    *H.nst += 1;
  }
  const int M = H.M;
  for (int k = blockIdx.x * HUGE_T + threadIdx.x; k < M; k += gridDim.x * HUGE_T) {
    const int64_t tk = H.t[k];
    const double dl = (double)(tn - tk) * A.tick;
    const double d2 = dl * dl * 0.5, d3 = dl * dl * dl * (1.0 / 6.0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double x = H.x[d * M + k], v = H.v[d * M + k], a = H.a[d * M + k], j = H.j[d * M + k];
      H.xp[d * M + k] = fmad(j, d3, fmad(a, d2, fmad(v, dl, x)));
      H.vp[d * M + k] = fmad(j, d2, fmad(a, dl, v));
    }
    const bool due = tk + ((int64_t)1 << (TICK_BITS - H.lev[k])) == tn;
    H.aflag[k] = due ? 1 : 0;
    if (due) H.act[atomicAdd(&H.nact[s & 1], 1)] = k;
  }
}

__global__ __launch_bounds__(HUGE_T) void k_huge_step(HermArgs A, HugeArgs H, int s) {
  if (*H.done) return;
  const unsigned long long tnu = H.tn[s & 1];
  if (tnu > (1ull << TICK_BITS)) return;
  const int64_t tn = (int64_t)tnu;
  const int M = H.M;
  unsigned long long *next = &H.tn[(s + 1) & 1];
  // members not due keep their state: their next time as it stands
  for (int k = blockIdx.x * HUGE_T + threadIdx.x; k < M; k += gridDim.x * HUGE_T)
    if (!H.aflag[k]) atomicMin(next, (unsigned long long)(H.t[k] + ((int64_t)1 << (TICK_BITS - H.lev[k]))));
  const int lane = threadIdx.x & (WAVE - 1);
  const int wave = (blockIdx.x * HUGE_T + threadIdx.x) / WAVE, n_waves = gridDim.x * (HUGE_T / WAVE);
  const int na = H.nact[s & 1];
  for (int q0 = wave; q0 < na; q0 += n_waves) {  // uniform per wavefront
    const int k = H.act[q0];
    const double xp[3] = {H.xp[k], H.xp[M + k], H.xp[2 * M + k]};
    const double vp[3] = {H.vp[k], H.vp[M + k], H.vp[2 * M + k]};
    const double ik = H.inv[k];
    double pa[3] = {0.0, 0.0, 0.0}, pj[3] = {0.0, 0.0, 0.0};
    for (int q = lane; q < M; q += WAVE) {
      if (q == k) continue;
      hard_pair(H.xp[q] - xp[0], H.xp[M + q] - xp[1], H.xp[2 * M + q] - xp[2], H.vp[q] - vp[0],
                H.vp[M + q] - vp[1], H.vp[2 * M + q] - vp[2], H.gm[q], fmin(ik, H.inv[q]), A, pa, pj);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      pa[d] = wave_sum(pa[d]);
      pj[d] = wave_sum(pj[d]);
    }
    if (lane == 0) {
      double a1[3], j1[3], x[3], v[3], a0[3], j0[3];
      star_term(xp, vp, A.GM, a1, j1);
      for (int d = 0; d < 3; ++d) {
        a1[d] += pa[d];
        j1[d] += pj[d];
        x[d] = H.x[d * M + k];
        v[d] = H.v[d * M + k];
        a0[d] = H.a[d * M + k];
        j0[d] = H.j[d * M + k];
      }
      const double h = (double)(tn - H.t[k]) * A.tick;
      int lev = H.lev[k];
      correct(x, v, a0, j0, xp, vp, a1, j1, h, tn, lev, A);
      for (int d = 0; d < 3; ++d) {
        H.x[d * M + k] = x[d];
        H.v[d * M + k] = v[d];
        H.a[d * M + k] = a0[d];
        H.j[d * M + k] = j0[d];
      }
      H.t[k] = tn;
      H.lev[k] = lev;
      atomicMin(next, (unsigned long long)(tn + ((int64_t)1 << (TICK_BITS - lev))));
    }
  }
  // work counters: the step's due members, each over M - 1 partners
  if (blockIdx.x == 0 && threadIdx.x == 0 && na > 0) {
    atomicAdd(&A.cnt->n_heval, (unsigned long long)na);
    atomicAdd(&A.cnt->n_hpair, (unsigned long long)na * (unsigned long long)(M - 1));
  }
}

__global__ __launch_bounds__(HUGE_T) void k_huge_store(HermArgs A, HugeArgs H) {
  const int64_t n = A.n;
  const int M = H.M;
  const int nst = *H.nst;
  for (int k = blockIdx.x * HUGE_T + threadIdx.x; k < M; k += gridDim.x * HUGE_T) {
    const int64_t g = H.mem[k];
    double x[3];
    for (int d = 0; d < 3; ++d) {
      x[d] = H.x[d * M + k];
      A.pos[d * n + g] = x[d];
      A.vel[d * n + g] = H.v[d * M + k];
    }
    if (A.dt_hard) A.dt_hard[g] = ldexp(A.dt_soft, -H.lev[k]);
    if (A.msteps) A.msteps[g] = nst;
    if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))) set_flag(A.cnt, P3T_FLAG_NAN);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (A.e_rel) A.e_rel[H.c] = fabs(H.E[1] - H.E[0]) / fabs(H.E[0]);
    if (A.nsteps) A.nsteps[H.c] = nst;
  }
}

namespace {

// device memory of the percolated-cluster path, sized for M members
hipError_t huge_buffers(p3t_ctx *c, int64_t M, HugeArgs &H) {
  auto bytes = [](int64_t count, size_t sz) { return ((size_t)count * sz + 255) & ~size_t(255); };
  const size_t need = 6 * bytes(3 * M, sizeof(double)) + 4 * bytes(M, sizeof(double)) + bytes(M, sizeof(int64_t)) +
                      3 * bytes(M, sizeof(int32_t)) + 4 * 256;
  hipError_t e;
  if (!c->huge_buf || c->huge_bytes < need) {
    if (c->huge_buf && (e = hipFree(c->huge_buf)) != hipSuccess) return e;
    c->huge_buf = nullptr;
    c->huge_bytes = 0;
    if ((e = hipMalloc((void **)&c->huge_buf, need)) != hipSuccess) return e;
    c->huge_bytes = need;
  }
  Arena A;
  A.base = c->huge_buf;
  A.size = c->huge_bytes;
  double **d3[6] = {&H.x, &H.v, &H.a, &H.j, &H.xp, &H.vp};
  for (auto p : d3) *p = A.take<double>(3 * M);
  H.m = A.take<double>(M);
  H.gm = A.take<double>(M);
  H.inv = A.take<double>(M);
  H.e = A.take<double>(M);
  H.t = A.take<int64_t>(M);
  H.lev = A.take<int32_t>(M);
  H.act = A.take<int32_t>(M);
  H.aflag = A.take<int32_t>(M);
  H.tn = A.take<unsigned long long>(2);
  H.nact = A.take<int32_t>(2);
  H.nst = A.take<int32_t>(2);
  H.done = H.nst + 1;
  H.E = A.take<double>(2);
  return H.E ? hipSuccess : hipErrorOutOfMemory;
}

constexpr int HUGE_BATCH = 32;  // block steps issued between two reads of the done word

// Every cluster of bucket 10 (above 1024 members), one after the other on
// stream s; blocks the host until they are integrated.
hipError_t huge_clusters(p3t_ctx *c, const HermArgs &A, int count, hipStream_t s) {
  hipError_t e;
  std::vector<int32_t> ids(count);
  if ((e = hipMemcpyAsync(ids.data(), A.blists + (int64_t)10 * A.nc, sizeof(int32_t) * count, hipMemcpyDeviceToHost,
                          s)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  std::vector<int32_t> lo(count), hi(count);
  int64_t m_max = 0;
  for (int q = 0; q < count; ++q) {
    int32_t b[2];
    if ((e = hipMemcpy(b, A.cl_ptr + ids[q], sizeof(b), hipMemcpyDeviceToHost)) != hipSuccess) return e;
    lo[q] = b[0];
    hi[q] = b[1];
    m_max = std::max<int64_t>(m_max, b[1] - b[0]);
  }
  HugeArgs H;
  if ((e = huge_buffers(c, m_max, H)) != hipSuccess) return e;
  for (int q = 0; q < count; ++q) {
    H.c = ids[q];
    H.M = hi[q] - lo[q];
    H.mem = A.members + lo[q];
    const unsigned g1 = (unsigned)std::min<int64_t>(4096, (H.M + HUGE_T - 1) / HUGE_T);
    const unsigned gw = (unsigned)std::min<int64_t>((int64_t)c->n_cu * 8, (H.M + 3) / 4);  // a wavefront per member
    hipLaunchKernelGGL(k_huge_load, dim3(g1), dim3(HUGE_T), 0, s, A, H);
    hipLaunchKernelGGL(k_huge_eval<true>, dim3(gw), dim3(HUGE_T), 0, s, A, H);
    hipLaunchKernelGGL(k_huge_esum, dim3(1), dim3(HUGE_T), 0, s, H, 0);
    for (int step = 0;;) {
      for (int b = 0; b < HUGE_BATCH; ++b, ++step) {
        hipLaunchKernelGGL(k_huge_predict, dim3(g1), dim3(HUGE_T), 0, s, A, H, step);
        hipLaunchKernelGGL(k_huge_step, dim3(gw), dim3(HUGE_T), 0, s, A, H, step);
      }
      int32_t st[2];
      if ((e = hipMemcpyAsync(st, H.nst, sizeof(st), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
      if (st[1]) break;  // done
      if (st[0] >= A.max_iter) {  // block-step limit, as in the other paths
        hipLaunchKernelGGL(k_huge_flag, dim3(1), dim3(1), 0, s, A.cnt, (unsigned)P3T_FLAG_NSTEPS);
        break;
      }
    }
    hipLaunchKernelGGL(k_huge_eval<false>, dim3(gw), dim3(HUGE_T), 0, s, A, H);
    hipLaunchKernelGGL(k_huge_esum, dim3(1), dim3(HUGE_T), 0, s, H, 1);
    hipLaunchKernelGGL(k_huge_store, dim3(g1), dim3(HUGE_T), 0, s, A, H);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // the scratch is reused by the next cluster and call: finish before returning
  return hipStreamSynchronize(s);
}

}  // namespace

}  // namespace p3t
