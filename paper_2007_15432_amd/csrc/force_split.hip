// force_split.hip -- the soft force as one lean kernel per interaction class
// (eq. (softforce) with the pair cut-off of eq. (rout2); neighbour pairs of
// Section 2.3), an alternative to the fused kernel of force.hip.
//
//   k_near   FP64 with the changeover K (mixed form: the pairs beyond both
//            cut-offs, where K = 1, in FP32 from FP64 offsets, the few
//            inside the changeover in FP64); while it runs, each lane
//            records in a bit mask which j of the current tile are
//            neighbour candidates
//            (r^2 <= max reach^2, with a relative margin that covers the
//            rounding of r^2) and appends them after the tile to a candidate
//            buffer.  Writes the sorted-order accumulator (=).
//   k_cand_test  the exact neighbour test of Section 2.3 on every candidate,
//            one thread each; neighbours go to the pair buffer.  Coincident
//            pairs (r = 0, i != j) are always candidates and are reported
//            here.
//   k_far    K = 1 particles, FP64 or (mixed) FP32 offsets from the group
//            centre with compensated accumulation.  Adds (+=).
//   k_cell   monopole or traceless-quadrupole cells, FP64 or FP32.  Adds.
//   k_scatter  sorted-order accumulator -> caller's order, NaN check.
//
// Every kernel is one wavefront per group; a lane owns one i-particle, or
// two when the group holds more than 64 (the choice is per group, so small
// groups do not pay for an idle second slot).  j data are staged 64 at a
// time in LDS and read back as broadcasts; the tile is padded to the unroll
// width with massless dummies placed far from the group.
#include "force_common.h"

namespace p3t {

namespace {

struct GroupHdr {
  long long off;
  int n_cell, n_near, n_far, first, count;
  double cx, cy, cz;
};

// Reads the list header of the gi-th group (in work order); every field is
// wave-uniform.  Returns false for a group whose walk overflowed.
__device__ __forceinline__ bool group_header(const ForceArgs &A, int gi, GroupHdr &h) {
  const int q = uniform_first(A.order ? A.order[gi] : gi);
  const GroupList L = A.gl[q];
  h.off = uniform_first64(L.off);
  if (h.off < 0) return false;
  h.n_cell = uniform_first(L.n_cell);
  h.n_near = uniform_first(L.n_near);
  h.n_far = uniform_first(L.n_far);
  const int node = uniform_first(L.node);
  h.first = uniform_first(A.wn[node].first);
  h.count = uniform_first(A.wn[node].count);
  h.cx = 0.5 * (A.wn[node].lo[0] + A.wn[node].hi[0]);
  h.cy = 0.5 * (A.wn[node].lo[1] + A.wn[node].hi[1]);
  h.cz = 0.5 * (A.wn[node].lo[2] + A.wn[node].hi[2]);
  return true;
}

__device__ __forceinline__ int next_gi(const ForceArgs &A, int lane, int iter, int ngroups) {
  if (A.persistent) return next_group(A.queue, lane);
  return iter == 0 ? (int)blockIdx.x : ngroups;
}

constexpr double kDummyOffset = 1.0e3;  // distance of padding entries from the group centre
constexpr double kTinyR2 = 1.0e-150;     // floor of r^2 in the near kernel (see there)
// relative margin on reach^2 for neighbour candidates: it covers the rounding
// of r^2 as computed here, so no pair the exact test keeps is missed
constexpr double kCandMargin = 1.0 + 1.0e-12;

// ------------------------------------------------------------------ near
struct NearTile {
  double4 a[WAVE];  // x, y, z, G m
  double2 b[WAVE];  // 1/r_out, reach^2
  float4 f[WAVE];   // MIXED: r_out^2 and reach^2 widened by kMixMargin, G m
  int j[WAVE];      // sorted index (-2: padding)
};

// MIXED screens each pair on the FP32 square of its offset.  Both tests
// take a margin far above the rounding of that square (a few units in
// 2^-24): every pair inside the changeover (y < 1) is flagged, and every
// pair within a search reach is a candidate.  The flagged pairs are then
// evaluated in FP64 (K = 1 for the few beyond the cut-off), and the exact
// test decides the candidates.  The tests compare the bit patterns of
// non-negative floats as integers, which orders them as the floats.
constexpr double kMixMargin = 1.0e-5;

// The FP64 pair term with the changeover for one near pair (r^2 floored,
// see near_group), added to (ax, ay, az).
__device__ __forceinline__ void near_term64(const ForceArgs &A, double dx, double dy, double dz, double r2, double gm,
                                            double invi, double invj, double &ax, double &ay, double &az) {
  // r = 0 (the particle itself, or a coincident pair, which the candidate
  // test reports) gives y ~ 0 < gamma, so K = 0 and the term vanishes
  // exactly: rinv^3 = 1e225 stays finite.  Adding the floor changes no r^2
  // above 1e-134 (it is below half an ulp there) and costs one add instead
  // of a max with operand canonicalisation.
  const double r2s = r2 + kTinyR2;
  const double rinv = rsqrt_pos(r2s);
  const double y = r2s * rinv * fmin(invi, invj);
  const double x = fmin(fmax((y - A.gamma) * A.inv1mg, 0.0), 1.0);
  const double x2 = x * x;
  const double K = x2 * x2 * (35.0 + x * (-84.0 + x * (70.0 - 20.0 * x)));
  const double f = gm * K * rinv * rinv * rinv;
  ax += f * dx;
  ay += f * dy;
  az += f * dz;
}

// MIXED: a pair beyond both cut-offs (y = r / max(r_out) >= 1, so K = 1)
// takes the Newtonian term in FP32 from its FP64 offset, summed per tile in
// FP32 and folded into the FP64 sums; the pairs inside the changeover
// (y < 1, a fraction of a percent of the near lists) are flagged per lane
// and evaluated in FP64 after the tile.  Without MIXED every pair is FP64.
// Candidate slots reserved by one wavefront and not used yet: [base, end).
// A wavefront reserves A.cand_slab slots at a time with one atomic (a
// returning atomic per tile on the one counter queued behind those of every
// other wavefront); slots it leaves unused are marked (-1, -1), which the
// exact test skips.
struct CandSlab {
  long long base = 0, end = 0;
};

__device__ __forceinline__ void close_slab(const ForceArgs &A, const CandSlab &S, int lane) {
  for (long long q = S.base + lane; q < S.end; q += WAVE)
    if (q < A.cand_cap) A.cands[q] = make_int2(-1, -1);
}

template <bool MIXED, int IPL, int UNR>
__device__ __forceinline__ void near_group(const ForceArgs &A, const GroupHdr &h, NearTile &T, int lane,
                                           CandSlab &S) {
  int ii[IPL];
  double xi[IPL], yi[IPL], zi[IPL], invi[IPL], rch2[IPL], ax[IPL], ay[IPL], az[IPL];
  int ro2q[IPL], rch2q[IPL];  // MIXED: bit patterns of the widened FP32 squares
#pragma unroll
  for (int s = 0; s < IPL; ++s) {
    const int k = lane + WAVE * s;
    ii[s] = k < h.count ? h.first + k : -1;
    const int i = ii[s] >= 0 ? ii[s] : h.first;
    // an empty slot sits far from the group and from the padding entries
    xi[s] = ii[s] >= 0 ? A.sx[i] : h.cx - 2.0 * kDummyOffset;
    yi[s] = A.sy[i];
    zi[s] = A.sz[i];
    invi[s] = A.sinv[i];
    rch2[s] = A.sreach[i] * A.sreach[i] * kCandMargin;
    ax[s] = ay[s] = az[s] = 0.0;
    if constexpr (MIXED) {
      const double ro = A.sro[i], r = A.sreach[i];
      ro2q[s] = __float_as_int((float)(ro * ro * (1.0 + kMixMargin)));
      rch2q[s] = __float_as_int((float)(r * r * (1.0 + kMixMargin)));
    }
  }
  const int32_t *Ln = A.pool + h.off + h.n_cell;
  // the next tile's entry of this lane is loaded into registers while the
  // current tile is evaluated (its gathers are the kernel's memory latency)
  double4 na;
  double2 nb;
  float4 nf;
  int nj = -2;
  auto fetch = [&](int t0) {
    const int nt = min(WAVE, h.n_near - t0);
    const int ntp = min(WAVE, (nt + UNR - 1) / UNR * UNR);
    if (lane < nt) {
      const int j = Ln[t0 + lane];
      const double r = A.sreach[j];
      na = make_double4(A.sx[j], A.sy[j], A.sz[j], A.G * A.sm[j]);
      nb = make_double2(A.sinv[j], r * r * kCandMargin);
      if constexpr (MIXED) {
        const double ro = A.sro[j];
        nf = make_float4((float)(ro * ro * (1.0 + kMixMargin)), (float)(r * r * (1.0 + kMixMargin)), (float)na.w, 0.0f);
      }
      nj = j;
    } else if (lane < ntp) {
      // padding: massless, beyond every reach and every cut-off
      na = make_double4(h.cx + kDummyOffset, h.cy, h.cz, 0.0);
      nb = make_double2(1.0, 0.0);
      nf = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      nj = -2;
    }
  };
  if (h.n_near > 0) fetch(0);
  for (int t0 = 0; t0 < h.n_near; t0 += WAVE) {
    const int nt = min(WAVE, h.n_near - t0);
    const int ntp = min(WAVE, (nt + UNR - 1) / UNR * UNR);
    __syncthreads();
    if (lane < ntp) {
      T.a[lane] = na;
      T.b[lane] = nb;
      if constexpr (MIXED) T.f[lane] = nf;
      T.j[lane] = nj;
    }
    __syncthreads();
    if (t0 + WAVE < h.n_near) fetch(t0 + WAVE);
    unsigned cm[2][IPL], chg_m[2][IPL];
    float tx[IPL], ty[IPL], tz[IPL];
#pragma unroll
    for (int s = 0; s < IPL; ++s) tx[s] = ty[s] = tz[s] = 0.0f;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
#pragma unroll
      for (int s = 0; s < IPL; ++s) cm[half][s] = chg_m[half][s] = 0u;
      const int lo = half * 32, hi = min(ntp, lo + 32);
      for (int jj = lo; jj < hi; jj += UNR) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const double4 a = T.a[jj + u];
          const int jidx = T.j[jj + u];
          const unsigned bit = 1u << ((jj + u) & 31);
          if constexpr (MIXED) {
            const float4 fj = T.f[jj + u];
            const int ro2j = __float_as_int(fj.x), rch2j = __float_as_int(fj.y);
#pragma unroll
            for (int s = 0; s < IPL; ++s) {
              const double dx = a.x - xi[s], dy = a.y - yi[s], dz = a.z - zi[s];
              const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
              const float r2f = fdx * fdx + fdy * fdy + fdz * fdz;
              const int r2q = __float_as_int(r2f);
              // inside the changeover of either side (or r = 0): FP64 below
              const bool chg = (r2q < ro2q[s]) | (r2q < ro2j);
              const float ri = __frsqrt_rn(r2f);
              const float f = chg ? 0.0f : fj.z * ri * ri * ri;
              tx[s] += f * fdx;
              ty[s] += f * fdy;
              tz[s] += f * fdz;
              const bool other = jidx != ii[s];
              chg_m[half][s] |= (chg & other) ? bit : 0u;
              // evaluated without short-circuit, so no branch per pair
              const bool cand = other & ((r2q <= rch2q[s]) | (r2q <= rch2j));
              cm[half][s] |= cand ? bit : 0u;
            }
          } else {
            const double2 b = T.b[jj + u];
            const long long rch2j = __double_as_longlong(b.y);
#pragma unroll
            for (int s = 0; s < IPL; ++s) {
              const double dx = a.x - xi[s], dy = a.y - yi[s], dz = a.z - zi[s];
              const double r2 = dx * dx + dy * dy + dz * dz;
              near_term64(A, dx, dy, dz, r2, a.w, invi[s], b.x, ax[s], ay[s], az[s]);
              // reach^2 of both sides carry the candidate margin already;
              // compared as bit patterns of non-negative doubles (ordered as
              // the doubles), without short-circuit, so no branch per pair
              const long long r2q = __double_as_longlong(r2);
              const bool cand = (jidx != ii[s]) & ((r2q <= __double_as_longlong(rch2[s])) | (r2q <= rch2j));
              cm[half][s] |= cand ? bit : 0u;
            }
          }
        }
      }
    }
    if constexpr (MIXED) {
      // the changeover pairs of this tile in FP64, then the tile's FP32 sums
#pragma unroll
      for (int s = 0; s < IPL; ++s) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          unsigned m = ii[s] >= 0 ? chg_m[half][s] : 0u;
          while (m != 0u) {
            const int q = 32 * half + __ffs(m) - 1;
            m &= m - 1u;
            const double4 a = T.a[q];
            const double dx = a.x - xi[s], dy = a.y - yi[s], dz = a.z - zi[s];
            const double r2 = dx * dx + dy * dy + dz * dz;
            near_term64(A, dx, dy, dz, r2, a.w, invi[s], T.b[q].x, ax[s], ay[s], az[s]);
          }
        }
        ax[s] += (double)tx[s];
        ay[s] += (double)ty[s];
        az[s] += (double)tz[s];
      }
    }
    // hand this tile's candidates (sorted indices) to the exact test
    int nc = 0;
#pragma unroll
    for (int s = 0; s < IPL; ++s) {
      if (ii[s] < 0) cm[0][s] = cm[1][s] = 0u;
      nc += __popc(cm[0][s]) + __popc(cm[1][s]);
    }
    const int incl = wave_incl_scan(nc);
    const int total = uniform_lane(incl, WAVE - 1);
    if (total > 0) {
      if (S.base + total > S.end) {  // uniform
        close_slab(A, S, lane);
        const long long want = total > A.cand_slab ? total : A.cand_slab;
        S.base = (long long)wave_fetch_add(&A.cnt->n_cand, (unsigned long long)want);
        S.end = S.base + want;
        if (S.end > A.cand_cap && lane == 0) set_flag(A.cnt, P3T_FLAG_PAIR_OVERFLOW);
      }
      long long o = S.base + incl - nc;
#pragma unroll
      for (int s = 0; s < IPL; ++s) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          unsigned m = cm[half][s];
          while (m != 0u) {
            const int b = __ffs(m) - 1;
            m &= m - 1u;
            if (o < A.cand_cap) A.cands[o] = make_int2(ii[s], T.j[32 * half + b]);
            ++o;
          }
        }
      }
      S.base += total;
    }
  }
  double *acc = A.acc;
#pragma unroll
  for (int s = 0; s < IPL; ++s) {
    if (ii[s] >= 0) {
      acc[ii[s]] = ax[s];
      acc[A.n + ii[s]] = ay[s];
      acc[2 * A.n + ii[s]] = az[s];
    }
  }
}

template <bool MIXED, int UNR>
__global__ __launch_bounds__(WAVE) void k_near(ForceArgs A) {
  __shared__ NearTile T;
  const int lane = threadIdx.x;
  const int ngroups = uniform_first(min((int)A.cnt->n_groups, A.ngroups_bound));
  CandSlab S;
  unsigned long long n_int = 0;  // this wavefront's interactions, added once at its end
  for (int iter = 0;; ++iter) {
    const int gi = next_gi(A, lane, iter, ngroups);
    if (gi >= ngroups) break;
    GroupHdr h;
    if (!group_header(A, gi, h)) continue;
    if (h.count > WAVE)
      near_group<MIXED, 2, UNR>(A, h, T, lane, S);
    else
      near_group<MIXED, 1, UNR>(A, h, T, lane, S);
    const unsigned long long ni = (unsigned long long)h.count;
    n_int += ni * (unsigned long long)h.n_near - ni;
  }
  close_slab(A, S, lane);
  if (lane == 0 && n_int) atomicAdd(&A.cnt->n_near, n_int);
}

// ------------------------------------------------------------------ far
union FarTile {
  double4 d[WAVE];  // x, y, z, G m
  float4 f[WAVE];   // offsets from the group centre, G m
};

template <bool MIXED, int IPL, int UNR>
__device__ __forceinline__ void far_group(const ForceArgs &A, const GroupHdr &h, FarTile &T, int lane) {
  int ii[IPL];
  double xi[IPL], yi[IPL], zi[IPL], ax[IPL], ay[IPL], az[IPL];
#pragma unroll
  for (int s = 0; s < IPL; ++s) {
    const int k = lane + WAVE * s;
    ii[s] = k < h.count ? h.first + k : -1;
    const int i = ii[s] >= 0 ? ii[s] : h.first;
    xi[s] = A.sx[i];
    yi[s] = A.sy[i];
    zi[s] = A.sz[i];
    ax[s] = ay[s] = az[s] = 0.0;
  }
  const int32_t *Lf = A.pool + h.off + h.n_cell + h.n_near;
  if (!MIXED) {
    for (int t0 = 0; t0 < h.n_far; t0 += WAVE) {
      const int nt = min(WAVE, h.n_far - t0);
      const int ntp = min(WAVE, (nt + UNR - 1) / UNR * UNR);
      __syncthreads();
      if (lane < nt) {
        const int j = Lf[t0 + lane];
        T.d[lane] = make_double4(A.sx[j], A.sy[j], A.sz[j], A.G * A.sm[j]);
      } else if (lane < ntp) {
        T.d[lane] = make_double4(h.cx + kDummyOffset, h.cy, h.cz, 0.0);
      }
      __syncthreads();
      for (int jj = 0; jj < ntp; jj += UNR) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const double4 a = T.d[jj + u];
#pragma unroll
          for (int s = 0; s < IPL; ++s) {
            const double dx = a.x - xi[s], dy = a.y - yi[s], dz = a.z - zi[s];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double rinv = rsqrt_pos(r2);  // r > 0: beyond the group's reach
            const double f = a.w * rinv * rinv * rinv;
            ax[s] += f * dx;
            ay[s] += f * dy;
            az[s] += f * dz;
          }
        }
      }
    }
  } else {
    float fxi[IPL], fyi[IPL], fzi[IPL], hx[IPL], hy[IPL], hz[IPL], lx[IPL], ly[IPL], lz[IPL];
#pragma unroll
    for (int s = 0; s < IPL; ++s) {
      fxi[s] = (float)(xi[s] - h.cx);
      fyi[s] = (float)(yi[s] - h.cy);
      fzi[s] = (float)(zi[s] - h.cz);
      hx[s] = hy[s] = hz[s] = lx[s] = ly[s] = lz[s] = 0.0f;
    }
    for (int t0 = 0; t0 < h.n_far; t0 += WAVE) {
      const int nt = min(WAVE, h.n_far - t0);
      const int ntp = min(WAVE, (nt + UNR - 1) / UNR * UNR);
      __syncthreads();
      if (lane < nt) {
        const int j = Lf[t0 + lane];
        T.f[lane] = make_float4((float)(A.sx[j] - h.cx), (float)(A.sy[j] - h.cy), (float)(A.sz[j] - h.cz),
                                (float)(A.G * A.sm[j]));
      } else if (lane < ntp) {
        T.f[lane] = make_float4((float)kDummyOffset, 0.0f, 0.0f, 0.0f);
      }
      __syncthreads();
      float tx[IPL], ty[IPL], tz[IPL];
#pragma unroll
      for (int s = 0; s < IPL; ++s) tx[s] = ty[s] = tz[s] = 0.0f;
      for (int jj = 0; jj < ntp; jj += UNR) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const float4 a = T.f[jj + u];
#pragma unroll
          for (int s = 0; s < IPL; ++s) {
            const float dx = a.x - fxi[s], dy = a.y - fyi[s], dz = a.z - fzi[s];
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float rinv = __frsqrt_rn(r2);
            const float f = a.w * rinv * rinv * rinv;
            tx[s] += f * dx;
            ty[s] += f * dy;
            tz[s] += f * dz;
          }
        }
      }
#pragma unroll
      for (int s = 0; s < IPL; ++s) {
        two_sum_acc(hx[s], lx[s], tx[s]);
        two_sum_acc(hy[s], ly[s], ty[s]);
        two_sum_acc(hz[s], lz[s], tz[s]);
      }
    }
#pragma unroll
    for (int s = 0; s < IPL; ++s) {
      ax[s] = (double)hx[s] + (double)lx[s];
      ay[s] = (double)hy[s] + (double)ly[s];
      az[s] = (double)hz[s] + (double)lz[s];
    }
  }
  double *acc = A.acc;
#pragma unroll
  for (int s = 0; s < IPL; ++s) {
    if (ii[s] >= 0) {
      acc[ii[s]] += ax[s];
      acc[A.n + ii[s]] += ay[s];
      acc[2 * A.n + ii[s]] += az[s];
    }
  }
}

template <bool MIXED, int UNR>
__global__ __launch_bounds__(WAVE) void k_far(ForceArgs A) {
  __shared__ FarTile T;
  const int lane = threadIdx.x;
  const int ngroups = uniform_first(min((int)A.cnt->n_groups, A.ngroups_bound));
  unsigned long long n_int = 0;  // this wavefront's interactions, added once at its end
  for (int iter = 0;; ++iter) {
    const int gi = next_gi(A, lane, iter, ngroups);
    if (gi >= ngroups) break;
    GroupHdr h;
    if (!group_header(A, gi, h)) continue;
    if (h.n_far == 0) continue;
    if (h.count > WAVE)
      far_group<MIXED, 2, UNR>(A, h, T, lane);
    else
      far_group<MIXED, 1, UNR>(A, h, T, lane);
    n_int += (unsigned long long)h.count * (unsigned long long)h.n_far;
  }
  if (lane == 0 && n_int) atomicAdd(&A.cnt->n_far, n_int);
}

// ------------------------------------------------------------------ cells
union CellTile {
  struct {
    double4 a[WAVE];  // centre of mass, G M
    double4 qa[WAVE];  // G q_xx, q_yy, q_zz, q_xy
    double2 qb[WAVE];  // G q_xz, q_yz
  } d;
  struct {
    float4 a[WAVE];
    float4 qa[WAVE];
    float2 qb[WAVE];
  } f;
};

template <typename R>
__device__ __forceinline__ R fma_r(R a, R b, R c) {
  return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fma_r<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// The cell term added to (ax, ay, az):
//   a = G [ M d / r^3 - Q d / r^5 + (5/2) (d.Q d) d / r^7 ],  d = X_c - x_i,
// as d (G M / r^3 + (5/2) (d.Q d) / r^7) - Q d / r^5, so that each
// component is two fused multiply-adds onto the running sum.
template <typename R>
__device__ __forceinline__ void cell_acc(R dx, R dy, R dz, R gm, R q0, R q1, R q2, R q3, R q4, R q5, bool quad,
                                         R rinv, R &ax, R &ay, R &az) {
  const R rinv2 = rinv * rinv;
  const R rinv3 = rinv * rinv2;
  if (!quad) {
    const R f = gm * rinv3;
    ax = fma_r(f, dx, ax);
    ay = fma_r(f, dy, ay);
    az = fma_r(f, dz, az);
    return;
  }
  const R qx = fma_r(q4, dz, fma_r(q3, dy, q0 * dx));
  const R qy = fma_r(q5, dz, fma_r(q1, dy, q3 * dx));
  const R qz = fma_r(q2, dz, fma_r(q5, dy, q4 * dx));
  const R dqd = fma_r(dz, qz, fma_r(dy, qy, dx * qx));
  const R rinv5 = rinv3 * rinv2;
  const R f = fma_r(gm, rinv3, R(2.5) * dqd * (rinv5 * rinv2));
  ax = fma_r(-qx, rinv5, fma_r(f, dx, ax));
  ay = fma_r(-qy, rinv5, fma_r(f, dy, ay));
  az = fma_r(-qz, rinv5, fma_r(f, dz, az));
}

template <bool MIXED, bool QUAD, int IPL, int UNR>
__device__ __forceinline__ void cell_group(const ForceArgs &A, const GroupHdr &h, CellTile &T, int lane) {
  int ii[IPL];
  double xi[IPL], yi[IPL], zi[IPL], ax[IPL], ay[IPL], az[IPL];
#pragma unroll
  for (int s = 0; s < IPL; ++s) {
    const int k = lane + WAVE * s;
    ii[s] = k < h.count ? h.first + k : -1;
    const int i = ii[s] >= 0 ? ii[s] : h.first;
    xi[s] = A.sx[i];
    yi[s] = A.sy[i];
    zi[s] = A.sz[i];
    ax[s] = ay[s] = az[s] = 0.0;
  }
  const int32_t *Lc = A.pool + h.off;
  const double G = A.G;
  if (!MIXED) {
    for (int t0 = 0; t0 < h.n_cell; t0 += WAVE) {
      const int nt = min(WAVE, h.n_cell - t0);
      const int ntp = min(WAVE, (nt + UNR - 1) / UNR * UNR);
      __syncthreads();
      if (lane < nt) {
        const CellMom c = A.cm[Lc[t0 + lane]];
        T.d.a[lane] = make_double4(c.com[0], c.com[1], c.com[2], G * c.mass);
        if (QUAD) {
          T.d.qa[lane] = make_double4(G * c.q[0], G * c.q[1], G * c.q[2], G * c.q[3]);
          T.d.qb[lane] = make_double2(G * c.q[4], G * c.q[5]);
        }
      } else if (lane < ntp) {
        T.d.a[lane] = make_double4(h.cx + kDummyOffset, h.cy, h.cz, 0.0);
        if (QUAD) {
          T.d.qa[lane] = make_double4(0.0, 0.0, 0.0, 0.0);
          T.d.qb[lane] = make_double2(0.0, 0.0);
        }
      }
      __syncthreads();
      for (int jj = 0; jj < ntp; jj += UNR) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const double4 a = T.d.a[jj + u];
          double4 qa = make_double4(0.0, 0.0, 0.0, 0.0);
          double2 qb = make_double2(0.0, 0.0);
          if (QUAD) {
            qa = T.d.qa[jj + u];
            qb = T.d.qb[jj + u];
          }
#pragma unroll
          for (int s = 0; s < IPL; ++s) {
            const double dx = a.x - xi[s], dy = a.y - yi[s], dz = a.z - zi[s];
            const double r2 = dx * dx + dy * dy + dz * dz;
            cell_acc<double>(dx, dy, dz, a.w, qa.x, qa.y, qa.z, qa.w, qb.x, qb.y, QUAD, rsqrt_pos(r2), ax[s], ay[s],
                             az[s]);
          }
        }
      }
    }
  } else {
    float fxi[IPL], fyi[IPL], fzi[IPL], hx[IPL], hy[IPL], hz[IPL], lx[IPL], ly[IPL], lz[IPL];
#pragma unroll
    for (int s = 0; s < IPL; ++s) {
      fxi[s] = (float)(xi[s] - h.cx);
      fyi[s] = (float)(yi[s] - h.cy);
      fzi[s] = (float)(zi[s] - h.cz);
      hx[s] = hy[s] = hz[s] = lx[s] = ly[s] = lz[s] = 0.0f;
    }
    for (int t0 = 0; t0 < h.n_cell; t0 += WAVE) {
      const int nt = min(WAVE, h.n_cell - t0);
      const int ntp = min(WAVE, (nt + UNR - 1) / UNR * UNR);
      __syncthreads();
      if (lane < nt) {
        const CellMom c = A.cm[Lc[t0 + lane]];
        T.f.a[lane] = make_float4((float)(c.com[0] - h.cx), (float)(c.com[1] - h.cy), (float)(c.com[2] - h.cz),
                                  (float)(G * c.mass));
        if (QUAD) {
          T.f.qa[lane] = make_float4((float)(G * c.q[0]), (float)(G * c.q[1]), (float)(G * c.q[2]),
                                     (float)(G * c.q[3]));
          T.f.qb[lane] = make_float2((float)(G * c.q[4]), (float)(G * c.q[5]));
        }
      } else if (lane < ntp) {
        T.f.a[lane] = make_float4((float)kDummyOffset, 0.0f, 0.0f, 0.0f);
        if (QUAD) {
          T.f.qa[lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
          T.f.qb[lane] = make_float2(0.0f, 0.0f);
        }
      }
      __syncthreads();
      float tx[IPL], ty[IPL], tz[IPL];
#pragma unroll
      for (int s = 0; s < IPL; ++s) tx[s] = ty[s] = tz[s] = 0.0f;
      for (int jj = 0; jj < ntp; jj += UNR) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const float4 a = T.f.a[jj + u];
          float4 qa = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
          float2 qb = make_float2(0.0f, 0.0f);
          if (QUAD) {
            qa = T.f.qa[jj + u];
            qb = T.f.qb[jj + u];
          }
#pragma unroll
          for (int s = 0; s < IPL; ++s) {
            const float dx = a.x - fxi[s], dy = a.y - fyi[s], dz = a.z - fzi[s];
            const float r2 = dx * dx + dy * dy + dz * dz;
            cell_acc<float>(dx, dy, dz, a.w, qa.x, qa.y, qa.z, qa.w, qb.x, qb.y, QUAD, __frsqrt_rn(r2), tx[s], ty[s],
                            tz[s]);
          }
        }
      }
#pragma unroll
      for (int s = 0; s < IPL; ++s) {
        two_sum_acc(hx[s], lx[s], tx[s]);
        two_sum_acc(hy[s], ly[s], ty[s]);
        two_sum_acc(hz[s], lz[s], tz[s]);
      }
    }
#pragma unroll
    for (int s = 0; s < IPL; ++s) {
      ax[s] = (double)hx[s] + (double)lx[s];
      ay[s] = (double)hy[s] + (double)ly[s];
      az[s] = (double)hz[s] + (double)lz[s];
    }
  }
  double *acc = A.acc;
#pragma unroll
  for (int s = 0; s < IPL; ++s) {
    if (ii[s] >= 0) {
      acc[ii[s]] += ax[s];
      acc[A.n + ii[s]] += ay[s];
      acc[2 * A.n + ii[s]] += az[s];
    }
  }
}

template <bool MIXED, bool QUAD, int UNR>
__global__ __launch_bounds__(WAVE) void k_cell(ForceArgs A) {
  __shared__ CellTile T;
  const int lane = threadIdx.x;
  const int ngroups = uniform_first(min((int)A.cnt->n_groups, A.ngroups_bound));
  unsigned long long n_int = 0;  // this wavefront's interactions, added once at its end
  for (int iter = 0;; ++iter) {
    const int gi = next_gi(A, lane, iter, ngroups);
    if (gi >= ngroups) break;
    GroupHdr h;
    if (!group_header(A, gi, h)) continue;
    if (h.n_cell == 0) continue;
    if (h.count > WAVE)
      cell_group<MIXED, QUAD, 2, UNR>(A, h, T, lane);
    else
      cell_group<MIXED, QUAD, 1, UNR>(A, h, T, lane);
    n_int += (unsigned long long)h.count * (unsigned long long)h.n_cell;
  }
  if (lane == 0 && n_int) atomicAdd(&A.cnt->n_cell, n_int);
}

// exact neighbour test of every candidate (sorted indices) -> pairs in the
// caller's indices
__global__ void k_cand_test(ForceArgs A) {
  const long long nc = (long long)A.cnt->n_cand;
  const long long m = nc < A.cand_cap ? nc : A.cand_cap;
  const int lane = lane_id();
  const long long stride = (long long)gridDim.x * blockDim.x;
  // the loop runs wave by wave, so the ballot below sees every lane
  for (long long p0 = blockIdx.x * (long long)blockDim.x + (threadIdx.x - lane); p0 < m; p0 += stride) {
    const long long p = p0 + lane;
    bool nb = false;
    int i = 0, j = 0;
    const int2 c = p < m ? A.cands[p] : make_int2(-1, -1);
    if (c.x >= 0) {  // (-1, -1): a slot its wavefront left unused
      i = c.x;
      j = c.y;
      // a slow member sits at its pre-drift position here; its pairs are
      // tested once its integration has finished
      const bool skip = A.slow && (A.slow[A.sid[i]] | A.slow[A.sid[j]]);
      if (!skip && A.sx[i] == A.sx[j] && A.sy[i] == A.sy[j] && A.sz[i] == A.sz[j]) set_flag(A.cnt, P3T_FLAG_COINCIDENT);
      nb = !skip && neighbour_test(A.sx[i], A.sy[i], A.sz[i], A.svx[i], A.svy[i], A.svz[i], A.sm[i], A.sro[i], A.srs[i],
                          A.sx[j], A.sy[j], A.sz[j], A.svx[j], A.svy[j], A.svz[j], A.sm[j], A.sro[j], A.srs[j], A.G,
                          A.rsch2, A.rsch3, A.dt);
    }
    const unsigned long long bal = __ballot(nb);
    if (bal == 0ull) continue;
    const int leader = __ffsll((long long)bal) - 1;
    const unsigned long long o0 = wave_fetch_add(&A.cnt->n_pairs, (unsigned long long)__popcll(bal), leader);
    if (nb) {
      mark_close_pair(A, i, j);
      const unsigned long long q = o0 + popc_below(bal);
      if ((int64_t)q < A.pair_cap)
        A.pairs[q] = make_int2(A.sid[i], A.sid[j]);
      else
        set_flag(A.cnt, P3T_FLAG_PAIR_OVERFLOW);
    }
  }
}

// sorted-order accumulator -> caller's order
__global__ void k_scatter(const double *__restrict__ acc_s, const int32_t *__restrict__ sid, int64_t n,
                          double *__restrict__ acc, DevCounters *cnt) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double x = acc_s[i], y = acc_s[n + i], z = acc_s[2 * n + i];
    const int64_t o = sid[i];
    acc[o] = x;
    acc[n + o] = y;
    acc[2 * n + o] = z;
    bad |= !(isfinite(x) && isfinite(y) && isfinite(z));
  }
  if (__ballot(bad) != 0ull && lane_id() == 0) set_flag(cnt, P3T_FLAG_NAN);
}

template <typename K>
unsigned persistent_grid(K kernel, int n_cu, int waves_cap) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, WAVE, 0) != hipSuccess || nb <= 0) nb = 8;
  return (unsigned)(n_cu * std::min(nb, waves_cap));
}

template <int UNR>
hipError_t launch_split(p3t_ctx *c, ForceArgs A, unsigned nonpersistent_grid, double *acc3) {
  const bool mixed = c->P.precision == 1, quad = c->P.multipole == 2;
  const hipStream_t s = c->stream;
  const int cap = c->fcfg.waves_per_cu;
  A.acc = c->acc_s;
  auto grid = [&](auto kernel) {
    return A.persistent ? persistent_grid(kernel, c->n_cu, cap) : nonpersistent_grid;
  };
  A.queue = &c->cnt->queue[0];
  if (mixed)
    hipLaunchKernelGGL((k_near<true, UNR>), dim3(grid(k_near<true, UNR>)), dim3(WAVE), 0, s, A);
  else
    hipLaunchKernelGGL((k_near<false, UNR>), dim3(grid(k_near<false, UNR>)), dim3(WAVE), 0, s, A);
  ev_record(c, 11);
  A.queue = &c->cnt->queue[1];
  if (mixed)
    hipLaunchKernelGGL((k_far<true, UNR>), dim3(grid(k_far<true, UNR>)), dim3(WAVE), 0, s, A);
  else
    hipLaunchKernelGGL((k_far<false, UNR>), dim3(grid(k_far<false, UNR>)), dim3(WAVE), 0, s, A);
  ev_record(c, 12);
  A.queue = &c->cnt->queue[2];
  if (mixed && quad)
    hipLaunchKernelGGL((k_cell<true, true, UNR>), dim3(grid(k_cell<true, true, UNR>)), dim3(WAVE), 0, s, A);
  else if (mixed)
    hipLaunchKernelGGL((k_cell<true, false, UNR>), dim3(grid(k_cell<true, false, UNR>)), dim3(WAVE), 0, s, A);
  else if (quad)
    hipLaunchKernelGGL((k_cell<false, true, UNR>), dim3(grid(k_cell<false, true, UNR>)), dim3(WAVE), 0, s, A);
  else
    hipLaunchKernelGGL((k_cell<false, false, UNR>), dim3(grid(k_cell<false, false, UNR>)), dim3(WAVE), 0, s, A);
  ev_record(c, 13);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)c->n_cu * 8, (c->n + 255) / 256));
  const unsigned gc = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)c->n_cu * 8, (c->cand_cap + 255) / 256));
  if (A.cand_cap > 0) hipLaunchKernelGGL(k_cand_test, dim3(gc), dim3(256), 0, s, A);
  ev_record(c, 14);
  hipLaunchKernelGGL(k_scatter, dim3(g), dim3(256), 0, s, (const double *)c->acc_s, (const int32_t *)c->sid, c->n,
                     acc3, c->cnt);
  return hipGetLastError();
}

}  // namespace

hipError_t soft_force_split(p3t_ctx *c, const ForceArgs &A, unsigned nonpersistent_grid, double *acc3) {
  switch (c->fcfg.unroll) {
    case 1:
      return launch_split<1>(c, A, nonpersistent_grid, acc3);
    case 2:
      return launch_split<2>(c, A, nonpersistent_grid, acc3);
    case 8:
      return launch_split<8>(c, A, nonpersistent_grid, acc3);
    default:
      return launch_split<4>(c, A, nonpersistent_grid, acc3);
  }
}

}  // namespace p3t
