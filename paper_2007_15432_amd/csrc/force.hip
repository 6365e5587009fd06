// force.hip -- soft acceleration over the interaction lists (eq. (softforce)
// with the pair cut-off of eq. (rout2)) and collection of neighbour pairs
// (Section 2.3).
//
// One wavefront per group; a lane owns IPL i-particles (group size <=
// 64 * IPL), so every j value read from LDS is used IPL times.  j-particles
// and cells are staged 64 at a time in LDS by the whole wave (coalesced
// gathers from the Morton-ordered arrays) and read back as broadcasts.
//
//   NEAR particles (inside some search reach): FP64 (mixed form: only the
//     pairs inside the changeover; those beyond both cut-offs, K = 1, in
//     FP32 from FP64 offsets), K(y) with
//     y = r / max(r_out,i, r_out,j) = r * min(1/r_out,i, 1/r_out,j),
//     K = x^4 (35 - 84x + 70x^2 - 20x^3), x = clamp((y - gamma)/(1 - gamma)),
//     which is W - y W' for the W of eq. (cutfuncW) in closed form; then a
//     separate pass over the same tile tests neighbour candidates with the
//     exact division-free FP64 predicate.
//   FAR particles and CELLS (K = 1): FP64, or in the mixed form FP32 on
//     offsets from the group centre (offsets formed in FP64) with per-tile
//     FP32 partial sums folded into a compensated (hi, lo) FP32 accumulator.
//   Cells are monopoles or traceless quadrupoles about their centre of mass.
#include "force_common.h"

namespace p3t {

// The fused kernel calls the exact test out of line (it is rare).
__device__ __noinline__ bool pair_is_neighbour(double xi, double yi, double zi, double vxi, double vyi, double vzi,
                                               double mi, double roi, double rsi, double xj, double yj, double zj,
                                               double vxj, double vyj, double vzj, double mj, double roj, double rsj,
                                               double G, double rsch2, double rsch3, double dt) {
  return neighbour_test(xi, yi, zi, vxi, vyi, vzi, mi, roi, rsi, xj, yj, zj, vxj, vyj, vzj, mj, roj, rsj, G, rsch2,
                        rsch3, dt);
}

template <bool MIXED, bool QUAD, int IPL>
__global__ __launch_bounds__(WAVE) void k_force(ForceArgs A) {
  __shared__ double4 tA[WAVE];  // x, y, z, G m (near/far/cells FP64)
  __shared__ double4 tB[WAVE];  // near: 1/r_out, reach | cells: G q0..q3
  __shared__ double2 tC[WAVE];  // cells: G q4, q5
  __shared__ int tI[WAVE];      // near: sorted index
  __shared__ float4 fA[WAVE];   // mixed: offset x, y, z, G m
  __shared__ float4 fB[WAVE];   // mixed cells: G q0..q3
  __shared__ float2 fC[WAVE];   // mixed cells: G q4, q5
  const int lane = threadIdx.x;
  const int ngroups = uniform_first(min((int)A.cnt->n_groups, A.ngroups_bound));
  int iter = 0;
  for (;;) {
    int gi;
    if (A.persistent) {
      // all lanes execute the atomic (only lane 0 adds); see uniform_first
      gi = next_group(A.queue, lane);
    } else {
      gi = iter == 0 ? (int)blockIdx.x : ngroups;
    }
    ++iter;
    if (gi >= ngroups) break;
    const int q = uniform_first(A.order ? A.order[gi] : gi);
    GroupList L = A.gl[q];
    L.off = uniform_first64(L.off);
    L.n_cell = uniform_first(L.n_cell);
    L.n_near = uniform_first(L.n_near);
    L.n_far = uniform_first(L.n_far);
    L.node = uniform_first(L.node);
    if (L.off < 0) continue;  // walk overflowed; the host retries with more room
    const int gfirst = uniform_first(A.wn[L.node].first);
    const int gcount = uniform_first(A.wn[L.node].count);
    const double gcx = 0.5 * (A.wn[L.node].lo[0] + A.wn[L.node].hi[0]);
    const double gcy = 0.5 * (A.wn[L.node].lo[1] + A.wn[L.node].hi[1]);
    const double gcz = 0.5 * (A.wn[L.node].lo[2] + A.wn[L.node].hi[2]);

    int ii[IPL];
    double xi[IPL], yi[IPL], zi[IPL], invi[IPL], reachi[IPL];
    double ax[IPL], ay[IPL], az[IPL];
#pragma unroll
    for (int s = 0; s < IPL; ++s) {
      const int k = lane + WAVE * s;
      ii[s] = k < gcount ? gfirst + k : -1;
      const int i = ii[s] >= 0 ? ii[s] : gfirst;
      xi[s] = A.sx[i];
      yi[s] = A.sy[i];
      zi[s] = A.sz[i];
      invi[s] = A.sinv[i];
      reachi[s] = A.sreach[i];
      ax[s] = ay[s] = az[s] = 0.0;
    }
    bool coincident = false;

    // ---------------- near particles: FP64 with the changeover
    const int32_t *Ln = A.pool + L.off + L.n_cell;
    for (int t0 = 0; t0 < L.n_near; t0 += WAVE) {
      const int nt = min(WAVE, L.n_near - t0);
      __syncthreads();
      if (lane < nt) {
        const int j = Ln[t0 + lane];
        tA[lane] = make_double4(A.sx[j], A.sy[j], A.sz[j], A.G * A.sm[j]);
        tB[lane] = make_double4(A.sinv[j], A.sreach[j], 0.0, 0.0);
        tI[lane] = j;
      }
      __syncthreads();
      // mixed form: the pairs beyond both cut-offs (K = 1) in FP32 from
      // their FP64 offsets, summed per tile in FP32 and folded into the FP64
      // sums; inside the changeover FP64 (as the split near kernel does)
      float tx[IPL], ty[IPL], tz[IPL];
#pragma unroll
      for (int s = 0; s < IPL; ++s) tx[s] = ty[s] = tz[s] = 0.0f;
      for (int jj = 0; jj < nt; ++jj) {
        const double4 a = tA[jj];
        const double4 b = tB[jj];
        const int jidx = tI[jj];
#pragma unroll
        for (int s = 0; s < IPL; ++s) {
          const double dx = a.x - xi[s], dy = a.y - yi[s], dz = a.z - zi[s];
          const double r2 = dx * dx + dy * dy + dz * dz;
          const bool ok = (jidx != ii[s]) && (r2 > 0.0);
          coincident |= (jidx != ii[s]) && !(r2 > 0.0) && ii[s] >= 0;
          bool chg = true;
          if (MIXED) {
            const double inv = fmin(invi[s], b.x);
            chg = r2 * (inv * inv) < 1.0;
            const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
            const float ri = __frsqrt_rn(fdx * fdx + fdy * fdy + fdz * fdz);
            const float f = (chg || !ok) ? 0.0f : (float)a.w * ri * ri * ri;
            tx[s] += f * fdx;
            ty[s] += f * fdy;
            tz[s] += f * fdz;
          }
          if (chg) {
            const double r2s = ok ? r2 : 1.0;
            const double rinv = rsqrt(r2s);
            const double y = r2s * rinv * fmin(invi[s], b.x);
            const double x = fmin(fmax((y - A.gamma) * A.inv1mg, 0.0), 1.0);
            const double x2 = x * x;
            const double K = x2 * x2 * (35.0 + x * (-84.0 + x * (70.0 - 20.0 * x)));
            const double f = ok ? a.w * K * rinv * rinv * rinv : 0.0;
            ax[s] += f * dx;
            ay[s] += f * dy;
            az[s] += f * dz;
          }
        }
      }
      if (MIXED) {
#pragma unroll
        for (int s = 0; s < IPL; ++s) {
          ax[s] += (double)tx[s];
          ay[s] += (double)ty[s];
          az[s] += (double)tz[s];
        }
      }
      // neighbour candidates of this tile (rare): exact predicate
      for (int jj = 0; jj < nt; ++jj) {
        const double4 a = tA[jj];
        const double reachj = tB[jj].y;
        const int jidx = tI[jj];
#pragma unroll
        for (int s = 0; s < IPL; ++s) {
          const double dx = a.x - xi[s], dy = a.y - yi[s], dz = a.z - zi[s];
          const double r2 = dx * dx + dy * dy + dz * dz;
          const double rr = fmax(reachi[s], reachj);
          if (ii[s] >= 0 && jidx != ii[s] && r2 <= rr * rr * (1.0 + 1e-12) &&
              !(A.slow && (A.slow[A.sid[ii[s]]] | A.slow[A.sid[jidx]]))) {
            const int i = ii[s], j = jidx;
            if (pair_is_neighbour(A.sx[i], A.sy[i], A.sz[i], A.svx[i], A.svy[i], A.svz[i], A.sm[i], A.sro[i],
                                  A.srs[i], A.sx[j], A.sy[j], A.sz[j], A.svx[j], A.svy[j], A.svz[j], A.sm[j],
                                  A.sro[j], A.srs[j], A.G, A.rsch2, A.rsch3, A.dt)) {
              mark_close_pair(A, i, j);
              const unsigned long long p = atomicAdd(&A.cnt->n_pairs, 1ull);
              if ((int64_t)p < A.pair_cap)
                A.pairs[p] = make_int2(A.sid[i], A.sid[j]);
              else
                set_flag(A.cnt, P3T_FLAG_PAIR_OVERFLOW);
            }
          }
        }
      }
    }

    // ---------------- far particles (K = 1)
    const int32_t *Lf = A.pool + L.off + L.n_cell + L.n_near;
    if (!MIXED) {
      for (int t0 = 0; t0 < L.n_far; t0 += WAVE) {
        const int nt = min(WAVE, L.n_far - t0);
        __syncthreads();
        if (lane < nt) {
          const int j = Lf[t0 + lane];
          tA[lane] = make_double4(A.sx[j], A.sy[j], A.sz[j], A.G * A.sm[j]);
        }
        __syncthreads();
        for (int jj = 0; jj < nt; ++jj) {
          const double4 a = tA[jj];
#pragma unroll
          for (int s = 0; s < IPL; ++s) {
            const double dx = a.x - xi[s], dy = a.y - yi[s], dz = a.z - zi[s];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double rinv = rsqrt(r2);
            const double f = a.w * rinv * rinv * rinv;
            ax[s] += f * dx;
            ay[s] += f * dy;
            az[s] += f * dz;
          }
        }
      }
    } else {
      float fxi[IPL], fyi[IPL], fzi[IPL];
      float hx[IPL], hy[IPL], hz[IPL], lx[IPL], ly[IPL], lz[IPL];
#pragma unroll
      for (int s = 0; s < IPL; ++s) {
        fxi[s] = (float)(xi[s] - gcx);
        fyi[s] = (float)(yi[s] - gcy);
        fzi[s] = (float)(zi[s] - gcz);
        hx[s] = hy[s] = hz[s] = lx[s] = ly[s] = lz[s] = 0.0f;
      }
      for (int t0 = 0; t0 < L.n_far; t0 += WAVE) {
        const int nt = min(WAVE, L.n_far - t0);
        __syncthreads();
        if (lane < nt) {
          const int j = Lf[t0 + lane];
          fA[lane] = make_float4((float)(A.sx[j] - gcx), (float)(A.sy[j] - gcy), (float)(A.sz[j] - gcz),
                                 (float)(A.G * A.sm[j]));
        }
        __syncthreads();
        float tx[IPL], ty[IPL], tz[IPL];
#pragma unroll
        for (int s = 0; s < IPL; ++s) tx[s] = ty[s] = tz[s] = 0.0f;
        for (int jj = 0; jj < nt; ++jj) {
          const float4 a = fA[jj];
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
#pragma unroll
        for (int s = 0; s < IPL; ++s) {
          two_sum_acc(hx[s], lx[s], tx[s]);
          two_sum_acc(hy[s], ly[s], ty[s]);
          two_sum_acc(hz[s], lz[s], tz[s]);
        }
      }
#pragma unroll
      for (int s = 0; s < IPL; ++s) {
        ax[s] += (double)hx[s] + (double)lx[s];
        ay[s] += (double)hy[s] + (double)ly[s];
        az[s] += (double)hz[s] + (double)lz[s];
      }
    }

    // ---------------- cells (K = 1): monopole or quadrupole
    const int32_t *Lc = A.pool + L.off;
    if (!MIXED) {
      for (int t0 = 0; t0 < L.n_cell; t0 += WAVE) {
        const int nt = min(WAVE, L.n_cell - t0);
        __syncthreads();
        if (lane < nt) {
          const CellMom c = A.cm[Lc[t0 + lane]];
          tA[lane] = make_double4(c.com[0], c.com[1], c.com[2], A.G * c.mass);
          if (QUAD) {
            tB[lane] = make_double4(A.G * c.q[0], A.G * c.q[1], A.G * c.q[2], A.G * c.q[3]);
            tC[lane] = make_double2(A.G * c.q[4], A.G * c.q[5]);
          }
        }
        __syncthreads();
        for (int jj = 0; jj < nt; ++jj) {
          const double4 a = tA[jj];
          double4 qa;
          double2 qb;
          if (QUAD) {
            qa = tB[jj];
            qb = tC[jj];
          }
#pragma unroll
          for (int s = 0; s < IPL; ++s) {
            const double dx = a.x - xi[s], dy = a.y - yi[s], dz = a.z - zi[s];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double rinv = rsqrt(r2);
            const double rinv2 = rinv * rinv;
            const double rinv3 = rinv * rinv2;
            double fx = a.w * rinv3 * dx, fy = a.w * rinv3 * dy, fz = a.w * rinv3 * dz;
            if (QUAD) {
              // a = G [ M d / r^3 - Q d / r^5 + (5/2) (d.Q d) d / r^7 ],  d = X_c - x_i
              const double qx = qa.x * dx + qa.w * dy + qb.x * dz;
              const double qy = qa.w * dx + qa.y * dy + qb.y * dz;
              const double qz = qb.x * dx + qb.y * dy + qa.z * dz;
              const double dqd = dx * qx + dy * qy + dz * qz;
              const double rinv5 = rinv3 * rinv2;
              const double c7 = 2.5 * dqd * rinv5 * rinv2;
              fx += c7 * dx - qx * rinv5;
              fy += c7 * dy - qy * rinv5;
              fz += c7 * dz - qz * rinv5;
            }
            ax[s] += fx;
            ay[s] += fy;
            az[s] += fz;
          }
        }
      }
    } else {
      float fxi[IPL], fyi[IPL], fzi[IPL];
      float hx[IPL], hy[IPL], hz[IPL], lx[IPL], ly[IPL], lz[IPL];
#pragma unroll
      for (int s = 0; s < IPL; ++s) {
        fxi[s] = (float)(xi[s] - gcx);
        fyi[s] = (float)(yi[s] - gcy);
        fzi[s] = (float)(zi[s] - gcz);
        hx[s] = hy[s] = hz[s] = lx[s] = ly[s] = lz[s] = 0.0f;
      }
      for (int t0 = 0; t0 < L.n_cell; t0 += WAVE) {
        const int nt = min(WAVE, L.n_cell - t0);
        __syncthreads();
        if (lane < nt) {
          const CellMom c = A.cm[Lc[t0 + lane]];
          fA[lane] = make_float4((float)(c.com[0] - gcx), (float)(c.com[1] - gcy), (float)(c.com[2] - gcz),
                                 (float)(A.G * c.mass));
          if (QUAD) {
            fB[lane] = make_float4((float)(A.G * c.q[0]), (float)(A.G * c.q[1]), (float)(A.G * c.q[2]),
                                   (float)(A.G * c.q[3]));
            fC[lane] = make_float2((float)(A.G * c.q[4]), (float)(A.G * c.q[5]));
          }
        }
        __syncthreads();
        float tx[IPL], ty[IPL], tz[IPL];
#pragma unroll
        for (int s = 0; s < IPL; ++s) tx[s] = ty[s] = tz[s] = 0.0f;
        for (int jj = 0; jj < nt; ++jj) {
          const float4 a = fA[jj];
          float4 qa;
          float2 qb;
          if (QUAD) {
            qa = fB[jj];
            qb = fC[jj];
          }
#pragma unroll
          for (int s = 0; s < IPL; ++s) {
            const float dx = a.x - fxi[s], dy = a.y - fyi[s], dz = a.z - fzi[s];
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float rinv = __frsqrt_rn(r2);
            const float rinv2 = rinv * rinv;
            const float rinv3 = rinv * rinv2;
            float fx = a.w * rinv3 * dx, fy = a.w * rinv3 * dy, fz = a.w * rinv3 * dz;
            if (QUAD) {
              const float qx = qa.x * dx + qa.w * dy + qb.x * dz;
              const float qy = qa.w * dx + qa.y * dy + qb.y * dz;
              const float qz = qb.x * dx + qb.y * dy + qa.z * dz;
              const float dqd = dx * qx + dy * qy + dz * qz;
              const float rinv5 = rinv3 * rinv2;
              const float c7 = 2.5f * dqd * rinv5 * rinv2;
              fx += c7 * dx - qx * rinv5;
              fy += c7 * dy - qy * rinv5;
              fz += c7 * dz - qz * rinv5;
            }
            tx[s] += fx;
            ty[s] += fy;
            tz[s] += fz;
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
        ax[s] += (double)hx[s] + (double)lx[s];
        ay[s] += (double)hy[s] + (double)ly[s];
        az[s] += (double)hz[s] + (double)lz[s];
      }
    }

    // ---------------- write back in original order
#pragma unroll
    for (int s = 0; s < IPL; ++s) {
      if (ii[s] >= 0) {
        const int64_t o = A.sid[ii[s]];
        A.acc[o] = ax[s];
        A.acc[A.n + o] = ay[s];
        A.acc[2 * A.n + o] = az[s];
        if (!(isfinite(ax[s]) && isfinite(ay[s]) && isfinite(az[s]))) set_flag(A.cnt, P3T_FLAG_NAN);
      }
    }
    if (__ballot(coincident) != 0ull && lane == 0) set_flag(A.cnt, P3T_FLAG_COINCIDENT);
    if (lane == 0) {
      const unsigned long long ni = (unsigned long long)gcount;
      atomicAdd(&A.cnt->n_near, ni * (unsigned long long)L.n_near - ni);
      atomicAdd(&A.cnt->n_far, ni * (unsigned long long)L.n_far);
      atomicAdd(&A.cnt->n_cell, ni * (unsigned long long)L.n_cell);
    }
  }
}

template <bool MIXED, bool QUAD>
static void launch_ipl(const ForceArgs &A, int ipl, unsigned grid, hipStream_t s) {
  if (ipl == 1)
    hipLaunchKernelGGL((k_force<MIXED, QUAD, 1>), dim3(grid), dim3(WAVE), 0, s, A);
  else
    hipLaunchKernelGGL((k_force<MIXED, QUAD, 2>), dim3(grid), dim3(WAVE), 0, s, A);
}

hipError_t soft_force(p3t_ctx *c, int64_t n_groups_max, double *acc3, bool frozen) {
  const p3t_params &P = c->P;
  ForceArgs A;
  A.sx = c->sx;
  A.sy = c->sy;
  A.sz = c->sz;
  A.sm = c->sm;
  A.sinv = c->sinv;
  A.sreach = c->sreach;
  A.svx = c->svx;
  A.svy = c->svy;
  A.svz = c->svz;
  A.srs = c->srs;
  A.sro = c->sro;
  A.sid = c->sid;
  A.wn = c->wnode;
  A.cm = c->cmom;
  A.gl = c->glist;
  A.order = c->group_order;
  A.pool = c->pool;
  A.cnt = c->cnt;
  A.pairs = c->pairs;
  A.pair_cap = c->pair_cap;
  A.cands = c->cands;
  A.cand_cap = c->cand_cap;
  A.cand_slab = c->force_persistent ? 512 : 0;
  A.slow = c->slow_active ? c->slow_flag : nullptr;
  if (frozen) A.pair_cap = A.cand_cap = 0;
  // the close pairs of this evaluation (a kernel clears the flags: the
  // evaluation may be captured into a graph)
  A.close = frozen ? nullptr : c->close_flag;
  A.close_k = P.G * P.dt_soft * P.dt_soft / (CLOSE_RATIO * CLOSE_RATIO);
  if (A.close) {
    const hipError_t e = fill_i32(reinterpret_cast<int32_t *>(c->close_flag), 0, (c->n + 3) / 4, c->stream);
    if (e != hipSuccess) return e;
  }
  A.acc = acc3;
  A.n = c->n;
  A.G = P.G;
  A.gamma = P.gamma;
  A.inv1mg = 1.0 / (1.0 - P.gamma);
  A.rsch2 = P.r_search2;
  A.rsch3 = P.r_search3;
  A.dt = P.dt_soft;
  A.persistent = c->force_persistent;
  A.ngroups_bound = (int)std::min<int64_t>(n_groups_max, INT32_MAX);
  A.queue = &c->cnt->force_queue;
  unsigned grid = A.persistent ? (unsigned)c->force_slots : (unsigned)std::max<int64_t>(1, n_groups_max);
  if (c->fcfg.split) return soft_force_split(c, A, (unsigned)std::max<int64_t>(1, n_groups_max), acc3);
  const int ipl = P.n_group_max > WAVE ? 2 : 1;
  const bool mixed = P.precision == 1, quad = P.multipole == 2;
  if (mixed && quad)
    launch_ipl<true, true>(A, ipl, grid, c->stream);
  else if (mixed)
    launch_ipl<true, false>(A, ipl, grid, c->stream);
  else if (quad)
    launch_ipl<false, true>(A, ipl, grid, c->stream);
  else
    launch_ipl<false, false>(A, ipl, grid, c->stream);
  return hipGetLastError();
}

}  // namespace p3t
