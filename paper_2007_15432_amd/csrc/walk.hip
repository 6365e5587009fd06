// walk.hip -- per-group tree walk producing three interaction lists.
//
// For a group g (a tree node of at most n_group_max particles) and a node c:
//   separated(g, c): the bounding-box distance exceeds max(reach_g, reach_c)
//     (reach = max(r_search, r_out) over the members) with a 1e-12 guard, so
//     no pair between them can be a neighbour candidate or feel K < 1;
//   accepted(g, c): separated, more than one particle, and the opening test
//     l_c < theta * d (l_c the longest edge of c's box, d the distance from
//     c's centre of mass to g's box);
// accepted nodes become multipole CELLS; opened leaves (<= n_leaf_max
// particles) give NEAR particles if not separated, FAR particles otherwise;
// other opened nodes push their two children.  theta = 0 accepts nothing,
// which reduces the tree force to the direct sum.
//
// One wavefront per group, persistent grid pulling groups from a counter.
// The DFS stack and the three lists live in per-wave global scratch; the
// finished lists are copied to a shared pool at an atomically reserved
// offset.  Every write is bounds-checked; an overflow marks the group
// (offset -1) and sets a status bit so that the host can grow and retry.
#include "p3t_internal.h"

namespace p3t {

constexpr int GROUP_CLASSES = 128;

__global__ __launch_bounds__(WAVE) void k_walk(const WalkNode *__restrict__ wn, const int32_t *__restrict__ group_node,
                                               DevCounters *cnt, GroupList *__restrict__ gl, int32_t *__restrict__ pool,
                                               int64_t pool_cap, int32_t *__restrict__ slot_lists, int cap,
                                               int32_t *__restrict__ slot_stack, int stack_cap, double theta2,
                                               int n_leaf) {
  const int lane = threadIdx.x;
  int32_t *Lc = slot_lists + (int64_t)blockIdx.x * 3 * cap;
  int32_t *Ln = Lc + cap;
  int32_t *Lf = Ln + cap;
  int32_t *stk = slot_stack + (int64_t)blockIdx.x * stack_cap;
  const int ngroups = uniform_first((int)cnt->n_groups);
  for (;;) {
    // every lane executes the atomic (lane 0 adds one, the others zero), so
    // no divergent branch feeds the loop exit; lane 0's ticket goes to an SGPR
    const int gi = (int)wave_fetch_add(&cnt->walk_queue, 1ull);
    if (gi >= ngroups) break;
    const int g = group_node[gi];
    double glo[3], ghi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      glo[d] = wn[g].lo[d];
      ghi[d] = wn[g].hi[d];
    }
    const double greach = wn[g].reach;
    int top = 1, ncell = 0, nnear = 0, nfar = 0;
    bool ovf = false;
    if (lane == 0) stk[0] = 0;  // root
    while (top > 0 && !ovf) {
      __syncthreads();
      const int npop = top < WAVE ? top : WAVE;
      const int node = lane < npop ? stk[top - npop + lane] : -1;
      top -= npop;
      __syncthreads();
      int outcome = 0;  // 0 none, 1 cell, 2 near leaf, 3 far leaf, 4 open
      int first = 0, count = 0, left = 0, right = 0;
      if (node >= 0) {
        const WalkNode W = wn[node];
        double dbb2 = 0.0, dc2 = 0.0, l = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double gap = fmax(fmax(W.lo[d] - ghi[d], glo[d] - W.hi[d]), 0.0);
          dbb2 += gap * gap;
          const double cg = fmax(fmax(glo[d] - W.com[d], W.com[d] - ghi[d]), 0.0);
          dc2 += cg * cg;
          l = fmax(l, W.hi[d] - W.lo[d]);
        }
        const double rr = fmax(greach, W.reach) * (1.0 + 1e-12);
        const bool sep = dbb2 > rr * rr;
        const bool accept = sep && W.count > 1 && l * l < theta2 * dc2;
        first = W.first;
        count = W.count;
        left = W.left;
        right = W.right;
        if (accept)
          outcome = 1;
        else if (W.count <= n_leaf || W.left < 0)
          outcome = sep ? 3 : 2;
        else
          outcome = 4;
      }
      // cells
      const unsigned long long mc = __ballot(outcome == 1);
      if (outcome == 1) {
        const int p = ncell + popc_below(mc);
        if (p < cap) Lc[p] = node;
      }
      ncell += (int)__popcll(mc);
      // near particles
      {
        const int cn = outcome == 2 ? count : 0;
        const int incl = wave_incl_scan(cn);
        const int start = nnear + incl - cn;
        for (int q = 0; q < cn && start + q < cap; ++q) Ln[start + q] = first + q;
        nnear += uniform_lane(incl, WAVE - 1);
      }
      // far particles
      {
        const int cf = outcome == 3 ? count : 0;
        const int incl = wave_incl_scan(cf);
        const int start = nfar + incl - cf;
        for (int q = 0; q < cf && start + q < cap; ++q) Lf[start + q] = first + q;
        nfar += uniform_lane(incl, WAVE - 1);
      }
      // opened internal nodes: push both children
      const unsigned long long mo = __ballot(outcome == 4);
      if (outcome == 4) {
        const int p = top + 2 * popc_below(mo);
        if (p + 1 < stack_cap) {
          stk[p] = left;
          stk[p + 1] = right;
        }
      }
      top += 2 * (int)__popcll(mo);
      if (ncell > cap || nnear > cap || nfar > cap || top > stack_cap) ovf = true;
    }
    if (ovf) {
      if (lane == 0) {
        set_flag(cnt, top > stack_cap ? P3T_FLAG_STACK_OVERFLOW : P3T_FLAG_LIST_OVERFLOW);
        GroupList o;
        o.off = -1;
        o.n_cell = o.n_near = o.n_far = 0;
        o.node = g;
        gl[gi] = o;
      }
      continue;
    }
    __syncthreads();
    const int total = ncell + nnear + nfar;
    const long long off = (long long)wave_fetch_add(&cnt->pool_cursor, (unsigned long long)total);
    if (off + total > pool_cap) {
      if (lane == 0) {
        set_flag(cnt, P3T_FLAG_LIST_OVERFLOW);
        GroupList o;
        o.off = -1;
        o.n_cell = o.n_near = o.n_far = 0;
        o.node = g;
        gl[gi] = o;
      }
      continue;
    }
    for (int q = lane; q < ncell; q += WAVE) pool[off + q] = Lc[q];
    for (int q = lane; q < nnear; q += WAVE) pool[off + ncell + q] = Ln[q];
    for (int q = lane; q < nfar; q += WAVE) pool[off + ncell + nnear + q] = Lf[q];
    if (lane == 0) {
      GroupList o;
      o.off = off;
      o.n_cell = ncell;
      o.n_near = nnear;
      o.n_far = nfar;
      o.node = g;
      gl[gi] = o;
    }
  }
}

__global__ void k_reset_queues(DevCounters *cnt) {
  cnt->walk_queue = 0;
  cnt->force_queue = 0;
  for (int k = 0; k < 3; ++k) cnt->queue[k] = 0;
  cnt->n_cand = 0;
  cnt->pool_cursor = 0;
  cnt->n_pairs = 0;
  cnt->n_near = 0;
  cnt->n_far = 0;
  cnt->n_cell = 0;
}

// Sort key of a group: (work descending, group index ascending).
// A device count above n_static (the host's bound, from the last evaluation)
// sets P3T_FLAG_GROUP_BOUND: the sort and the force then cover only the
// first n_static groups and the host evaluates again with the bound n.
// Work of a group (its i-particles times its list entries, cells counted
// twice), in classes of half an octave: the force kernels take the groups
// in descending class, so the longest lists start first and the tail of
// the launch is short.  Only the order of the work depends on it.
__device__ __forceinline__ int group_class(const GroupList &L, const WalkNode *__restrict__ wn) {
  const uint64_t ni = (uint64_t)wn[L.node].count;
  const uint64_t work = ni * (uint64_t)(L.n_near + L.n_far + 2 * L.n_cell) / 64 + 1;
  const int msb = 63 - __clzll((long long)work);
  const int half = msb > 0 ? (int)((work >> (msb - 1)) & 1ull) : 0;
  return min(GROUP_CLASSES - 1, 2 * msb + half);
}

// One workgroup: a counting sort of the groups by class, largest first
// (within a class in any order).  A device count above n_static (the host's
// bound, from the last evaluation) sets P3T_FLAG_GROUP_BOUND: the order and
// the force then cover only the first n_static groups and the host
// evaluates again with the bound n.
__global__ __launch_bounds__(1024) void k_group_order(const GroupList *__restrict__ gl,
                                                      const WalkNode *__restrict__ wn, int n_static, DevCounters *cnt,
                                                      int32_t *__restrict__ order) {
  __shared__ int hist[GROUP_CLASSES];
  const int t = threadIdx.x;
  int ng = (int)cnt->n_groups;
  if (ng > n_static) {
    if (t == 0) atomicOr(&cnt->status, P3T_FLAG_GROUP_BOUND);
    ng = n_static;
  }
  for (int q = t; q < GROUP_CLASSES; q += blockDim.x) hist[q] = 0;
  __syncthreads();
  for (int g = t; g < ng; g += blockDim.x) atomicAdd(&hist[group_class(gl[g], wn)], 1);
  __syncthreads();
  if (t == 0) {  // exclusive offsets, largest class first
    int acc = 0;
    for (int q = GROUP_CLASSES - 1; q >= 0; --q) {
      const int h = hist[q];
      hist[q] = acc;
      acc += h;
    }
  }
  __syncthreads();
  for (int g = t; g < ng; g += blockDim.x) order[atomicAdd(&hist[group_class(gl[g], wn)], 1)] = g;
}

hipError_t walk_groups(p3t_ctx *c, int64_t n_groups_max) {
  hipStream_t s = c->stream;
  hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(1), 0, s, c->cnt);
  const double th = c->P.theta;
  hipLaunchKernelGGL(k_walk, dim3(c->walk_slots), dim3(WAVE), 0, s, c->wnode, c->group_node, c->cnt, c->glist, c->pool,
                     c->pool_cap, c->slot_lists, (int)c->slot_cap_list, c->slot_stack, (int)c->slot_cap_stack, th * th,
                     c->P.n_leaf_max);
  // longest-first order for the force kernels; the device-side group count
  // bounds it, so n_groups_max may be any upper bound (a captured graph
  // passes the particle count)
  const int ns = (int)std::min<int64_t>(n_groups_max, INT32_MAX);
  hipLaunchKernelGGL(k_group_order, dim3(1), dim3(1024), 0, s, c->glist, c->wnode, ns, c->cnt, c->group_order);
  return hipGetLastError();
}

void reset_queues(p3t_ctx *c) { hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(1), 0, c->stream, c->cnt); }

}  // namespace p3t
