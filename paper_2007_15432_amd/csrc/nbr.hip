// nbr.hip -- neighbour lists as CSR (Section 2.3), neighbour-cluster indices
// and the cluster CSR.
//
// Neighbour pairs (i, j) in original indices arrive unordered from the force
// kernel.  CSR: per-row counts, exclusive scan, scatter, then each row is
// sorted ascending (rows are short: <n_b> << 1 in the regime the method is
// meant for).  The result does not depend on the arrival order.
//
// Cluster index (Section 2.3 steps i-iii: the fixed point of "take the
// minimum index over yourself and your neighbours") is the minimum index of
// the particle's connected component.  Computed with a lock-free union-find
// that always hooks the larger root under the smaller one, so every
// component's root is its minimum index.
#include "p3t_internal.h"

namespace p3t {

__global__ void k_pair_count(const int2 *__restrict__ pairs, int64_t np, int32_t *__restrict__ cnt) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[pairs[p].x], 1);
}

__global__ void k_pair_fill(const int2 *__restrict__ pairs, int64_t np, const int64_t *__restrict__ row_ptr,
                            int32_t *__restrict__ cur, int32_t *__restrict__ col) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    const int2 e = pairs[p];
    const int64_t pos = row_ptr[e.x] + atomicAdd(&cur[e.x], 1);
    col[pos] = e.y;
  }
}

__global__ void k_row_sort(int64_t n, const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = row_ptr[i], b = row_ptr[i + 1];
    for (int64_t k = a + 1; k < b; ++k) {
      const int32_t v = col[k];
      int64_t q = k - 1;
      while (q >= a && col[q] > v) {
        col[q + 1] = col[q];
        --q;
      }
      col[q + 1] = v;
    }
  }
}

static inline unsigned g1d(int64_t n, int64_t cap = 65536) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

hipError_t build_csr(p3t_ctx *c, int64_t n, int64_t np) {
  hipStream_t s = c->stream;
  hipError_t e;
  if ((e = fill_i32(c->row_cnt, 0, n, s)) != hipSuccess) return e;
  if (np > 0) hipLaunchKernelGGL(k_pair_count, dim3(g1d(np)), dim3(256), 0, s, c->pairs, np, c->row_cnt);
  if ((e = scan_i32_to_i64(c->row_cnt, c->csr_ptr, n, c->scan_tmp, c->scan_tmp_cap, s)) != hipSuccess) return e;
  if ((e = fill_i32(c->row_cnt, 0, n, s)) != hipSuccess) return e;
  if (np > 0) {
    hipLaunchKernelGGL(k_pair_fill, dim3(g1d(np)), dim3(256), 0, s, c->pairs, np, c->csr_ptr, c->row_cnt, c->csr_col);
    hipLaunchKernelGGL(k_row_sort, dim3(g1d(n)), dim3(256), 0, s, n, c->csr_ptr, c->csr_col);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ union-find
__device__ __forceinline__ int uf_load(int32_t *p, int i) {
  return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int uf_find(int32_t *p, int i) {
  int r = uf_load(p, i);
  while (r != i) {
    i = r;
    r = uf_load(p, i);
  }
  return i;
}

__global__ void k_uf_init(int64_t n, int32_t *__restrict__ p) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}

// Joins the components of a and b: the larger root is hooked under the
// smaller one, so every root stays its component's minimum index.
__device__ __forceinline__ void uf_union(int32_t *p, int a, int b) {
  a = uf_find(p, a);
  b = uf_find(p, b);
  while (a != b) {
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    // a > b: hook root a under b
    const int old = atomicCAS(p + a, a, b);
    if (old == a) break;
    a = uf_find(p, old);
    b = uf_find(p, b);
  }
}

__global__ void k_uf_link(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, int32_t *p) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
      const int j = col[q];
      if (j <= i) continue;  // each undirected edge once
      uf_union(p, (int)i, j);
    }
  }
}

// The same components straight from the unordered pair list, whose length
// is read on the device (clamped to the buffer): a component does not
// depend on the order in which its edges are joined.  The list holds every
// pair in both directions (the neighbour test is symmetric, and the direct
// terms of parked members report both), so each edge is joined once, from
// its (smaller, larger) entry.
__global__ void k_uf_link_pairs(int64_t n, const int2 *__restrict__ pairs, const unsigned long long *__restrict__ np_dev,
                                int64_t cap, int32_t *p) {
  const int64_t np = (int64_t)*np_dev < cap ? (int64_t)*np_dev : cap;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < np; q += (int64_t)gridDim.x * blockDim.x) {
    const int2 e = pairs[q];
    if (e.x >= e.y || (uint32_t)e.x >= (uint64_t)n || (uint32_t)e.y >= (uint64_t)n) continue;
    uf_union(p, e.x, e.y);
  }
}

// The pairs appended last to a pair list of np_dev entries: the nd_dev
// (clamped to cap_d) at its end, which the direct terms of parked members
// append after the join.
__global__ void k_uf_link_tail(int64_t n, const int2 *__restrict__ pairs, const unsigned long long *__restrict__ np_dev,
                               const unsigned long long *__restrict__ nd_dev, int64_t cap_d, int64_t cap, int32_t *p) {
  const int64_t np = (int64_t)*np_dev < cap ? (int64_t)*np_dev : cap;
  const int64_t nd = (int64_t)*nd_dev < cap_d ? (int64_t)*nd_dev : cap_d;
  const int64_t q0 = np - nd > 0 ? np - nd : 0;
  for (int64_t q = q0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < np; q += (int64_t)gridDim.x * blockDim.x) {
    const int2 e = pairs[q];
    if (e.x >= e.y || (uint32_t)e.x >= (uint64_t)n || (uint32_t)e.y >= (uint64_t)n) continue;
    uf_union(p, e.x, e.y);
  }
}

__global__ void k_uf_final(int64_t n, int32_t *p, int32_t *__restrict__ label) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    label[i] = uf_find(p, (int)i);
}

// labels and the (label, index) sort keys of the cluster CSR in one pass
__global__ void k_uf_final_keys(int64_t n, int32_t *p, int32_t *__restrict__ label, uint64_t *__restrict__ key) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int r = uf_find(p, (int)i);
    label[i] = r;
    key[i] = ((uint64_t)(uint32_t)r << 32) | (uint64_t)(uint32_t)i;
  }
}

hipError_t labels_cc(p3t_ctx *c, int64_t n, int32_t *label) {
  hipStream_t s = c->stream;
  c->uf_early = 0;  // the parents are rebuilt here
  hipLaunchKernelGGL(k_uf_init, dim3(g1d(n)), dim3(256), 0, s, n, c->uf_parent);
  hipLaunchKernelGGL(k_uf_link, dim3(g1d(n)), dim3(256), 0, s, n, c->csr_ptr, c->csr_col, c->uf_parent);
  hipLaunchKernelGGL(k_uf_final, dim3(g1d(n)), dim3(256), 0, s, n, c->uf_parent, label);
  return hipGetLastError();
}

// Labels from the pair list of the last evaluation without building its
// CSR (the pair count stays on the device), and the cluster sort keys
// (c->cl_keys) for clusters_csr_dev(..., keys_ready = true).
hipError_t labels_pairs(p3t_ctx *c, int64_t n, int32_t *label) {
  hipStream_t s = c->stream;
  if (c->uf_early == n) {
    // the evaluation's own pairs are joined already (labels_pairs_early):
    // only the parked members' pairs, appended after the join, remain
    const unsigned gt = (unsigned)std::max<int64_t>(1, std::min<int64_t>(256, (c->pairs_d_cap + 255) / 256));
    hipLaunchKernelGGL(k_uf_link_tail, dim3(gt), dim3(256), 0, s, n, c->pairs, &c->cnt->n_pairs, &c->cnt->n_pairs_d,
                       c->pairs_d_cap, c->pair_cap, c->uf_parent);
  } else {
    hipLaunchKernelGGL(k_uf_init, dim3(g1d(n)), dim3(256), 0, s, n, c->uf_parent);
    const unsigned gp = (unsigned)std::min<int64_t>(2048, (c->pair_cap + 255) / 256);
    hipLaunchKernelGGL(k_uf_link_pairs, dim3(gp < 1 ? 1 : gp), dim3(256), 0, s, n, c->pairs, &c->cnt->n_pairs,
                       c->pair_cap, c->uf_parent);
  }
  c->uf_early = 0;
  hipLaunchKernelGGL(k_uf_final_keys, dim3(g1d(n)), dim3(256), 0, s, n, c->uf_parent, label, c->cl_keys);
  return hipGetLastError();
}

// The union-find over the pairs an evaluation has written so far, on the
// main stream while it waits for the parked members' direct terms;
// labels_pairs then joins only the pairs those append.  Marks the parents
// as holding the first pass for n particles.
hipError_t labels_pairs_early(p3t_ctx *c, int64_t n) {
  hipStream_t s = c->stream;
  hipLaunchKernelGGL(k_uf_init, dim3(g1d(n)), dim3(256), 0, s, n, c->uf_parent);
  const unsigned gp = (unsigned)std::min<int64_t>(2048, (c->pair_cap + 255) / 256);
  hipLaunchKernelGGL(k_uf_link_pairs, dim3(gp < 1 ? 1 : gp), dim3(256), 0, s, n, c->pairs, &c->cnt->n_pairs,
                     c->pair_cap, c->uf_parent);
  const hipError_t e = hipGetLastError();
  c->uf_early = e == hipSuccess ? n : 0;
  return e;
}

// ------------------------------------------------------------------ cluster CSR
__global__ void k_cl_keys(int64_t n, const int32_t *__restrict__ label, uint64_t *__restrict__ key) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    key[i] = ((uint64_t)(uint32_t)label[i] << 32) | (uint64_t)(uint32_t)i;
}

__global__ void k_cl_flags(int64_t n, const uint64_t *__restrict__ key, int32_t *__restrict__ members,
                           int32_t *__restrict__ flag) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    members[k] = (int32_t)(key[k] & 0xffffffffull);
    flag[k] = (k == 0 || (key[k] >> 32) != (key[k - 1] >> 32)) ? 1 : 0;
  }
}

__global__ void k_cl_ptr(int64_t n, const int32_t *__restrict__ flag, const int64_t *__restrict__ pos,
                         int32_t *__restrict__ cl_ptr) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    if (flag[k]) cl_ptr[pos[k]] = (int32_t)k;
  if (blockIdx.x == 0 && threadIdx.x == 0) cl_ptr[pos[n]] = (int32_t)n;
}

hipError_t clusters_csr(p3t_ctx *c, int64_t n, const int32_t *label, int32_t *cl_ptr, int32_t *cl_members,
                        int64_t *n_clusters) {
  hipError_t e = clusters_csr_dev(c, n, label, cl_ptr, cl_members);
  if (e != hipSuccess) return e;
  int64_t nc = 0;
  if ((e = hipMemcpyAsync(&nc, c->node_scan + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
  *n_clusters = nc;
  return hipSuccess;
}

// The same without the host round trip: the cluster count is left at
// node_scan[n] on the device.  keys_ready: c->cl_keys already holds the
// keys of label (labels_pairs wrote them).
hipError_t clusters_csr_dev(p3t_ctx *c, int64_t n, const int32_t *label, int32_t *cl_ptr, int32_t *cl_members,
                            bool keys_ready) {
  hipStream_t s = c->stream;
  hipError_t e;
  if (!keys_ready) hipLaunchKernelGGL(k_cl_keys, dim3(g1d(n)), dim3(256), 0, s, n, label, c->cl_keys);
  int bits = 1;
  while ((int64_t(1) << bits) < n) ++bits;
  // keys start ascending in the particle index, so a stable sort on the
  // label bits alone orders by (label, index)
  uint64_t *k = c->cl_keys, *ka = c->cl_keys_alt;
  int32_t *v = nullptr, *va = nullptr;
  if ((e = radix_sort_pairs(k, v, ka, va, n, nullptr, 32, 32 + bits, c->radix_hist, c->radix_hist_cap, c->scan_tmp,
                            c->scan_tmp_cap, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_cl_flags, dim3(g1d(n)), dim3(256), 0, s, n, k, cl_members, c->row_cnt);
  // (the node-scan buffer is free here; the neighbour CSR stays intact)
  if ((e = scan_i32_to_i64(c->row_cnt, c->node_scan, n, c->scan_tmp, c->scan_tmp_cap, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cl_ptr, dim3(g1d(n)), dim3(256), 0, s, n, c->row_cnt, c->node_scan, cl_ptr);
  return hipGetLastError();
}

}  // namespace p3t
