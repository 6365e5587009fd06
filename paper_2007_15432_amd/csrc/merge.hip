// merge.hip -- perfect accretion after a hard part with collisions (Section
// 2.5.1): every composite left by the hard part (its parts share one state)
// becomes one particle.  The part with the lowest index keeps the state and
// takes the composite's mass (its own mass plus the absorbed parts' masses,
// added in index order); the other parts are removed and the particle arrays
// are compacted in index order (stride n_new).
#include "p3t_internal.h"

namespace p3t {

namespace {

constexpr int MT = 256;

__device__ __forceinline__ int64_t grid_stride() { return (int64_t)gridDim.x * blockDim.x; }
__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

// keep flags; a merged index outside [0, i] or not naming a survivor is an error
__global__ void k_merge_flags(int64_t n, const int32_t *__restrict__ merged, int32_t *__restrict__ keep,
                              int32_t *__restrict__ bad) {
  for (int64_t i = gtid(); i < n; i += grid_stride()) {
    const int32_t s = merged[i];
    const bool ok = s >= 0 && (int64_t)s <= i && merged[s] == s;
    if (!ok) atomicOr(bad, 1);
    keep[i] = s == (int32_t)i ? 1 : 0;
  }
}

// absorbed parts in index order: i - rank[i] absorbed parts precede i
__global__ void k_merge_list(int64_t n, const int32_t *__restrict__ merged, const int64_t *__restrict__ rank,
                             int32_t *__restrict__ list) {
  for (int64_t i = gtid(); i < n; i += grid_stride())
    if (merged[i] != (int32_t)i) list[i - rank[i]] = (int32_t)i;
}

__global__ void k_merge_copy_mass(int64_t n, const double *__restrict__ mass, double *__restrict__ tot) {
  for (int64_t i = gtid(); i < n; i += grid_stride()) tot[i] = mass[i];
}

// one thread: the absorbed masses onto their survivors, in index order
__global__ void k_merge_mass(int64_t n, const int64_t *__restrict__ rank, const int32_t *__restrict__ list,
                             const int32_t *__restrict__ merged, const double *__restrict__ mass,
                             double *__restrict__ tot) {
  const int64_t na = n - rank[n];
  for (int64_t k = 0; k < na; ++k) {
    const int32_t g = list[k];
    tot[merged[g]] += mass[g];
  }
}

// survivors into the staging buffer (stride n_new)
__global__ void k_merge_gather(int64_t n, const int64_t *__restrict__ rank, const int32_t *__restrict__ merged,
                               const double *__restrict__ pos3, const double *__restrict__ vel3,
                               const double *__restrict__ tot, const double *__restrict__ dt_hard,
                               const int32_t *__restrict__ steps, double *__restrict__ st, int32_t *__restrict__ ss) {
  const int64_t nn = rank[n];
  for (int64_t i = gtid(); i < n; i += grid_stride()) {
    if (merged[i] != (int32_t)i) continue;
    const int64_t j = rank[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      st[d * nn + j] = pos3[d * n + i];
      st[(3 + d) * nn + j] = vel3[d * n + i];
    }
    st[6 * nn + j] = tot[i];
    if (dt_hard) st[7 * nn + j] = dt_hard[i];
    if (steps) ss[j] = steps[i];
  }
}

__global__ void k_merge_scatter(int64_t n, const int64_t *__restrict__ rank, const double *__restrict__ st,
                                const int32_t *__restrict__ ss, double *__restrict__ pos3, double *__restrict__ vel3,
                                double *__restrict__ mass, double *__restrict__ dt_hard, int32_t *__restrict__ steps) {
  const int64_t nn = rank[n];
  for (int64_t j = gtid(); j < nn; j += grid_stride()) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      pos3[d * nn + j] = st[d * nn + j];
      vel3[d * nn + j] = st[(3 + d) * nn + j];
    }
    mass[j] = st[6 * nn + j];
    if (dt_hard) dt_hard[j] = st[7 * nn + j];
    if (steps) steps[j] = ss[j];
  }
}

// sums of six columns over nc rows, in a fixed order: thread t takes rows
// t, t + MT, ...; the partials are added in thread order
__global__ __launch_bounds__(MT) void k_sum_rows6(int64_t nc, const double *__restrict__ rows, double *__restrict__ out) {
  __shared__ double part[6][MT];
  const int t = threadIdx.x;
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t r = t; r < nc; r += MT)
    for (int q = 0; q < 6; ++q) s[q] += rows[6 * r + q];
  for (int q = 0; q < 6; ++q) part[q][t] = s[q];
  __syncthreads();
  if (t < 6) {
    double a = 0.0;
    for (int k = 0; k < MT; ++k) a += part[t][k];
    out[t] = a;
  }
}

__global__ void k_fill_one_i32(int32_t *p, int32_t v) { *p = v; }

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (n + MT - 1) / MT)); }

}  // namespace

hipError_t sum_rows6(int64_t nc, const double *rows, double *out6, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_rows6, dim3(1), dim3(MT), 0, s, nc, rows, out6);
  return hipGetLastError();
}

// scratch: c->merge_st (9 n doubles: 8 staging rows of n_new <= n, the
// summed masses), c->merge_i32 (2 n + 1 int32), c->node_scan (n + 1 int64).
// The composite map is checked (and the host waits for the check) before
// any kernel indexes with it.
hipError_t merge_bodies(p3t_ctx *c, int64_t n, const int32_t *merged, double *pos3, double *vel3, double *mass,
                        double *dt_hard, int32_t *steps, int64_t *n_new) {
  hipStream_t s = c->stream;
  int32_t *keep = c->merge_i32, *ss = c->merge_i32 + n, *bad = c->merge_i32 + 2 * n;
  int64_t *rank = c->node_scan;
  double *st = c->merge_st, *tot = c->merge_st + 8 * n;
  hipError_t e;
  int32_t bad_h = 0;
  hipLaunchKernelGGL(k_fill_one_i32, dim3(1), dim3(1), 0, s, bad, 0);
  hipLaunchKernelGGL(k_merge_flags, dim3(grid_of(n)), dim3(MT), 0, s, n, merged, keep, bad);
  if ((e = hipMemcpyAsync(&bad_h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  if (bad_h) return hipErrorInvalidValue;
  if ((e = scan_i32_to_i64(keep, rank, n, c->scan_tmp, c->scan_tmp_cap, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_merge_list, dim3(grid_of(n)), dim3(MT), 0, s, n, merged, rank, keep);  // keep now holds the list
  hipLaunchKernelGGL(k_merge_copy_mass, dim3(grid_of(n)), dim3(MT), 0, s, n, mass, tot);
  hipLaunchKernelGGL(k_merge_mass, dim3(1), dim3(1), 0, s, n, rank, keep, merged, mass, tot);
  hipLaunchKernelGGL(k_merge_gather, dim3(grid_of(n)), dim3(MT), 0, s, n, rank, merged, pos3, vel3, tot, dt_hard,
                     steps, st, ss);
  hipLaunchKernelGGL(k_merge_scatter, dim3(grid_of(n)), dim3(MT), 0, s, n, rank, st, ss, pos3, vel3, mass, dt_hard,
                     steps);
  if ((e = hipMemcpyAsync(n_new, rank + n, sizeof(int64_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace p3t
