// util.hip -- device-wide building blocks: exclusive scans, a stable LSD radix
// sort of 64-bit keys with 32-bit values, bounding-box reduction, fills and
// the soft kick.  All kernels take their element count either as a host value
// or from a device counter (so data-dependent sizes need no host round trip).
#include "p3t_internal.h"

namespace p3t {

// ------------------------------------------------------------------ scan
constexpr int SCAN_T = 256;
constexpr int SCAN_I = 16;
constexpr int SCAN_TILE = SCAN_T * SCAN_I;

template <typename Tin>
__global__ __launch_bounds__(SCAN_T) void k_scan_sums(const Tin *__restrict__ in, int64_t n, int64_t *__restrict__ sums) {
  __shared__ int64_t ws[SCAN_T / WAVE];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int64_t s = 0;
#pragma unroll
  for (int r = 0; r < SCAN_I; ++r) {
    int64_t k = base + (int64_t)r * SCAN_T + t;
    if (k < n) s += (int64_t)in[k];
  }
  s = wave_sum(s);
  if ((t & (WAVE - 1)) == 0) ws[t / WAVE] = s;
  __syncthreads();
  if (t == 0) {
    int64_t tot = 0;
    for (int w = 0; w < SCAN_T / WAVE; ++w) tot += ws[w];
    sums[blockIdx.x] = tot;
  }
}

// exclusive scan of one tile (+ block offset).  If total_out, out[n] = total.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(SCAN_T) void k_scan_down(const Tin *__restrict__ in, Tout *__restrict__ out, int64_t n,
                                                      const int64_t *__restrict__ offs, int total_out) {
  __shared__ int64_t buf[SCAN_TILE];
  __shared__ int64_t ws[SCAN_T / WAVE];
  const int t = threadIdx.x, w = t / WAVE, l = t & (WAVE - 1);
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
  for (int r = 0; r < SCAN_I; ++r) {
    int64_t k = base + (int64_t)r * SCAN_T + t;
    buf[r * SCAN_T + t] = k < n ? (int64_t)in[k] : 0;
  }
  __syncthreads();
  int64_t s = 0;
#pragma unroll
  for (int q = 0; q < SCAN_I; ++q) s += buf[t * SCAN_I + q];
  int64_t incl = s;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int64_t v = __shfl_up(incl, o, WAVE);
    if (l >= o) incl += v;
  }
  if (l == WAVE - 1) ws[w] = incl;
  __syncthreads();
  int64_t run = (offs ? offs[blockIdx.x] : 0) + incl - s;
  for (int q = 0; q < w; ++q) run += ws[q];
#pragma unroll
  for (int q = 0; q < SCAN_I; ++q) {
    int64_t v = buf[t * SCAN_I + q];
    buf[t * SCAN_I + q] = run;
    run += v;
    // the thread holding element n-1 writes the grand total to out[n]
    if (total_out && base + t * SCAN_I + q == n - 1) out[n] = (Tout)run;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < SCAN_I; ++r) {
    int64_t k = base + (int64_t)r * SCAN_T + t;
    if (k < n) out[k] = (Tout)buf[r * SCAN_T + t];
  }
}

__global__ void k_write_zero_i64(int64_t *p) { *p = 0; }

int64_t scan_tmp_need(int64_t n) {
  int64_t need = 0;
  while (n > SCAN_TILE) {
    n = (n + SCAN_TILE - 1) / SCAN_TILE;
    need += n;
  }
  return need + 16;
}

template <typename Tin, typename Tout>
static hipError_t scan_impl(const Tin *in, Tout *out, int64_t n, int total_out, int64_t *tmp, int64_t tmp_cap,
                            hipStream_t s) {
  if (n <= 0) {
    if (total_out) hipLaunchKernelGGL(k_write_zero_i64, dim3(1), dim3(1), 0, s, (int64_t *)out);
    return hipGetLastError();
  }
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 1) {
    hipLaunchKernelGGL((k_scan_down<Tin, Tout>), dim3(1), dim3(SCAN_T), 0, s, in, out, n, (const int64_t *)nullptr,
                       total_out);
    return hipGetLastError();
  }
  if (tmp_cap < nb) return hipErrorInvalidValue;
  int64_t *sums = tmp;
  hipLaunchKernelGGL((k_scan_sums<Tin>), dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, n, sums);
  hipError_t e = scan_impl<int64_t, int64_t>(sums, sums, nb, 0, tmp + nb, tmp_cap - nb, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_scan_down<Tin, Tout>), dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, out, n,
                     (const int64_t *)sums, total_out);
  return hipGetLastError();
}

hipError_t scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, int64_t *tmp, int64_t tmp_cap, hipStream_t s) {
  return scan_impl<int32_t, int64_t>(in, out, n, 1, tmp, tmp_cap, s);
}

// ------------------------------------------------------------------ radix sort
// Stable LSD radix sort, 8-bit digits.  One block sorts a tile of RS_TILE
// keys per pass: a digit histogram per tile (hist[digit][tile]); one
// workgroup per digit scans its row over the tiles (exclusive, in place) and
// stores the row total; the stable scatter adds the exclusive scan of the
// 256 row totals (done again by every scatter block, in LDS) and ranks equal
// digits inside a wavefront with ballots and across wavefronts with
// per-round counters.  Three launches per pass, no device-wide scan.
constexpr int RS_T = 256;
constexpr int RS_I = 8;  // tiles of 2048 keys: 512 workgroups per pass for 2^20 keys
constexpr int RS_TILE = RS_T * RS_I;
constexpr int RS_W = RS_T / WAVE;

__device__ __forceinline__ int64_t dev_count(int64_t n_static, const unsigned long long *n_dev) {
  if (!n_dev) return n_static;
  int64_t d = (int64_t)(*n_dev);
  return d < n_static ? d : n_static;
}

__global__ __launch_bounds__(RS_T) void k_radix_hist(const uint64_t *__restrict__ kin, int64_t n_static,
                                                     const unsigned long long *n_dev, int shift,
                                                     uint32_t *__restrict__ hist, int nblocks) {
  __shared__ uint32_t h[256];
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const int64_t n = dev_count(n_static, n_dev);
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll 4
  for (int r = 0; r < RS_I; ++r) {
    int64_t k = base + (int64_t)r * RS_T + t;
    if (k < n) atomicAdd(&h[(unsigned)(kin[k] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)t * nblocks + blockIdx.x] = h[t];
}

// Row d of hist (nblocks tile counts of digit d) becomes its exclusive scan;
// tot[d] receives the row total.  One workgroup per digit.
constexpr int RR_I = 8;
__global__ __launch_bounds__(RS_T) void k_radix_rowscan(uint32_t *__restrict__ hist, int nblocks,
                                                        uint32_t *__restrict__ tot) {
  __shared__ uint32_t ws[RS_W];
  uint32_t *row = hist + (int64_t)blockIdx.x * nblocks;
  const int t = threadIdx.x, w = t / WAVE, l = t & (WAVE - 1);
  uint32_t carry = 0;
  for (int c0 = 0; c0 < nblocks; c0 += RS_T * RR_I) {  // uniform
    uint32_t v[RR_I], s = 0;
#pragma unroll
    for (int q = 0; q < RR_I; ++q) {
      const int i = c0 + t * RR_I + q;
      v[q] = i < nblocks ? row[i] : 0u;
      s += v[q];
    }
    const uint32_t incl = (uint32_t)wave_incl_scan((int)s);
    if (l == WAVE - 1) ws[w] = incl;
    __syncthreads();
    uint32_t run = carry + incl - s, chunk = 0;
#pragma unroll
    for (int q = 0; q < RS_W; ++q) {
      run += q < w ? ws[q] : 0u;
      chunk += ws[q];
    }
#pragma unroll
    for (int q = 0; q < RR_I; ++q) {
      const int i = c0 + t * RR_I + q;
      if (i < nblocks) row[i] = run;
      run += v[q];
    }
    carry += chunk;
    __syncthreads();  // ws is rewritten by the next chunk
  }
  if (t == 0) tot[blockIdx.x] = carry;
}

__global__ __launch_bounds__(RS_T) void k_radix_scatter(const uint64_t *__restrict__ kin, const int32_t *__restrict__ vin,
                                                        uint64_t *__restrict__ kout, int32_t *__restrict__ vout,
                                                        int64_t n_static, const unsigned long long *n_dev, int shift,
                                                        const uint32_t *__restrict__ offs, const uint32_t *__restrict__ tot,
                                                        int nblocks) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wc[RS_W][256];
  const int t = threadIdx.x, w = t / WAVE;
  const int64_t n = dev_count(n_static, n_dev);
  {
    // first position of digit t: exclusive scan of the row totals
    const uint32_t tv = tot[t];
    const uint32_t incl = (uint32_t)wave_incl_scan((int)tv);
    if ((t & (WAVE - 1)) == WAVE - 1) wc[0][w] = incl;
    __syncthreads();
    uint32_t base = incl - tv;
#pragma unroll
    for (int q = 0; q < RS_W; ++q) base += q < w ? wc[0][q] : 0u;
    run[t] = base + offs[(int64_t)t * nblocks + blockIdx.x];
    __syncthreads();  // wc is cleared below
  }
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_I; ++r) {
#pragma unroll
    for (int q = 0; q < RS_W; ++q) wc[q][t] = 0;
    __syncthreads();
    const int64_t k = base + (int64_t)r * RS_T + t;
    const bool valid = k < n;
    const uint64_t key = valid ? kin[k] : 0ull;
    const int32_t val = (valid && vin) ? vin[k] : 0;
    const unsigned d = (unsigned)(key >> shift) & 255u;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const int rank = popc_below(peers);
    if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t off = run[d] + (uint32_t)rank;
      for (int q = 0; q < w; ++q) off += wc[q][d];
      kout[off] = key;
      if (vout) vout[off] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int q = 0; q < RS_W; ++q) add += wc[q][t];
    run[t] += add;
    __syncthreads();
  }
}

int64_t radix_hist_need(int64_t n) { return 256 * ((n + RS_TILE - 1) / RS_TILE) + 256; }

hipError_t radix_sort_pairs(uint64_t *&keys, int32_t *&vals, uint64_t *&keys_alt, int32_t *&vals_alt, int64_t n_static,
                            const unsigned long long *n_dev, int bit_lo, int bit_hi, uint32_t *hist, int64_t hist_cap,
                            int64_t *tmp, int64_t tmp_cap, hipStream_t s) {
  if (n_static <= 0) return hipSuccess;
  const int64_t nb64 = (n_static + RS_TILE - 1) / RS_TILE;
  if (256 * nb64 + 256 > hist_cap || nb64 > (1 << 30)) return hipErrorInvalidValue;
  const int nb = (int)nb64;
  uint32_t *tot = hist + 256 * nb64;  // the 256 row totals follow the counters
  (void)tmp;
  (void)tmp_cap;
  for (int shift = bit_lo; shift < bit_hi; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(RS_T), 0, s, keys, n_static, n_dev, shift, hist, nb);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(RS_T), 0, s, hist, nb, tot);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(RS_T), 0, s, keys, vals, keys_alt, vals_alt, n_static, n_dev,
                       shift, hist, tot, nb);
    uint64_t *tk = keys;
    keys = keys_alt;
    keys_alt = tk;
    int32_t *tv = vals;
    vals = vals_alt;
    vals_alt = tv;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ fills, kick
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) p[k] = v;
}

static inline unsigned grid_for(int64_t n, int threads = 256, int64_t cap = 65536) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

__global__ void k_iota_i32(int32_t *p, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    p[k] = (int32_t)k;
}

__global__ void k_fill_f64(double *p, double v, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) p[k] = v;
}

hipError_t iota_i32(int32_t *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota_i32, dim3(grid_for(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t fill_f64(double *p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

__global__ void k_kick(int64_t n3, double h, const double *__restrict__ a, double *__restrict__ v) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n3; k += (int64_t)gridDim.x * blockDim.x)
    v[k] += h * a[k];
}

hipError_t kick(int64_t n, double h, const double *acc3, double *vel3, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kick, dim3(grid_for(3 * n)), dim3(256), 0, s, 3 * n, h, acc3, vel3);
  return hipGetLastError();
}

// ------------------------------------------------------------------ bounding box
constexpr int BB_BLOCKS = 1024;

__global__ __launch_bounds__(256) void k_bbox_part(const double *__restrict__ pos, int64_t n, double *__restrict__ part) {
  __shared__ double sh[6][256 / WAVE];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double x = pos[c * n + k];
      lo[c] = fmin(lo[c], x);
      hi[c] = fmax(hi[c], x);
    }
  }
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    lo[c] = wave_min(lo[c]);
    hi[c] = wave_max(hi[c]);
  }
  if ((t & (WAVE - 1)) == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sh[c][t / WAVE] = lo[c];
      sh[3 + c][t / WAVE] = hi[c];
    }
  }
  __syncthreads();
  if (t < 6) {
    double v = sh[t][0];
    for (int w = 1; w < 256 / WAVE; ++w) v = t < 3 ? fmin(v, sh[t][w]) : fmax(v, sh[t][w]);
    part[blockIdx.x * 6 + t] = v;
  }
}

// one 256-thread block: min / max over the per-block partials
__global__ __launch_bounds__(256) void k_bbox_final(const double *__restrict__ part, int nb, double *__restrict__ out) {
  __shared__ double sh[6][256 / WAVE];
  const int t = threadIdx.x;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = t; b < nb; b += 256) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lo[c] = fmin(lo[c], part[b * 6 + c]);
      hi[c] = fmax(hi[c], part[b * 6 + 3 + c]);
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    lo[c] = wave_min(lo[c]);
    hi[c] = wave_max(hi[c]);
  }
  if ((t & (WAVE - 1)) == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sh[c][t / WAVE] = lo[c];
      sh[3 + c][t / WAVE] = hi[c];
    }
  }
  __syncthreads();
  if (t < 6) {
    double v = sh[t][0];
    for (int w = 1; w < 256 / WAVE; ++w) v = t < 3 ? fmin(v, sh[t][w]) : fmax(v, sh[t][w]);
    out[t] = v;
  }
}

hipError_t bbox_reduce(const double *pos3, int64_t n, double *part, double *out, hipStream_t s) {
  const int nb = (int)grid_for(n, 256, BB_BLOCKS);
  hipLaunchKernelGGL(k_bbox_part, dim3(nb), dim3(256), 0, s, pos3, n, part);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(256), 0, s, part, nb, out);
  return hipGetLastError();
}

}  // namespace p3t
