// cutoff.hip -- per-particle cut-off and search radii (Hill radius of
// Section 2.1.1, eq. (routi2), eq. (rsearch); shared mode eq. (rout1)).
//
// The random velocity of a particle is |v - v_K| with v_K the circular speed
// sqrt(G M_* / |x|) along phi-hat; v_ran,i is the rms of that quantity over
// the particle's bin among `vran_bins` log-spaced bins in cylindrical radius
// (bins with too few members fall back to the rms over all particles).
// Bin sums are formed per block in a fixed order and combined in block order,
// so the result does not depend on scheduling.
#include <algorithm>
#include <cstdio>
#include <mutex>
#include <string>

#include "p3t_internal.h"

// No multiply-add contraction in this file: the staged and the recomputing
// passes then form every per-particle term with the same roundings (the
// compiler would otherwise fuse differently in different kernels), so both
// entry points give the same bits.  The passes are bound by memory, not by
// arithmetic.
#pragma clang fp contract(off)

namespace p3t {

constexpr int CUT_T = 256;
constexpr int CUT_PER = 4;
constexpr int CUT_CHUNK = CUT_T * CUT_PER;
constexpr int CUT_MAX_BINS = 256;

// The caller's particles and the constants of the per-particle terms.
struct CutIn {
  const double *pos, *vel, *m;
  int64_t n;
  double GM, m_star;
  int hill_length;
};

// Per-particle terms: cylindrical radius, squared random velocity |v -
// v_K phi-hat|^2 and the Hill radius (osculating semi-major axis, or |x|).
// The staged path stores them; the allocation-free path recomputes them
// where they are needed, with the same operations (same bits).
__device__ __forceinline__ void cut_terms(const CutIn &I, int64_t i, double &Rc, double &u2, double &rh) {
  const int64_t n = I.n;
  const double x = I.pos[i], y = I.pos[n + i], z = I.pos[2 * n + i];
  const double vx = I.vel[i], vy = I.vel[n + i], vz = I.vel[2 * n + i];
  const double r = sqrt(x * x + y * y + z * z);
  Rc = sqrt(x * x + y * y);
  const double v2 = vx * vx + vy * vy + vz * vz;
  double a;
  if (I.hill_length == 1) {
    a = r;
  } else {
    const double inv_a = 2.0 / r - v2 / I.GM;
    a = inv_a > 0.0 ? 1.0 / inv_a : r;  // unbound: fall back to |x|
  }
  rh = cbrt(I.m[i] / (3.0 * I.m_star)) * a;
  const double vk = sqrt(I.GM / r);
  const double phx = Rc > 0.0 ? -y / Rc : 0.0;
  const double phy = Rc > 0.0 ? x / Rc : 0.0;
  const double ux = vx - vk * phx, uy = vy - vk * phy, uz = vz;
  u2 = ux * ux + uy * uy + uz * uz;
}

// log-spaced bin of cylindrical radius R over [Rmin, Rmax]
__device__ __forceinline__ int cut_bin(double R, double Rmin, double lspan, int nbins) {
  int bb = 0;
  if (lspan > 0.0) {
    const double tt = floor((double)nbins * (log(R / Rmin) / lspan));
    bb = tt < 0.0 ? 0 : (tt > (double)(nbins - 1) ? nbins - 1 : (int)tt);
  }
  return bb;
}

__device__ __forceinline__ double cut_lspan(const double *mm) {
  const double Rmin = mm[0], Rmax = mm[1];
  return (Rmax > Rmin && Rmin > 0.0) ? log(Rmax / Rmin) : 0.0;
}

// STORE: keep R, u2 and the Hill radius per particle for the later passes
// (R_out, u2_out, rh_out); otherwise only the range of R is formed.
template <bool STORE>
__global__ __launch_bounds__(CUT_T) void k_cut_prep(CutIn I, double *__restrict__ R_out, double *__restrict__ u2_out,
                                                    double *__restrict__ rh_out, double *__restrict__ part) {
  __shared__ double sh[2][CUT_T / WAVE];
  double rmin = INFINITY, rmax = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < I.n; i += (int64_t)gridDim.x * blockDim.x) {
    double Rc, u2, rh;
    cut_terms(I, i, Rc, u2, rh);
    if (STORE) {
      rh_out[i] = rh;
      u2_out[i] = u2;
      R_out[i] = Rc;
    }
    rmin = fmin(rmin, Rc);
    rmax = fmax(rmax, Rc);
  }
  rmin = wave_min(rmin);
  rmax = wave_max(rmax);
  const int t = threadIdx.x;
  if ((t & (WAVE - 1)) == 0) {
    sh[0][t / WAVE] = rmin;
    sh[1][t / WAVE] = rmax;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < CUT_T / WAVE; ++w) {
      rmin = fmin(rmin, sh[0][w]);
      rmax = fmax(rmax, sh[1][w]);
    }
    part[2 * blockIdx.x] = fmin(sh[0][0], rmin);
    part[2 * blockIdx.x + 1] = fmax(sh[1][0], rmax);
  }
}

__global__ __launch_bounds__(256) void k_cut_minmax(const double *__restrict__ part, int nb, double *__restrict__ out) {
  __shared__ double sh[2][256 / WAVE];
  const int t = threadIdx.x;
  double lo = INFINITY, hi = -INFINITY;
  for (int b = t; b < nb; b += 256) {
    lo = fmin(lo, part[2 * b]);
    hi = fmax(hi, part[2 * b + 1]);
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  if ((t & (WAVE - 1)) == 0) {
    sh[0][t / WAVE] = lo;
    sh[1][t / WAVE] = hi;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < 256 / WAVE; ++w) {
      lo = fmin(lo, sh[0][w]);
      hi = fmax(hi, sh[1][w]);
    }
    out[0] = lo;
    out[1] = hi;
  }
}

// Per chunk of CUT_CHUNK particles: bin index of each particle and, per bin,
// the chunk's sum of u^2 and member count.  The chunk's bins and u^2 are
// staged in LDS; L = CUT_T / nbins threads share a bin, each summing every
// L-th entry in index order, and the L partials are added in order: a fixed
// reduction order, so the result does not depend on scheduling.
// STORE: R and u2 come from the prep pass, and the bins are kept for the
// last pass; otherwise R and u2 are recomputed here and nothing is kept.
template <bool STORE>
__global__ __launch_bounds__(CUT_T) void k_cut_bins(CutIn I, const double *__restrict__ R,
                                                    const double *__restrict__ u2, const double *__restrict__ mm,
                                                    int nbins, int32_t *__restrict__ bin_out,
                                                    double *__restrict__ psum, double *__restrict__ pcnt) {
  __shared__ int sb[CUT_CHUNK];
  __shared__ double su[CUT_CHUNK];
  __shared__ double ps[CUT_T], pc[CUT_T];
  const int t = threadIdx.x;
  const int64_t n = I.n;
  const int64_t base = (int64_t)blockIdx.x * CUT_CHUNK;
  const double Rmin = mm[0];
  const double lspan = cut_lspan(mm);
#pragma unroll
  for (int q = 0; q < CUT_PER; ++q) {
    const int j = q * CUT_T + t;
    const int64_t i = base + j;
    int bb = -1;
    double u = 0.0;
    if (i < n) {
      double Ri;
      if (STORE) {
        Ri = R[i];
        u = u2[i];
      } else {
        double rh;
        cut_terms(I, i, Ri, u, rh);
      }
      bb = cut_bin(Ri, Rmin, lspan, nbins);
      if (STORE) bin_out[i] = bb;
    }
    sb[j] = bb;
    su[j] = u;
  }
  __syncthreads();
  const int L = nbins >= CUT_T ? 1 : CUT_T / nbins;  // threads per bin
  const int k = t / L, part = t - k * L;
  double s = 0.0, c = 0.0;
  if (k < nbins) {
    for (int j = part; j < CUT_CHUNK; j += L) {
      if (sb[j] == k) {
        s += su[j];
        c += 1.0;
      }
    }
  }
  ps[t] = s;
  pc[t] = c;
  __syncthreads();
  for (int kk = t; kk < nbins; kk += CUT_T) {
    double ts = 0.0, tc = 0.0;
    if (nbins <= CUT_T) {
      for (int p = 0; p < L; ++p) {
        ts += ps[kk * L + p];
        tc += pc[kk * L + p];
      }
    }
    psum[(int64_t)kk * gridDim.x + blockIdx.x] = ts;  // [bin][chunk]
    pcnt[(int64_t)kk * gridDim.x + blockIdx.x] = tc;
  }
}

// One block per bin: the bin's chunk partials in a fixed reduction order.
__global__ __launch_bounds__(256) void k_cut_binsum(const double *__restrict__ psum, const double *__restrict__ pcnt,
                                                    int nblk, double *__restrict__ bsum, double *__restrict__ bcnt) {
  __shared__ double shs[256 / WAVE], shc[256 / WAVE];
  const int k = blockIdx.x, t = threadIdx.x;
  double s = 0.0, c = 0.0;
  for (int b = t; b < nblk; b += 256) {
    s += psum[(int64_t)k * nblk + b];
    c += pcnt[(int64_t)k * nblk + b];
  }
  s = wave_sum(s);
  c = wave_sum(c);
  if ((t & (WAVE - 1)) == 0) {
    shs[t / WAVE] = s;
    shc[t / WAVE] = c;
  }
  __syncthreads();
  if (t == 0) {
    double ts = 0.0, tc = 0.0;
    for (int w = 0; w < 256 / WAVE; ++w) {
      ts += shs[w];
      tc += shc[w];
    }
    bsum[k] = ts;
    bcnt[k] = tc;
  }
}

// rms per bin, and the rms over all particles for sparse bins.
__global__ void k_cut_binfinal(const double *__restrict__ bsum, const double *__restrict__ bcnt, int nbins,
                               int min_count, double *__restrict__ vr_bin) {
  __shared__ double ssum[CUT_MAX_BINS], scnt[CUT_MAX_BINS];
  __shared__ double vglob;
  const int k = threadIdx.x;
  if (k < nbins) {
    ssum[k] = bsum[k];
    scnt[k] = bcnt[k];
  }
  __syncthreads();
  if (k == 0) {
    double s = 0.0, c = 0.0;
    for (int q = 0; q < nbins; ++q) {
      s += ssum[q];
      c += scnt[q];
    }
    vglob = c > 0.0 ? sqrt(s / c) : 0.0;
  }
  __syncthreads();
  if (k < nbins) vr_bin[k] = scnt[k] >= (double)min_count ? sqrt(ssum[k] / scnt[k]) : vglob;
}

// STORE: bins and Hill radii from the earlier passes; otherwise recomputed.
template <bool STORE>
__global__ void k_cut_out(CutIn I, const int32_t *__restrict__ bin, const double *__restrict__ rh_in,
                          const double *__restrict__ mm, int nbins, const double *__restrict__ vr_bin, double rc0,
                          double rc1, double rs0, double rs1, double dt, double *__restrict__ r_out,
                          double *__restrict__ r_search, double *__restrict__ v_ran) {
  const double Rmin = mm[0], lspan = cut_lspan(mm);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < I.n; i += (int64_t)gridDim.x * blockDim.x) {
    int b;
    double rh;
    if (STORE) {
      b = bin[i];
      rh = rh_in[i];
    } else {
      double Rc, u2;
      cut_terms(I, i, Rc, u2, rh);
      b = cut_bin(Rc, Rmin, lspan, nbins);
    }
    const double vr = vr_bin[b];
    const double ro = fmax(rc0 * rh, rc1 * vr * dt);
    r_out[i] = ro;
    r_search[i] = rs0 * ro + rs1 * vr * dt;
    if (v_ran) v_ran[i] = vr;
  }
}

// shared cut-off (eq. (rout1)): r_out,i = max_k r_out,k for every particle
__global__ __launch_bounds__(256) void k_max_part(const double *__restrict__ v, int64_t n, double *__restrict__ part) {
  __shared__ double sh[256 / WAVE];
  double mx = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    mx = fmax(mx, v[i]);
  mx = wave_max(mx);
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 256 / WAVE; ++w) mx = fmax(mx, sh[w]);
    part[blockIdx.x] = fmax(mx, sh[0]);
  }
}

__global__ void k_max_final(const double *__restrict__ part, int nb, double *__restrict__ out) {
  if (threadIdx.x == 0) {
    double mx = part[0];
    for (int b = 1; b < nb; ++b) mx = fmax(mx, part[b]);
    *out = mx;
  }
}

__global__ void k_cut_shared(int64_t n, const double *__restrict__ mx, double *__restrict__ r_out,
                             double *__restrict__ r_search) {
  const double ro = mx[0], rs = mx[1];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    r_out[i] = ro;
    r_search[i] = rs;
  }
}

// The passes on stream s.  tmp (3n doubles) and bin (n int32) hold the
// per-particle terms between passes; with tmp == nullptr they are recomputed
// in each pass instead (the allocation-free entry point), with the same
// result.  part: cut_part_need(n) doubles, nothing in it needs clearing.
hipError_t cutoffs_run(const p3t_params &P, int64_t n, const double *pos3, const double *vel3, const double *mass,
                       double *r_out, double *r_search, double *v_ran, double *tmp, int32_t *bin, double *part,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const bool store = tmp != nullptr;
  double *R = store ? tmp : nullptr, *u2 = store ? tmp + n : nullptr, *rh = store ? tmp + 2 * n : nullptr;
  double *mm = part + 2048;  // [0, 2*1024) min/max partials; then the range, the bins
  double *vr_bin = mm + 8;
  double *psum = vr_bin + CUT_MAX_BINS;
  const int nbins = P.vran_bins;
  const int64_t nblk = (n + CUT_CHUNK - 1) / CUT_CHUNK;
  double *pcnt = psum + nblk * nbins;
  const int nb_prep = (int)std::min<int64_t>(1024, (n + CUT_T - 1) / CUT_T);
  CutIn I;
  I.pos = pos3;
  I.vel = vel3;
  I.m = mass;
  I.n = n;
  I.GM = P.G * P.m_star;
  I.m_star = P.m_star;
  I.hill_length = P.hill_length;
  if (store)
    hipLaunchKernelGGL(k_cut_prep<true>, dim3(nb_prep), dim3(CUT_T), 0, s, I, R, u2, rh, part);
  else
    hipLaunchKernelGGL(k_cut_prep<false>, dim3(nb_prep), dim3(CUT_T), 0, s, I, R, u2, rh, part);
  hipLaunchKernelGGL(k_cut_minmax, dim3(1), dim3(256), 0, s, part, nb_prep, mm);
  if (store)
    hipLaunchKernelGGL(k_cut_bins<true>, dim3((unsigned)nblk), dim3(CUT_T), 0, s, I, R, u2, mm, nbins, bin, psum, pcnt);
  else
    hipLaunchKernelGGL(k_cut_bins<false>, dim3((unsigned)nblk), dim3(CUT_T), 0, s, I, R, u2, mm, nbins, bin, psum,
                       pcnt);
  double *bsum = part, *bcnt = part + CUT_MAX_BINS;  // the min/max partials are consumed
  hipLaunchKernelGGL(k_cut_binsum, dim3(nbins), dim3(256), 0, s, psum, pcnt, (int)nblk, bsum, bcnt);
  hipLaunchKernelGGL(k_cut_binfinal, dim3(1), dim3(CUT_MAX_BINS), 0, s, bsum, bcnt, nbins, P.vran_min_count, vr_bin);
  const unsigned g = (unsigned)std::min<int64_t>(65536, (n + 255) / 256);
  if (store)
    hipLaunchKernelGGL(k_cut_out<true>, dim3(g), dim3(256), 0, s, I, bin, rh, mm, nbins, vr_bin, P.r_cut0, P.r_cut1,
                       P.r_search0, P.r_search1, P.dt_soft, r_out, r_search, v_ran);
  else
    hipLaunchKernelGGL(k_cut_out<false>, dim3(g), dim3(256), 0, s, I, bin, rh, mm, nbins, vr_bin, P.r_cut0, P.r_cut1,
                       P.r_search0, P.r_search1, P.dt_soft, r_out, r_search, v_ran);
  if (P.cutoff_mode == 1) {
    // shared cut-off (eq. (rout1)) and shared search radius (Section 2.3):
    // every particle takes the maxima over all particles
    const int nbm = (int)std::min<int64_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_max_part, dim3(nbm), dim3(256), 0, s, r_out, n, part);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(64), 0, s, part, nbm, mm + 2);
    hipLaunchKernelGGL(k_max_part, dim3(nbm), dim3(256), 0, s, r_search, n, part);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(64), 0, s, part, nbm, mm + 3);
    hipLaunchKernelGGL(k_cut_shared, dim3(g), dim3(256), 0, s, n, mm + 2, r_out, r_search);
  }
  return hipGetLastError();
}

hipError_t compute_cutoffs(p3t_ctx *c, int64_t n, const double *pos3, const double *vel3, const double *mass,
                           double *r_out, double *r_search, double *v_ran) {
  return cutoffs_run(c->P, n, pos3, vel3, mass, r_out, r_search, v_ran, c->tmp_d, c->cut_bin, c->cut_part, c->stream);
}

int64_t cut_part_need(int64_t n_cap) {
  const int64_t nblk = (n_cap + CUT_CHUNK - 1) / CUT_CHUNK;
  return 2048 + 8 + CUT_MAX_BINS + 2 * nblk * CUT_MAX_BINS + 64;
}

}  // namespace p3t

// ---------------------------------------------------------------- allocation-free entry point
// p3t_compute_cutoffs_noalloc keeps its scratch (the range partials, the
// per-chunk bin sums, the bin values) in this array instead of a context's
// memory: every GPU the library runs on holds one copy until the process
// ends.  In host code `scratch` only names the symbol; its device address is
// looked up per device with hipGetSymbolAddress and used from then on.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(8) << 20;  // 8 MiB per GPU
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};  // device address of `scratch` per device
thread_local std::string g_noalloc_error;

p3t_status noalloc_fail(p3t_status st, const char *msg) {
  g_noalloc_error = msg;
  return st;
}

// The device address of `scratch` on the current device (looked up once).
hipError_t scratch_ptr(int dev, double **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

namespace p3t {
const char *noalloc_last_error() { return g_noalloc_error.c_str(); }
}  // namespace p3t

extern "C" p3t_status p3t_compute_cutoffs_noalloc(const p3t_params *p_host, int64_t n, const double *pos3,
                                                  const double *vel3, const double *mass, double *r_out,
                                                  double *r_search, double *v_ran, void *hip_stream) {
  using namespace p3t;
  if (!p_host) return noalloc_fail(P3T_ERR_ARG, "compute_cutoffs_noalloc: null parameters");
  const char *why = params_error(*p_host);
  if (why) return noalloc_fail(P3T_ERR_ARG, why);
  if (n < 0 || n > (int64_t(1) << 30)) return noalloc_fail(P3T_ERR_ARG, "compute_cutoffs_noalloc: n out of range");
  if (bad_ptr(pos3, n) || bad_ptr(vel3, n) || bad_ptr(mass, n) || bad_ptr(r_out, n) || bad_ptr(r_search, n))
    return noalloc_fail(P3T_ERR_ARG, "compute_cutoffs_noalloc: null pointer");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return noalloc_fail(P3T_ERR_HIP, "compute_cutoffs_noalloc: no usable current device");
  double *part = nullptr;
  hipError_t e = scratch_ptr(dev, &part);
  if (e != hipSuccess) {
    char buf[256];
    snprintf(buf, sizeof(buf), "compute_cutoffs_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    return noalloc_fail(P3T_ERR_HIP, buf);
  }
  if (n == 0) return P3T_OK;
  // doubles the passes use: range partials, range, bin values, per-chunk bin sums and counts
  const int64_t nblk = (n + CUT_CHUNK - 1) / CUT_CHUNK;
  const int64_t need = 2048 + 8 + CUT_MAX_BINS + 2 * nblk * (int64_t)p_host->vran_bins;
  if (need * (int64_t)sizeof(double) > (int64_t)NOALLOC_SCRATCH_BYTES) {
    char buf[256];
    snprintf(buf, sizeof(buf),
             "compute_cutoffs_noalloc: n = %lld with %d bins needs %lld bytes of scratch, above its %zu",
             (long long)n, p_host->vran_bins, (long long)(need * (int64_t)sizeof(double)), NOALLOC_SCRATCH_BYTES);
    return noalloc_fail(P3T_ERR_CAPACITY, buf);
  }
  e = cutoffs_run(*p_host, n, pos3, vel3, mass, r_out, r_search, v_ran, nullptr, nullptr, part,
                  (hipStream_t)hip_stream);
  if (e != hipSuccess) {
    char buf[256];
    snprintf(buf, sizeof(buf), "compute_cutoffs_noalloc: launch: %s", hipGetErrorString(e));
    return noalloc_fail(P3T_ERR_HIP, buf);
  }
  return P3T_OK;
}

