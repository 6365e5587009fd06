// adjoint.hip -- vector-Jacobian product of the soft kick v' = v + h a(x, m)
// (eq. (HamiltonSol) with the soft force of eq. (softforce)) over the current
// tree, its interaction lists and the pair cut-offs r_out,ij held fixed.
//
// With a_i = sum_{j in P(i)} m_j phi(r_ij) d_ij + sum_{c in C(i)} M_c phi_1(r_ic) e_ic,
//   d_ij = x_j - x_i, e_ic = X_c - x_i, phi = G K(r / R_ij) / r^3, phi_1 = G / r^3,
// and the cotangent lambda of v', the loss L = sum_i lambda_i . a_i has, per
// list entry (i, j) with T_ij = m_j phi lambda_i . d_ij,
//   dT/dx_j = -dT/dx_i = m_j [ phi lambda_i + (phi'/r) (lambda_i . d) d ] =: g_ij,
//   dT/dm_j = phi lambda_i . d,
//   phi'/r = G [ K_y / (R r^4) - 3 K / r^5 ],
// and the same for a monopole cell with (X_c, M_c) in place of (x_j, m_j),
// K = 1.  A cell's centre of mass and mass depend on its members k:
//   dX_c/dx_k = m_k / M_c,  dX_c/dm_k = (x_k - X_c) / M_c,  dM_c/dm_k = 1,
// so the cell adjoints (dL/dX_c, dL/dM_c) are pushed down to every member.
//
// Kernels (one wavefront per group, i-particles in lanes as in the force):
//   pass A: lane = i, loop over the tile's j / cells: the i-side terms -g_ij
//     accumulate in registers and are written once per i;
//   pass B: lane = tile entry j (or cell), loop over the group's i (staged in
//     LDS): the j-side terms accumulate in registers and go to memory with one
//     atomic add per (group, j) and component.
// Then per node A_c = dL/dX_c / M_c, B_c = dL/dM_c - X_c . A_c, and per
// particle the sums of A and B over its ancestors:
//   dL/dx_k += m_k sum A,  dL/dm_k += sum B + x_k . sum A.
// Mixed precision (precision = 1, as the forward force): the K = 1 terms
// (far particles and cells) are evaluated in FP32 from offsets d formed in
// FP64 and the cotangent rounded to FP32; every sum stays FP64.  The
// changeover terms (near particles) are FP64 in both modes.
#include "p3t_internal.h"

namespace p3t {

namespace {

struct AdjArgs {
  const double *sx, *sy, *sz, *sm, *sinv;
  const int32_t *sid;
  const WalkNode *wn;
  const CellMom *cm;
  const GroupList *gl;
  const int32_t *order;
  const int32_t *pool;
  const int32_t *parent;
  DevCounters *cnt;
  const double *lam;  // cotangent in sorted order (3n)
  double *own;        // i-side terms, sorted order (3n), written once per particle
  double *gx;         // j-side terms, sorted order (3n), atomic
  double *gm;         // mass terms, sorted order (n), atomic
  double *cx;         // cell adjoints dL/dX_c (3 n_nodes), atomic
  double *cmass;      // cell adjoints dL/dM_c (n_nodes), atomic
  int64_t n;
  int n_nodes;
  double G, gamma, inv1mg;
  unsigned long long *queue;
};

// g_ij and phi lambda . d for one entry; invR < 0 selects K = 1
__device__ __forceinline__ void adj_term(double dx, double dy, double dz, double lx, double ly, double lz, double mj,
                                         double invR, const AdjArgs &A, double &gx, double &gy, double &gz,
                                         double &s) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double rinv = rsqrt(r2);
  const double rinv2 = rinv * rinv;
  double K = 1.0, Ky = 0.0;
  if (invR >= 0.0) {
    const double y = r2 * rinv * invR;
    const double x = fmin(fmax((y - A.gamma) * A.inv1mg, 0.0), 1.0);
    const double x2 = x * x, omx = 1.0 - x;
    K = x2 * x2 * (35.0 + x * (-84.0 + x * (70.0 - 20.0 * x)));
    Ky = 140.0 * x2 * x * omx * omx * omx * A.inv1mg;
  }
  const double phi = A.G * K * rinv * rinv2;
  const double dphi_r = A.G * rinv2 * rinv2 * (Ky * invR - 3.0 * K * rinv);  // phi'(r) / r
  const double ld = lx * dx + ly * dy + lz * dz;
  const double c = dphi_r * ld;
  gx = mj * (phi * lx + c * dx);
  gy = mj * (phi * ly + c * dy);
  gz = mj * (phi * lz + c * dz);
  s = phi * ld;
}

// the K = 1 term in FP32: g = m (phi lambda + (phi'/r)(lambda . d) d),
// phi = G / r^3, phi'/r = -3 G / r^5
__device__ __forceinline__ void adj_term_f32(double dx, double dy, double dz, double lx, double ly, double lz,
                                             double mj, float G, double &gx, double &gy, double &gz, double &s) {
  const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
  const float flx = (float)lx, fly = (float)ly, flz = (float)lz;
  const float r2 = fx * fx + fy * fy + fz * fz;
  const float rinv = rsqrtf(r2);
  const float rinv2 = rinv * rinv;
  const float phi = G * rinv * rinv2;
  const float dphi_r = -3.0f * phi * rinv2;
  const float ld = flx * fx + fly * fy + flz * fz;
  const float c = dphi_r * ld;
  const float m = (float)mj;
  gx = (double)(m * (phi * flx + c * fx));
  gy = (double)(m * (phi * fly + c * fy));
  gz = (double)(m * (phi * flz + c * fz));
  s = (double)(phi * ld);
}

// one K = 1 term in the path's precision
template <bool MIXED>
__device__ __forceinline__ void adj_far(double dx, double dy, double dz, double lx, double ly, double lz, double mj,
                                        const AdjArgs &A, double &gx, double &gy, double &gz, double &s) {
  if (MIXED)
    adj_term_f32(dx, dy, dz, lx, ly, lz, mj, (float)A.G, gx, gy, gz, s);
  else
    adj_term(dx, dy, dz, lx, ly, lz, mj, -1.0, A, gx, gy, gz, s);
}

__global__ void k_adj_prep(AdjArgs A, const double *__restrict__ lam_v3) {
  const int64_t n = A.n;
  double *lam = const_cast<double *>(A.lam);
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = A.sid[k];
    lam[k] = lam_v3[o];
    lam[n + k] = lam_v3[n + o];
    lam[2 * n + k] = lam_v3[2 * n + o];
    A.gx[k] = A.gx[n + k] = A.gx[2 * n + k] = 0.0;
    A.gm[k] = 0.0;
  }
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < A.n_nodes;
       c += (int64_t)gridDim.x * blockDim.x) {
    A.cx[c] = A.cx[A.n_nodes + c] = A.cx[2 * (int64_t)A.n_nodes + c] = 0.0;
    A.cmass[c] = 0.0;
  }
}

struct AdjLds {
  // the group's i-particles (pass B)
  double ix[2 * WAVE], iy[2 * WAVE], iz[2 * WAVE], ilx[2 * WAVE], ily[2 * WAVE], ilz[2 * WAVE], iinv[2 * WAVE];
  int iid[2 * WAVE];
  // one tile of j-particles or cells
  double jx[WAVE], jy[WAVE], jz[WAVE], jm[WAVE], jinv[WAVE];
  int jid[WAVE];
};

// one tile of particles (near: K from the pair cut-off; far: K = 1)
template <int IPL, bool MIXED>
__device__ __forceinline__ void adj_tile(const AdjArgs &A, AdjLds &S, const int32_t *L, int t0, int nt, bool near,
                                         int gcount, int lane, const int *ii, const double *xi, const double *yi,
                                         const double *zi, const double *lxi, const double *lyi, const double *lzi,
                                         const double *invi, double *ox, double *oy, double *oz) {
  __syncthreads();
  if (lane < nt) {
    const int j = L[t0 + lane];
    S.jx[lane] = A.sx[j];
    S.jy[lane] = A.sy[j];
    S.jz[lane] = A.sz[j];
    S.jm[lane] = A.sm[j];
    S.jinv[lane] = A.sinv[j];
    S.jid[lane] = j;
  }
  __syncthreads();
  // pass A: i in lanes
  for (int jj = 0; jj < nt; ++jj) {
    const double x = S.jx[jj], y = S.jy[jj], z = S.jz[jj], m = S.jm[jj], inv = S.jinv[jj];
    const int jid = S.jid[jj];
#pragma unroll
    for (int s = 0; s < IPL; ++s) {
      const bool ok = ii[s] >= 0 && ii[s] != jid;
      const double dx = ok ? x - xi[s] : 1.0, dy = ok ? y - yi[s] : 0.0, dz = ok ? z - zi[s] : 0.0;
      double gx, gy, gz, sc;
      if (near)
        adj_term(dx, dy, dz, lxi[s], lyi[s], lzi[s], m, fmin(invi[s], inv), A, gx, gy, gz, sc);
      else
        adj_far<MIXED>(dx, dy, dz, lxi[s], lyi[s], lzi[s], m, A, gx, gy, gz, sc);
      if (ok) {
        ox[s] -= gx;
        oy[s] -= gy;
        oz[s] -= gz;
      }
    }
  }
  // pass B: j in lanes, loop over the group's i
  if (lane < nt) {
    const double x = S.jx[lane], y = S.jy[lane], z = S.jz[lane], m = S.jm[lane], inv = S.jinv[lane];
    const int jid = S.jid[lane];
    double ax = 0.0, ay = 0.0, az = 0.0, am = 0.0;
    for (int q = 0; q < gcount; ++q) {
      if (S.iid[q] == jid) continue;
      double gx, gy, gz, sc;
      if (near)
        adj_term(x - S.ix[q], y - S.iy[q], z - S.iz[q], S.ilx[q], S.ily[q], S.ilz[q], m, fmin(S.iinv[q], inv), A, gx,
                 gy, gz, sc);
      else
        adj_far<MIXED>(x - S.ix[q], y - S.iy[q], z - S.iz[q], S.ilx[q], S.ily[q], S.ilz[q], m, A, gx, gy, gz, sc);
      ax += gx;
      ay += gy;
      az += gz;
      am += sc;
    }
    unsafeAtomicAdd(&A.gx[jid], ax);
    unsafeAtomicAdd(&A.gx[A.n + jid], ay);
    unsafeAtomicAdd(&A.gx[2 * A.n + jid], az);
    unsafeAtomicAdd(&A.gm[jid], am);
  }
}

template <int IPL, bool MIXED>
__device__ __forceinline__ void adj_group(const AdjArgs &A, AdjLds &S, int gi, int lane) {
  const int q = uniform_first(A.order ? A.order[gi] : gi);
  const GroupList Lh = A.gl[q];
  const long long off = uniform_first64(Lh.off);
  const int n_cell = uniform_first(Lh.n_cell), n_near = uniform_first(Lh.n_near), n_far = uniform_first(Lh.n_far);
  const int node = uniform_first(Lh.node);
  const int first = uniform_first(A.wn[node].first), gcount = uniform_first(A.wn[node].count);
  const int64_t n = A.n;
  int ii[IPL];
  double xi[IPL], yi[IPL], zi[IPL], lxi[IPL], lyi[IPL], lzi[IPL], invi[IPL], ox[IPL], oy[IPL], oz[IPL];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < IPL; ++s) {
    const int k = lane + WAVE * s;
    ii[s] = k < gcount ? first + k : -1;
    const int i = ii[s] >= 0 ? ii[s] : first;
    xi[s] = A.sx[i];
    yi[s] = A.sy[i];
    zi[s] = A.sz[i];
    lxi[s] = A.lam[i];
    lyi[s] = A.lam[n + i];
    lzi[s] = A.lam[2 * n + i];
    invi[s] = A.sinv[i];
    ox[s] = oy[s] = oz[s] = 0.0;
    if (k < gcount) {
      S.ix[k] = xi[s];
      S.iy[k] = yi[s];
      S.iz[k] = zi[s];
      S.ilx[k] = lxi[s];
      S.ily[k] = lyi[s];
      S.ilz[k] = lzi[s];
      S.iinv[k] = invi[s];
      S.iid[k] = ii[s];
    }
  }
  const int32_t *Ln = A.pool + off + n_cell;
  for (int t0 = 0; t0 < n_near; t0 += WAVE)
    adj_tile<IPL, MIXED>(A, S, Ln, t0, min(WAVE, n_near - t0), true, gcount, lane, ii, xi, yi, zi, lxi, lyi, lzi, invi, ox,
                  oy, oz);
  const int32_t *Lf = Ln + n_near;
  for (int t0 = 0; t0 < n_far; t0 += WAVE)
    adj_tile<IPL, MIXED>(A, S, Lf, t0, min(WAVE, n_far - t0), false, gcount, lane, ii, xi, yi, zi, lxi, lyi, lzi, invi, ox,
                  oy, oz);
  // monopole cells
  const int32_t *Lc = A.pool + off;
  for (int t0 = 0; t0 < n_cell; t0 += WAVE) {
    const int nt = min(WAVE, n_cell - t0);
    __syncthreads();
    if (lane < nt) {
      const int c = Lc[t0 + lane];
      const CellMom cm = A.cm[c];
      S.jx[lane] = cm.com[0];
      S.jy[lane] = cm.com[1];
      S.jz[lane] = cm.com[2];
      S.jm[lane] = cm.mass;
      S.jid[lane] = c;
    }
    __syncthreads();
    for (int jj = 0; jj < nt; ++jj) {
      const double x = S.jx[jj], y = S.jy[jj], z = S.jz[jj], m = S.jm[jj];
#pragma unroll
      for (int s = 0; s < IPL; ++s) {
        double gx, gy, gz, sc;
        adj_far<MIXED>(x - xi[s], y - yi[s], z - zi[s], lxi[s], lyi[s], lzi[s], m, A, gx, gy, gz, sc);
        if (ii[s] >= 0) {
          ox[s] -= gx;
          oy[s] -= gy;
          oz[s] -= gz;
        }
      }
    }
    if (lane < nt) {
      const double x = S.jx[lane], y = S.jy[lane], z = S.jz[lane], m = S.jm[lane];
      const int c = S.jid[lane];
      double ax = 0.0, ay = 0.0, az = 0.0, am = 0.0;
      for (int q2 = 0; q2 < gcount; ++q2) {
        double gx, gy, gz, sc;
        adj_far<MIXED>(x - S.ix[q2], y - S.iy[q2], z - S.iz[q2], S.ilx[q2], S.ily[q2], S.ilz[q2], m, A, gx, gy, gz,
                       sc);
        ax += gx;
        ay += gy;
        az += gz;
        am += sc;
      }
      const int64_t nn = A.n_nodes;
      unsafeAtomicAdd(&A.cx[c], ax);
      unsafeAtomicAdd(&A.cx[nn + c], ay);
      unsafeAtomicAdd(&A.cx[2 * nn + c], az);
      unsafeAtomicAdd(&A.cmass[c], am);
    }
  }
#pragma unroll
  for (int s = 0; s < IPL; ++s) {
    if (ii[s] >= 0) {
      A.own[ii[s]] = ox[s];
      A.own[n + ii[s]] = oy[s];
      A.own[2 * n + ii[s]] = oz[s];
    }
  }
}

template <bool MIXED>
__global__ __launch_bounds__(WAVE) void k_adj_groups(AdjArgs A) {
  __shared__ AdjLds S;
  const int lane = threadIdx.x;
  const int ngroups = uniform_first((int)A.cnt->n_groups);
  for (;;) {
    const int gi = (int)wave_fetch_add(A.queue, 1ull);
    if (gi >= ngroups) break;
    const int q = uniform_first(A.order ? A.order[gi] : gi);
    if (uniform_first64(A.gl[q].off) < 0) continue;
    const int cnt = uniform_first(A.wn[uniform_first(A.gl[q].node)].count);
    if (cnt > WAVE)
      adj_group<2, MIXED>(A, S, gi, lane);
    else
      adj_group<1, MIXED>(A, S, gi, lane);
  }
}

// A_c = dL/dX_c / M_c, B_c = dL/dM_c - X_c . A_c (in place)
__global__ void k_adj_cell_coeffs(AdjArgs A) {
  const int64_t nn = A.n_nodes;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nn; c += (int64_t)gridDim.x * blockDim.x) {
    const double ax = A.cx[c], ay = A.cx[nn + c], az = A.cx[2 * nn + c];
    if (ax == 0.0 && ay == 0.0 && az == 0.0 && A.cmass[c] == 0.0) continue;  // cell never used
    const double M = A.cm[c].mass;  // (the records of nodes no walk reaches are not written)
    const double iM = 1.0 / M;
    const double px = ax * iM, py = ay * iM, pz = az * iM;
    A.cx[c] = px;
    A.cx[nn + c] = py;
    A.cx[2 * nn + c] = pz;
    A.cmass[c] -= A.cm[c].com[0] * px + A.cm[c].com[1] * py + A.cm[c].com[2] * pz;
  }
}

// per particle: the ancestors' push-down, the three parts summed, scaled by h,
// written in the caller's order
__global__ void k_adj_final(AdjArgs A, double h, double *__restrict__ g_pos3, double *__restrict__ g_mass) {
  const int64_t n = A.n, nn = A.n_nodes;
  const int leaf0 = (int)n - 1;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    double sx = 0.0, sy = 0.0, sz = 0.0, sb = 0.0;
    int node = n > 1 ? A.parent[leaf0 + k] : -1;
    while (node >= 0) {
      sx += A.cx[node];
      sy += A.cx[nn + node];
      sz += A.cx[2 * nn + node];
      sb += A.cmass[node];
      node = A.parent[node];
    }
    const double m = A.sm[k];
    const double gx = A.own[k] + A.gx[k] + m * sx;
    const double gy = A.own[n + k] + A.gx[n + k] + m * sy;
    const double gz = A.own[2 * n + k] + A.gx[2 * n + k] + m * sz;
    const double gm = A.gm[k] + sb + A.sx[k] * sx + A.sy[k] * sy + A.sz[k] * sz;
    const int64_t o = A.sid[k];
    g_pos3[o] = h * gx;
    g_pos3[n + o] = h * gy;
    g_pos3[2 * n + o] = h * gz;
    g_mass[o] = h * gm;
  }
}

__global__ void k_adj_reset(unsigned long long *q) { *q = 0ull; }

}  // namespace

hipError_t soft_kick_adjoint(p3t_ctx *c, double h, const double *lam_v3, double *g_pos3, double *g_mass) {
  const hipStream_t s = c->stream;
  const int64_t n = c->n;
  AdjArgs A;
  A.sx = c->sx;
  A.sy = c->sy;
  A.sz = c->sz;
  A.sm = c->sm;
  A.sinv = c->sinv;
  A.sid = c->sid;
  A.wn = c->wnode;
  A.cm = c->cmom;
  A.gl = c->glist;
  A.order = c->group_order;
  A.pool = c->pool;
  A.parent = c->parent;
  A.cnt = c->cnt;
  A.lam = c->adj_buf;
  A.own = c->adj_buf + 3 * n;
  A.gx = c->adj_buf + 6 * n;
  A.gm = c->adj_buf + 9 * n;
  A.n_nodes = (int)(n > 0 ? 2 * n - 1 : 0);
  A.cx = c->adj_buf + 10 * n;
  A.cmass = A.cx + 3 * (int64_t)A.n_nodes;
  A.n = n;
  A.G = c->P.G;
  A.gamma = c->P.gamma;
  A.inv1mg = 1.0 / (1.0 - c->P.gamma);
  A.queue = &c->cnt->queue[0];
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)c->n_cu * 8, (2 * n + 255) / 256));
  hipLaunchKernelGGL(k_adj_prep, dim3(g), dim3(256), 0, s, A, lam_v3);
  hipLaunchKernelGGL(k_adj_reset, dim3(1), dim3(1), 0, s, A.queue);
  if (c->P.precision == 1)
    hipLaunchKernelGGL(k_adj_groups<true>, dim3(c->n_cu * 8), dim3(WAVE), 0, s, A);
  else
    hipLaunchKernelGGL(k_adj_groups<false>, dim3(c->n_cu * 8), dim3(WAVE), 0, s, A);
  hipLaunchKernelGGL(k_adj_cell_coeffs, dim3(g), dim3(256), 0, s, A);
  hipLaunchKernelGGL(k_adj_final, dim3(g), dim3(256), 0, s, A, h, g_pos3, g_mass);
  return hipGetLastError();
}

int64_t adjoint_buf_need(int64_t n_cap) { return 10 * n_cap + 4 * (2 * n_cap); }

}  // namespace p3t
