/*
 * p3t_oracle.c -- CPU reference ("oracle") for the soft-force hot path of the
 * P3T scheme with individual cut-off radii (Ishigaki et al. 2021, GPLUM).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is built into oracle/liboracle.so and
 * is loaded by the test-suite, by the smoke check and by the CPU-baseline leg
 * of the benchmark, nothing else.  It shares no code, header, table or
 * constant with the GPU library; the two never include or link each other.
 *
 * Everything is plain, slow and direct: O(N^2) sums in FP64, no tree, no
 * blocking, no reordering beyond what the definitions state.  Each function
 * names the passage of the paper it follows.  Where the paper is silent or
 * ambiguous the reading taken is stated at the function.
 *
 * Layout conventions: positions/velocities are structure-of-arrays with n
 * entries per row, row 0 = x, row 1 = y, row 2 = z (pointer p, entries
 * p[k*n + i]).  Indices are int64 unless stated.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double G, m_star, gamma;
  double r_cut0, r_cut1;                                  /* eq. (routi2) */
  double r_search0, r_search1, r_search2, r_search3;     /* eq. (rsearch), (rsearch1) */
  double dt_soft;                                         /* soft step */
  double eta, eta0;                                       /* Hermite accuracy parameters */
  int32_t hill_length;    /* 0: a_i = osculating semi-major axis, 1: a_i = |x_i| */
  int32_t vran_bins;      /* number of log-spaced radial bins for v_ran */
  int32_t vran_min_count; /* bins with fewer members use the global rms */
  int32_t k_max;          /* deepest block-step level: dt_soft * 2^-k_max */
  int32_t cutoff_mode;    /* 0: individual radii (eq. (rout2)), 1: shared radii (eq. (rout1)) */
} orc_params;

/* status bits reported by the oracle */
#define ORC_ERR_COINCIDENT 1
#define ORC_ERR_KMAX 2
#define ORC_ERR_NSTEPS 4
#define ORC_ERR_NAN 8

/* ------------------------------------------------------------------------ */
/* Changeover functions, eq. (cutfuncW) and the integral relation between W
 * and K in Section 2.1.1.  W is written out exactly as printed:
 *   W = c y                      (y < gamma)
 *   W = f(y) + (1 - f(1)) y      (gamma <= y < 1)
 *   W = 1                        (y >= 1)
 * with c and f(y; gamma) as printed.  K follows from W(r) = r int_r^inf
 * K(s)/s^2 ds: dividing by r and differentiating gives K = W - y dW/dy.  In
 * the middle branch that is f - y f'.  Evaluated in long double to keep the
 * cancellation between f and y f' well below FP64 rounding.
 * Reading: y = r_ij / r_out,ij (the argument of W is not defined in the text;
 * this is the scaling under which K vanishes below r_in = gamma r_out and is
 * one above r_out). */
static long double orc_c(long double g) {
  long double g2 = g * g, g3 = g2 * g, g4 = g3 * g, g5 = g4 * g, g6 = g5 * g;
  long double gm1 = g - 1.0L;
  long double gm1_7 = gm1 * gm1 * gm1 * gm1 * gm1 * gm1 * gm1;
  return 7.0L * (g6 - 9.0L * g5 + 45.0L * g4 - 60.0L * g3 * logl(g) - 45.0L * g2 + 9.0L * g - 1.0L) /
         (3.0L * gm1_7);
}

static long double orc_f(long double y, long double g) {
  long double g2 = g * g, g3 = g2 * g, g4 = g3 * g, g5 = g4 * g, g6 = g5 * g, g7 = g6 * g;
  long double gm1 = g - 1.0L;
  long double gm1_7 = gm1 * gm1 * gm1 * gm1 * gm1 * gm1 * gm1;
  long double y2 = y * y, y3 = y2 * y, y4 = y3 * y, y5 = y4 * y, y6 = y5 * y, y7 = y6 * y;
  long double num = -10.0L / 3.0L * y7 + 14.0L * (g + 1.0L) * y6 - 21.0L * (g2 + 3.0L * g + 1.0L) * y5 +
                    (35.0L * (g3 + 9.0L * g2 + 9.0L * g + 1.0L) / 3.0L) * y4 -
                    70.0L * (g3 + 3.0L * g2 + g) * y3 + 210.0L * (g3 + g2) * y2 -
                    140.0L * g3 * y * logl(y) + (g7 - 7.0L * g6 + 21.0L * g5 - 35.0L * g4);
  return num / gm1_7;
}

/* f'(y), term by term from f */
static long double orc_fp(long double y, long double g) {
  long double g2 = g * g, g3 = g2 * g;
  long double gm1 = g - 1.0L;
  long double gm1_7 = gm1 * gm1 * gm1 * gm1 * gm1 * gm1 * gm1;
  long double y2 = y * y, y3 = y2 * y, y4 = y3 * y, y5 = y4 * y, y6 = y5 * y;
  long double num = -70.0L / 3.0L * y6 + 84.0L * (g + 1.0L) * y5 - 105.0L * (g2 + 3.0L * g + 1.0L) * y4 +
                    (140.0L * (g3 + 9.0L * g2 + 9.0L * g + 1.0L) / 3.0L) * y3 -
                    210.0L * (g3 + 3.0L * g2 + g) * y2 + 420.0L * (g3 + g2) * y -
                    140.0L * g3 * (logl(y) + 1.0L);
  return num / gm1_7;
}

/* f''(y), term by term from f' */
static long double orc_fpp(long double y, long double g) {
  long double g2 = g * g, g3 = g2 * g;
  long double gm1 = g - 1.0L;
  long double gm1_7 = gm1 * gm1 * gm1 * gm1 * gm1 * gm1 * gm1;
  long double y2 = y * y, y3 = y2 * y, y4 = y3 * y, y5 = y4 * y;
  long double num = -140.0L * y5 + 420.0L * (g + 1.0L) * y4 - 420.0L * (g2 + 3.0L * g + 1.0L) * y3 +
                    140.0L * (g3 + 9.0L * g2 + 9.0L * g + 1.0L) * y2 -
                    420.0L * (g3 + 3.0L * g2 + g) * y + 420.0L * (g3 + g2) - 140.0L * g3 / y;
  return num / gm1_7;
}

/* W(y; gamma), eq. (cutfuncW) */
double orc_W(double y, double gamma) {
  long double g = gamma, yy = y;
  if (yy < g) return (double)(orc_c(g) * yy);
  if (yy < 1.0L) return (double)(orc_f(yy, g) + (1.0L - orc_f(1.0L, g)) * yy);
  return 1.0;
}

/* dW/dy, branch by branch */
double orc_dWdy(double y, double gamma) {
  long double g = gamma, yy = y;
  if (yy < g) return (double)orc_c(g);
  if (yy < 1.0L) return (double)(orc_fp(yy, g) + (1.0L - orc_f(1.0L, g)));
  return 0.0;
}

/* K(y; gamma) = W - y W' (from W(r) = r int_r^inf K/s^2 ds) */
double orc_K(double y, double gamma) {
  long double g = gamma, yy = y;
  if (yy < g) return 0.0; /* c y - y c */
  if (yy < 1.0L) return (double)(orc_f(yy, g) - yy * orc_fp(yy, g));
  return 1.0; /* 1 - y * 0 */
}

/* dK/dy = -y f''(y) in the middle branch, zero outside */
double orc_dKdy(double y, double gamma) {
  long double g = gamma, yy = y;
  if (yy < g || yy >= 1.0L) return 0.0;
  return (double)(-yy * orc_fpp(yy, g));
}

/* ------------------------------------------------------------------------ */
/* Cut-off and search radii: Hill radius (Section 2.1.1), eq. (routi2) and
 * eq. (rsearch).
 *   r_Hill,i  = (m_i / 3 M_*)^(1/3) a_i,   a_i the osculating semi-major axis
 *   r_out,i   = max(Rcut0 r_Hill,i, Rcut1 v_ran,i dt)
 *   r_search,i = Rsearch0 r_out,i + Rsearch1 v_ran,i dt
 * Readings (eq. (routi2) takes v_ran,i as an average random velocity of
 * the particles near particle i, without saying which particles or which
 * average; the random velocity is the departure of a particle's velocity
 * from the Kepler velocity):
 *   - Kepler velocity: circular speed sqrt(G M_* / |x|) along phi-hat =
 *     (-y, x, 0) / sqrt(x^2 + y^2);
 *   - "around the particle": the particle's bin among vran_bins log-spaced
 *     bins in cylindrical radius R over [min R, max R];
 *   - "mean": root mean square of |v - v_K| over the bin; a bin with fewer
 *     than vran_min_count members uses the rms over all particles;
 *   - an unbound particle (2/r - v^2/GM <= 0) uses a_i = |x_i|.
 * Shared cut-off (cutoff_mode = 1): eq. (rout1) gives every interaction the
 * largest cut-off radius of all particles, and Section 2.3 gives every pair
 * the largest search radius of all particles; both maxima are taken over
 * the individual radii above and stored for every particle.
 * Outputs r_out, r_search and v_ran per particle.  Returns 0. */
int orc_cutoffs(int64_t n, const double *pos, const double *vel, const double *m, const orc_params *p,
                double *r_out, double *r_search, double *v_ran) {
  if (n <= 0) return 0;
  const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
  const double *VX = vel, *VY = vel + n, *VZ = vel + 2 * n;
  double *R = (double *)malloc(sizeof(double) * n);
  double *u2 = (double *)malloc(sizeof(double) * n);
  double *rh = (double *)malloc(sizeof(double) * n);
  int nb = p->vran_bins > 0 ? p->vran_bins : 1;
  double *bsum = (double *)calloc(nb, sizeof(double));
  int64_t *bcnt = (int64_t *)calloc(nb, sizeof(int64_t));
  int32_t *bin = (int32_t *)malloc(sizeof(int32_t) * n);
  double GM = p->G * p->m_star;
  for (int64_t i = 0; i < n; ++i) {
    double x = X[i], y = Y[i], z = Z[i];
    double r = sqrt(x * x + y * y + z * z);
    double Rc = sqrt(x * x + y * y);
    double v2 = VX[i] * VX[i] + VY[i] * VY[i] + VZ[i] * VZ[i];
    double a;
    if (p->hill_length == 1) {
      a = r;
    } else {
      double inv_a = 2.0 / r - v2 / GM;
      a = inv_a > 0.0 ? 1.0 / inv_a : r;
    }
    rh[i] = cbrt(m[i] / (3.0 * p->m_star)) * a;
    double vk = sqrt(GM / r);
    double phx = Rc > 0.0 ? -y / Rc : 0.0;
    double phy = Rc > 0.0 ? x / Rc : 0.0;
    double ux = VX[i] - vk * phx, uy = VY[i] - vk * phy, uz = VZ[i];
    u2[i] = ux * ux + uy * uy + uz * uz;
    R[i] = Rc;
  }
  double Rmin = R[0], Rmax = R[0];
  for (int64_t i = 1; i < n; ++i) {
    if (R[i] < Rmin) Rmin = R[i];
    if (R[i] > Rmax) Rmax = R[i];
  }
  double lspan = (Rmax > Rmin && Rmin > 0.0) ? log(Rmax / Rmin) : 0.0;
  double gsum = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    int b = 0;
    if (lspan > 0.0) {
      double t = floor((double)nb * (log(R[i] / Rmin) / lspan));
      b = t < 0.0 ? 0 : (t > (double)(nb - 1) ? nb - 1 : (int)t);
    }
    bin[i] = b;
    bsum[b] += u2[i];
    bcnt[b] += 1;
    gsum += u2[i];
  }
  double vglob = sqrt(gsum / (double)n);
  for (int64_t i = 0; i < n; ++i) {
    int b = bin[i];
    double vr = bcnt[b] >= p->vran_min_count ? sqrt(bsum[b] / (double)bcnt[b]) : vglob;
    double ro = fmax(p->r_cut0 * rh[i], p->r_cut1 * vr * p->dt_soft);
    r_out[i] = ro;
    r_search[i] = p->r_search0 * ro + p->r_search1 * vr * p->dt_soft;
    if (v_ran) v_ran[i] = vr;
  }
  if (p->cutoff_mode == 1) {
    double ro_max = r_out[0], rs_max = r_search[0];
    for (int64_t i = 1; i < n; ++i) {
      if (r_out[i] > ro_max) ro_max = r_out[i];
      if (r_search[i] > rs_max) rs_max = r_search[i];
    }
    for (int64_t i = 0; i < n; ++i) {
      r_out[i] = ro_max;
      r_search[i] = rs_max;
    }
  }
  free(R); free(u2); free(rh); free(bsum); free(bcnt); free(bin);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Soft acceleration, eq. (softforce) divided by m_i, with the individual
 * pair cut-off of eq. (rout2):
 *   a_i = sum_{j != i} G m_j K(r_ij / r_out,ij) (x_j - x_i) / r_ij^3,
 *   r_out,ij = max(r_out,i, r_out,j).
 * Direct O(N^2) sum over all j for each i in idx[0..ni).  acc is (3, ni).
 * A coincident pair (r = 0, j != i) sets ORC_ERR_COINCIDENT and is skipped. */
int orc_soft_acc(int64_t n, const double *pos, const double *m, const double *r_out, double G, double gamma,
                 int64_t ni, const int64_t *idx, double *acc) {
  const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
  int err = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : err)
  for (int64_t k = 0; k < ni; ++k) {
    int64_t i = idx[k];
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
      double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 == 0.0) { err |= ORC_ERR_COINCIDENT; continue; }
      double r = sqrt(r2);
      double R = fmax(r_out[i], r_out[j]);
      double K = orc_K(r / R, gamma);
      double f = G * m[j] * K / (r2 * r);
      ax += f * dx; ay += f * dy; az += f * dz;
    }
    acc[k] = ax; acc[ni + k] = ay; acc[2 * ni + k] = az;
  }
  return err;
}

/* Plain Newtonian pair acceleration sum (no changeover), the special case
 * that eq. (softforce) + eq. (hardforce) add up to; used by the identity
 * tests only. */
int orc_newton_acc(int64_t n, const double *pos, const double *m, double G, int64_t ni, const int64_t *idx,
                   double *acc) {
  const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < ni; ++k) {
    int64_t i = idx[k];
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
      double r2 = dx * dx + dy * dy + dz * dz;
      double r = sqrt(r2);
      double f = G * m[j] / (r2 * r);
      ax += f * dx; ay += f * dy; az += f * dz;
    }
    acc[k] = ax; acc[ni + k] = ay; acc[2 * ni + k] = az;
  }
  return 0;
}

/* Soft potential energy, eq. (soft):
 *   H_soft = - sum_i sum_{j>i} G m_i m_j W(r_ij / r_out,ij) / r_ij. */
double orc_soft_energy(int64_t n, const double *pos, const double *m, const double *r_out, double G,
                       double gamma) {
  const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
  double e = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j) {
      double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      double R = fmax(r_out[i], r_out[j]);
      e -= G * m[i] * m[j] * orc_W(r / R, gamma) / r;
    }
  return e;
}

/* ------------------------------------------------------------------------ */
/* Hard acceleration and jerk, eq. (hardforce) divided by m_i, over a set of
 * nm particles given contiguously (x, v are (3, nm)):
 *   a_i = -G M_* x_i / |x_i|^3 + sum_{j != i} G m_j (1 - K) d / r^3
 * with d = x_j - x_i, r = |d|, y = r / r_out,ij, and the time derivative
 *   jerk_i = -G M_* (v_i / |x_i|^3 - 3 (x_i . v_i) x_i / |x_i|^5)
 *          + sum_j G m_j [ (1 - K)(u / r^3 - 3 s d / r^5) - K'(y) s / (r R) d / r^3 ]
 * with u = v_j - v_i, s = d . u, R = r_out,ij (the last term is dK/dt).
 * Only the particles i in [i0, i1) are evaluated; all nm act as sources. */
static int orc_hard_acc_jerk_range(int64_t nm, const double *x, const double *v, const double *m,
                                   const double *r_out, const orc_params *p, int64_t i0, int64_t i1,
                                   const unsigned char *mask, const int32_t *comp, double *a, double *jk) {
  const double *X = x, *Y = x + nm, *Z = x + 2 * nm;
  const double *VX = v, *VY = v + nm, *VZ = v + 2 * nm;
  double GM = p->G * p->m_star;
  int err = 0;
  for (int64_t i = i0; i < i1; ++i) {
    if (mask && !mask[i]) continue;
    double r2 = X[i] * X[i] + Y[i] * Y[i] + Z[i] * Z[i];
    double r = sqrt(r2);
    double ir3 = 1.0 / (r2 * r);
    double xv = X[i] * VX[i] + Y[i] * VY[i] + Z[i] * VZ[i];
    double ax = -GM * X[i] * ir3, ay = -GM * Y[i] * ir3, az = -GM * Z[i] * ir3;
    double c5 = 3.0 * xv / r2;
    double jx = -GM * (VX[i] - c5 * X[i]) * ir3;
    double jy = -GM * (VY[i] - c5 * Y[i]) * ir3;
    double jz = -GM * (VZ[i] - c5 * Z[i]) * ir3;
    for (int64_t j = 0; j < nm; ++j) {
      if (j == i) continue;
      if (comp && comp[j] == comp[i]) continue; /* the two parts of one merged body */
      double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
      double ux = VX[j] - VX[i], uy = VY[j] - VY[i], uz = VZ[j] - VZ[i];
      double d2 = dx * dx + dy * dy + dz * dz;
      if (d2 == 0.0) { err |= ORC_ERR_COINCIDENT; continue; }
      double d = sqrt(d2);
      double R = fmax(r_out[i], r_out[j]);
      double y = d / R;
      double K = orc_K(y, p->gamma);
      double Ky = orc_dKdy(y, p->gamma);
      double s = dx * ux + dy * uy + dz * uz;
      double id3 = 1.0 / (d2 * d);
      double w = p->G * m[j] * (1.0 - K) * id3;
      ax += w * dx; ay += w * dy; az += w * dz;
      double c1 = 3.0 * s / d2;
      double c2 = p->G * m[j] * Ky * s / (d * R) * id3;
      jx += w * (ux - c1 * dx) - c2 * dx;
      jy += w * (uy - c1 * dy) - c2 * dy;
      jz += w * (uz - c1 * dz) - c2 * dz;
    }
    a[i] = ax; a[nm + i] = ay; a[2 * nm + i] = az;
    jk[i] = jx; jk[nm + i] = jy; jk[2 * nm + i] = jz;
    if (!(isfinite(ax) && isfinite(ay) && isfinite(az))) err |= ORC_ERR_NAN;
  }
  return err;
}

int orc_hard_acc_jerk(int64_t nm, const double *x, const double *v, const double *m, const double *r_out,
                      const orc_params *p, double *a, double *jk) {
  return orc_hard_acc_jerk_range(nm, x, v, m, r_out, p, 0, nm, NULL, NULL, a, jk);
}

/* Hard-part energy of a particle set, eq. (hard):
 *   E = sum_i [ m_i |v_i|^2 / 2 - G M_* m_i / |x_i| ]
 *     - sum_i sum_{j>i} G m_i m_j (1 - W(r_ij / r_out,ij)) / r_ij. */
double orc_cluster_energy(int64_t nm, const double *x, const double *v, const double *m, const double *r_out,
                          const orc_params *p) {
  const double *X = x, *Y = x + nm, *Z = x + 2 * nm;
  const double *VX = v, *VY = v + nm, *VZ = v + 2 * nm;
  double e = 0.0;
  for (int64_t i = 0; i < nm; ++i) {
    double v2 = VX[i] * VX[i] + VY[i] * VY[i] + VZ[i] * VZ[i];
    double r = sqrt(X[i] * X[i] + Y[i] * Y[i] + Z[i] * Z[i]);
    e += 0.5 * m[i] * v2 - p->G * p->m_star * m[i] / r;
  }
  for (int64_t i = 0; i < nm; ++i)
    for (int64_t j = i + 1; j < nm; ++j) {
      double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      double R = fmax(r_out[i], r_out[j]);
      e -= p->G * m[i] * m[j] * (1.0 - orc_W(r / R, p->gamma)) / r;
    }
  return e;
}

/* ------------------------------------------------------------------------ */
/* Fourth-order Hermite integration of one neighbour cluster over one soft
 * step with individual (block) time steps (Section 2.1.1, step (5)(i) of the
 * time-integration procedure in Section 2.2; parameters eta, eta_0 of
 * Section 3.1).
 * Readings (the paper names the scheme but not its details):
 *   - forces: the central star plus every intra-cluster pair with (1 - K),
 *     eq. (hardforce), and the jerk including the dK/dt term;
 *   - steps are dt_soft * 2^-k, 0 <= k <= k_max; time is kept in integer
 *     ticks of dt_soft * 2^-40 so block bookkeeping is exact;
 *   - initial step: eta_0 |a| / |jerk|, quantised down to a block step,
 *     unless the particle carries a hard step from the previous soft step
 *     (the particle data holds "time step for the hard part", Section 2.2;
 *     eta_0 is for the initial step only, Section 3.1), which is used;
 *   - each block step: predict every member to the block time, evaluate the
 *     active members, correct once (predict-evaluate-correct), with the
 *     second and third derivatives from the two-point Hermite interpolation;
 *   - new step from Aarseth's criterion with eta, evaluated with the
 *     derivatives at the end of the step, quantised down; a step may grow by
 *     at most a factor two and only when the current time is a multiple of
 *     the doubled step.
 * The cluster's members are given contiguously (x, v: (3, nm)).  Updated in
 * place.  Returns status bits; *nsteps_out counts block steps. */
#define ORC_TICK_BITS 40

static int orc_level_for(double dt_soft, double dtc, int kmax) {
  int k = 0;
  while (k <= kmax && ldexp(dt_soft, -k) > dtc) ++k;
  return k;
}

static double orc_norm3(double a, double b, double c) { return sqrt(a * a + b * b + c * c); }

int orc_hermite_one(int64_t nm, double *x, double *v, const double *m, const double *r_out,
                    const orc_params *p, double dt_soft, double *dt_hard, int64_t *nsteps_out) {
  int err = 0;
  const int64_t T = (int64_t)1 << ORC_TICK_BITS;
  const double tick = ldexp(dt_soft, -ORC_TICK_BITS);
  size_t s3 = sizeof(double) * 3 * nm;
  double *a0 = (double *)malloc(s3), *j0 = (double *)malloc(s3);
  double *a1 = (double *)malloc(s3), *j1 = (double *)malloc(s3);
  double *xp = (double *)malloc(s3), *vp = (double *)malloc(s3);
  int64_t *t = (int64_t *)calloc(nm, sizeof(int64_t));
  int *lev = (int *)malloc(sizeof(int) * nm);
  unsigned char *act = (unsigned char *)malloc(nm);
  int64_t nsteps = 0;

  err |= orc_hard_acc_jerk_range(nm, x, v, m, r_out, p, 0, nm, NULL, NULL, a0, j0);
  for (int64_t i = 0; i < nm; ++i) {
    double an = orc_norm3(a0[i], a0[nm + i], a0[2 * nm + i]);
    double jn = orc_norm3(j0[i], j0[nm + i], j0[2 * nm + i]);
    double dtc = jn > 0.0 ? p->eta0 * an / jn : dt_soft;
    if (dt_hard && dt_hard[i] > 0.0) dtc = dt_hard[i]; /* step carried from the previous soft step */
    int k = orc_level_for(dt_soft, dtc, p->k_max);
    if (k > p->k_max) { err |= ORC_ERR_KMAX; k = p->k_max; }
    lev[i] = k;
  }
  for (;;) {
    int64_t tn = T;
    for (int64_t i = 0; i < nm; ++i) {
      int64_t te = t[i] + ((int64_t)1 << (ORC_TICK_BITS - lev[i]));
      if (te < tn) tn = te;
    }
    for (int64_t i = 0; i < nm; ++i) act[i] = (t[i] + ((int64_t)1 << (ORC_TICK_BITS - lev[i]))) == tn;
    /* predictor for every member */
    for (int64_t i = 0; i < nm; ++i) {
      double dl = (double)(tn - t[i]) * tick;
      double d2 = dl * dl / 2.0, d3 = dl * dl * dl / 6.0;
      for (int c = 0; c < 3; ++c) {
        int64_t q = c * nm + i;
        xp[q] = x[q] + v[q] * dl + a0[q] * d2 + j0[q] * d3;
        vp[q] = v[q] + a0[q] * dl + j0[q] * d2;
      }
    }
    /* evaluation of the active members from the predicted states */
    err |= orc_hard_acc_jerk_range(nm, xp, vp, m, r_out, p, 0, nm, act, NULL, a1, j1);
    /* corrector and new steps */
    for (int64_t i = 0; i < nm; ++i) {
      if (!act[i]) continue;
      double h = (double)(tn - t[i]) * tick;
      double a2[3], a3[3];
      for (int c = 0; c < 3; ++c) {
        int64_t q = c * nm + i;
        double da = a0[q] - a1[q];
        a2[c] = (-6.0 * da - h * (4.0 * j0[q] + 2.0 * j1[q])) / (h * h);
        a3[c] = (12.0 * da + 6.0 * h * (j0[q] + j1[q])) / (h * h * h);
        x[q] = xp[q] + a2[c] * (h * h * h * h) / 24.0 + a3[c] * (h * h * h * h * h) / 120.0;
        v[q] = vp[q] + a2[c] * (h * h * h) / 6.0 + a3[c] * (h * h * h * h) / 24.0;
        a0[q] = a1[q];
        j0[q] = j1[q];
      }
      t[i] = tn;
      double a2e[3] = {a2[0] + a3[0] * h, a2[1] + a3[1] * h, a2[2] + a3[2] * h};
      double an = orc_norm3(a1[i], a1[nm + i], a1[2 * nm + i]);
      double jn = orc_norm3(j1[i], j1[nm + i], j1[2 * nm + i]);
      double a2n = orc_norm3(a2e[0], a2e[1], a2e[2]);
      double a3n = orc_norm3(a3[0], a3[1], a3[2]);
      double den = jn * a3n + a2n * a2n;
      double dtc = den > 0.0 ? sqrt(p->eta * (an * a2n + jn * jn) / den) : dt_soft;
      int knew = orc_level_for(dt_soft, dtc, p->k_max);
      int k = lev[i];
      if (knew < k) {
        int64_t dbl = (int64_t)1 << (ORC_TICK_BITS - k + 1);
        if (k > 0 && (t[i] % dbl) == 0) k = k - 1;
      } else {
        k = knew;
      }
      if (k > p->k_max) { err |= ORC_ERR_KMAX; k = p->k_max; }
      lev[i] = k;
    }
    ++nsteps;
    if (tn == T) {
      int done = 1;
      for (int64_t i = 0; i < nm; ++i) done &= (t[i] == T);
      if (done) break;
    }
    if (nsteps > 100000000) { err |= ORC_ERR_NSTEPS; break; }
  }
  *nsteps_out = nsteps;
  if (dt_hard)
    for (int64_t i = 0; i < nm; ++i) dt_hard[i] = ldexp(dt_soft, -lev[i]);
  free(a0); free(j0); free(a1); free(j1); free(xp); free(vp); free(t); free(lev); free(act);
  return err;
}

/* Batch driver: clusters given by cl_ptr (n_clusters + 1) and members
 * (particle indices into the (3, n) arrays).  Each cluster is integrated
 * independently (OpenMP over clusters).  dt_hard (n, nullable) carries each
 * particle's hard step in and out (<= 0: use the initial-step criterion).
 * e0/e1 receive the hard-part energy before and after (nullable), nsteps the
 * block-step count (nullable). */
int orc_hermite_clusters(int64_t n, int64_t n_clusters, const int32_t *cl_ptr, const int32_t *members,
                         double *pos, double *vel, const double *m, const double *r_out, const orc_params *p,
                         double dt_soft, double *dt_hard, double *e0, double *e1, int64_t *nsteps) {
  int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int64_t c = 0; c < n_clusters; ++c) {
    int64_t b = cl_ptr[c], nm = cl_ptr[c + 1] - b;
    if (nm <= 0) continue;
    double *x = (double *)malloc(sizeof(double) * 3 * nm);
    double *v = (double *)malloc(sizeof(double) * 3 * nm);
    double *mm = (double *)malloc(sizeof(double) * nm);
    double *ro = (double *)malloc(sizeof(double) * nm);
    double *dh = dt_hard ? (double *)malloc(sizeof(double) * nm) : NULL;
    for (int64_t k = 0; k < nm; ++k) {
      int64_t i = members[b + k];
      for (int q = 0; q < 3; ++q) {
        x[q * nm + k] = pos[q * n + i];
        v[q * nm + k] = vel[q * n + i];
      }
      mm[k] = m[i];
      ro[k] = r_out[i];
      if (dh) dh[k] = dt_hard[i];
    }
    if (e0) e0[c] = orc_cluster_energy(nm, x, v, mm, ro, p);
    int64_t ns = 0;
    err |= orc_hermite_one(nm, x, v, mm, ro, p, dt_soft, dh, &ns);
    if (nsteps) nsteps[c] = ns;
    if (e1) e1[c] = orc_cluster_energy(nm, x, v, mm, ro, p);
    for (int64_t k = 0; k < nm; ++k) {
      int64_t i = members[b + k];
      for (int q = 0; q < 3; ++q) {
        pos[q * n + i] = x[q * nm + k];
        vel[q * n + i] = v[q * nm + k];
      }
      if (dh) dt_hard[i] = dh[k];
    }
    free(x); free(v); free(mm); free(ro); free(dh);
  }
  return err;
}

/* ------------------------------------------------------------------------ */
/* Perfect-accretion collisions in the hard part (Section 2.5.1).
 *
 * Two bodies collide when r_ij < f (R_p,i + R_p,j), R_p the radius of a
 * sphere of the body's mass at density rho.  The merged body keeps the
 * centre of mass and the momentum of the two.  Inside the hard part the two
 * stay two particles of one composite (Section 2.5.1: each keeps its own
 * cut-off radius): the hard force on each part is computed without the
 * mutual term of the composite's parts, and every part then moves with the
 * mass-weighted mean of its parts' accelerations (and jerks).
 *
 * Readings (the paper gives the model, not the scheme's details):
 *   - collisions are looked for at every block step, between two bodies of
 *     which at least one is due, with the predicted states at the block time
 *     (the states the force evaluation uses); of several colliding pairs the
 *     first in (lower slot, higher slot) order merges, one merger per block
 *     step;
 *   - the merger takes the states at the block time after the corrector
 *     (corrected for due members, predicted for the others); the composite's
 *     parts get the merged state, the block time, the hard acceleration and
 *     jerk evaluated there (mass-weighted mean over its parts) and a new step
 *     from the initial-step criterion with eta_0 (Section 3.1: "also for the
 *     first step after a collision"), quantised down and refined until the
 *     block time is a multiple of it; the other members keep their states;
 *   - the radius of a composite is that of its total mass;
 *   - the neighbours N_i of eq. (e3) are the other members of the cluster;
 *   - per merger the dissipations eq. (e0) ... eq. (e3) are added to eps[0..3]
 *     with W as printed; eps[4] receives the same sum with W replaced by one
 *     (the change of the Newtonian energy of the cluster, the reading the
 *     paper gives for that replacement), eps[5] the same with 1 - W (the
 *     change of the cluster's hard energy, eq. (hard)), so that
 *     E_hard(end) + sum eps[5] = E_hard(start) up to the integration error.
 * comp[k] (out) receives the lowest slot of member k's composite. */
static double orc_body_radius(double M, double rho) { return cbrt(3.0 * M / (4.0 * 3.14159265358979323846 * rho)); }

/* hard-part energy of eq. (hard) with the pairs inside a composite left out */
static double orc_cluster_energy_comp(int64_t nm, const double *x, const double *v, const double *m,
                                      const double *r_out, const orc_params *p, const int32_t *comp) {
  const double *X = x, *Y = x + nm, *Z = x + 2 * nm;
  const double *VX = v, *VY = v + nm, *VZ = v + 2 * nm;
  double e = 0.0;
  for (int64_t i = 0; i < nm; ++i) {
    double v2 = VX[i] * VX[i] + VY[i] * VY[i] + VZ[i] * VZ[i];
    double r = sqrt(X[i] * X[i] + Y[i] * Y[i] + Z[i] * Z[i]);
    e += 0.5 * m[i] * v2 - p->G * p->m_star * m[i] / r;
  }
  for (int64_t i = 0; i < nm; ++i)
    for (int64_t j = i + 1; j < nm; ++j) {
      if (comp[i] == comp[j]) continue;
      double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      double R = fmax(r_out[i], r_out[j]);
      e -= p->G * m[i] * m[j] * (1.0 - orc_W(r / R, p->gamma)) / r;
    }
  return e;
}

/* mass-weighted mean of a (3, nm) field over the parts of every composite
 * of more than one part: sum over the parts in slot order of m q, divided by
 * the composite's mass; only members with sel[k] (nullable: all) change */
static void orc_composite_mean(int64_t nm, const double *m, const int32_t *comp, const unsigned char *sel, double *q) {
  double *tmp = (double *)malloc(sizeof(double) * 3 * nm);
  memcpy(tmp, q, sizeof(double) * 3 * nm);
  for (int64_t k = 0; k < nm; ++k) {
    if (sel && !sel[k]) continue;
    int multi = 0;
    for (int64_t l = 0; l < nm; ++l) multi |= (l != k && comp[l] == comp[k]);
    if (!multi) continue;
    double M = 0.0, s[3] = {0.0, 0.0, 0.0};
    for (int64_t l = 0; l < nm; ++l) {
      if (comp[l] != comp[k]) continue;
      M += m[l];
      for (int c = 0; c < 3; ++c) s[c] += m[l] * tmp[c * nm + l];
    }
    for (int c = 0; c < 3; ++c) q[c * nm + k] = s[c] / M;
  }
  free(tmp);
}

int orc_hermite_collide_one(int64_t nm, double *x, double *v, const double *m, const double *r_out,
                            const orc_params *p, double dt_soft, double *dt_hard, double f, double rho,
                            int32_t *comp, double *eps, int64_t *nsteps_out, int64_t *ncoll_out, int64_t *tcoll_out) {
  int err = 0;
  const int64_t T = (int64_t)1 << ORC_TICK_BITS;
  const double tick = ldexp(dt_soft, -ORC_TICK_BITS);
  const double G = p->G, GM = p->G * p->m_star;
  size_t s3 = sizeof(double) * 3 * nm;
  double *a0 = (double *)malloc(s3), *j0 = (double *)malloc(s3);
  double *a1 = (double *)malloc(s3), *j1 = (double *)malloc(s3);
  double *xp = (double *)malloc(s3), *vp = (double *)malloc(s3);
  double *sx = (double *)malloc(s3), *sv = (double *)malloc(s3);
  double *an_ = (double *)malloc(s3), *jn_ = (double *)malloc(s3);
  double *rad = (double *)malloc(sizeof(double) * nm);
  int64_t *t = (int64_t *)calloc(nm, sizeof(int64_t));
  int *lev = (int *)malloc(sizeof(int) * nm);
  unsigned char *act = (unsigned char *)malloc(nm), *sel = (unsigned char *)malloc(nm);
  int64_t nsteps = 0, ncoll = 0;
  *tcoll_out = -1;
  for (int64_t k = 0; k < nm; ++k) {
    comp[k] = (int32_t)k;
    rad[k] = orc_body_radius(m[k], rho);
  }

  err |= orc_hard_acc_jerk_range(nm, x, v, m, r_out, p, 0, nm, NULL, comp, a0, j0);
  for (int64_t i = 0; i < nm; ++i) {
    double an = orc_norm3(a0[i], a0[nm + i], a0[2 * nm + i]);
    double jn = orc_norm3(j0[i], j0[nm + i], j0[2 * nm + i]);
    double dtc = jn > 0.0 ? p->eta0 * an / jn : dt_soft;
    if (dt_hard && dt_hard[i] > 0.0) dtc = dt_hard[i];
    int k = orc_level_for(dt_soft, dtc, p->k_max);
    if (k > p->k_max) { err |= ORC_ERR_KMAX; k = p->k_max; }
    lev[i] = k;
  }
  for (;;) {
    int64_t tn = T;
    for (int64_t i = 0; i < nm; ++i) {
      int64_t te = t[i] + ((int64_t)1 << (ORC_TICK_BITS - lev[i]));
      if (te < tn) tn = te;
    }
    for (int64_t i = 0; i < nm; ++i) act[i] = (t[i] + ((int64_t)1 << (ORC_TICK_BITS - lev[i]))) == tn;
    for (int64_t i = 0; i < nm; ++i) {
      double dl = (double)(tn - t[i]) * tick;
      double d2 = dl * dl / 2.0, d3 = dl * dl * dl / 6.0;
      for (int c = 0; c < 3; ++c) {
        int64_t q = c * nm + i;
        xp[q] = x[q] + v[q] * dl + a0[q] * d2 + j0[q] * d3;
        vp[q] = v[q] + a0[q] * dl + j0[q] * d2;
      }
    }
    /* collision test on the predicted states: the first colliding pair of
     * distinct bodies, at least one of them due */
    int64_t ci = -1, cj = -1;
    if (f > 0.0)
      for (int64_t i = 0; i < nm && ci < 0; ++i)
        for (int64_t j = i + 1; j < nm; ++j) {
          if (comp[i] == comp[j] || !(act[i] || act[j])) continue;
          double dx = xp[j] - xp[i], dy = xp[nm + j] - xp[nm + i], dz = xp[2 * nm + j] - xp[2 * nm + i];
          double r2 = dx * dx + dy * dy + dz * dz;
          double rs = f * (rad[i] + rad[j]);
          if (r2 < rs * rs) { ci = i; cj = j; break; }
        }
    err |= orc_hard_acc_jerk_range(nm, xp, vp, m, r_out, p, 0, nm, act, comp, a1, j1);
    orc_composite_mean(nm, m, comp, act, a1);
    orc_composite_mean(nm, m, comp, act, j1);
    for (int64_t i = 0; i < nm; ++i) {
      if (!act[i]) continue;
      double h = (double)(tn - t[i]) * tick;
      double a2[3], a3[3];
      for (int c = 0; c < 3; ++c) {
        int64_t q = c * nm + i;
        double da = a0[q] - a1[q];
        a2[c] = (-6.0 * da - h * (4.0 * j0[q] + 2.0 * j1[q])) / (h * h);
        a3[c] = (12.0 * da + 6.0 * h * (j0[q] + j1[q])) / (h * h * h);
        x[q] = xp[q] + a2[c] * (h * h * h * h) / 24.0 + a3[c] * (h * h * h * h * h) / 120.0;
        v[q] = vp[q] + a2[c] * (h * h * h) / 6.0 + a3[c] * (h * h * h * h) / 24.0;
        a0[q] = a1[q];
        j0[q] = j1[q];
      }
      t[i] = tn;
      double a2e[3] = {a2[0] + a3[0] * h, a2[1] + a3[1] * h, a2[2] + a3[2] * h};
      double an = orc_norm3(a1[i], a1[nm + i], a1[2 * nm + i]);
      double jn = orc_norm3(j1[i], j1[nm + i], j1[2 * nm + i]);
      double a2n = orc_norm3(a2e[0], a2e[1], a2e[2]);
      double a3n = orc_norm3(a3[0], a3[1], a3[2]);
      double den = jn * a3n + a2n * a2n;
      double dtc = den > 0.0 ? sqrt(p->eta * (an * a2n + jn * jn) / den) : dt_soft;
      int knew = orc_level_for(dt_soft, dtc, p->k_max);
      int k = lev[i];
      if (knew < k) {
        int64_t dbl = (int64_t)1 << (ORC_TICK_BITS - k + 1);
        if (k > 0 && (t[i] % dbl) == 0) k = k - 1;
      } else {
        k = knew;
      }
      if (k > p->k_max) { err |= ORC_ERR_KMAX; k = p->k_max; }
      lev[i] = k;
    }
    if (ci >= 0) {
      /* states at tn: corrected (due members) or predicted (the others) */
      for (int64_t i = 0; i < nm; ++i)
        for (int c = 0; c < 3; ++c) {
          sx[c * nm + i] = act[i] ? x[c * nm + i] : xp[c * nm + i];
          sv[c * nm + i] = act[i] ? v[c * nm + i] : vp[c * nm + i];
        }
      const int32_t A = comp[ci], B = comp[cj];
      double MA = 0.0, MB = 0.0;
      for (int64_t k = 0; k < nm; ++k) {
        if (comp[k] == A) MA += m[k];
        if (comp[k] == B) MB += m[k];
      }
      const double M = MA + MB;
      double xa[3], xb[3], va[3], vb[3], xn[3], vn[3];
      for (int c = 0; c < 3; ++c) {
        xa[c] = sx[c * nm + ci]; xb[c] = sx[c * nm + cj];
        va[c] = sv[c * nm + ci]; vb[c] = sv[c * nm + cj];
        xn[c] = (MA * xa[c] + MB * xb[c]) / M;
        vn[c] = (MA * va[c] + MB * vb[c]) / M;
      }
      const double dvx = va[0] - vb[0], dvy = va[1] - vb[1], dvz = va[2] - vb[2];
      const double e0 = 0.5 * (MA * MB / M) * (dvx * dvx + dvy * dvy + dvz * dvz);          /* eq. (e0) */
      const double rab = orc_norm3(xb[0] - xa[0], xb[1] - xa[1], xb[2] - xa[2]);
      double e1 = 0.0, e1u = 0.0, e1h = 0.0;                                                 /* eq. (e1) */
      for (int64_t a = 0; a < nm; ++a) {
        if (comp[a] != A) continue;
        for (int64_t b = 0; b < nm; ++b) {
          if (comp[b] != B) continue;
          double W = orc_W(rab / fmax(r_out[a], r_out[b]), p->gamma);
          e1 -= G * m[a] * m[b] * W / rab;
          e1u -= G * m[a] * m[b] / rab;
          e1h -= G * m[a] * m[b] * (1.0 - W) / rab;
        }
      }
      const double e2 = -GM * (MA / orc_norm3(xa[0], xa[1], xa[2]) + MB / orc_norm3(xb[0], xb[1], xb[2]) -
                               M / orc_norm3(xn[0], xn[1], xn[2]));                      /* eq. (e2) */
      double e3 = 0.0, e3u = 0.0, e3h = 0.0;                                                 /* eq. (e3) */
      for (int64_t a = 0; a < nm; ++a) {
        if (comp[a] != A && comp[a] != B) continue;
        const double *xo = comp[a] == A ? xa : xb;
        for (int64_t k = 0; k < nm; ++k) {
          if (comp[k] == A || comp[k] == B) continue;
          const double R = fmax(r_out[a], r_out[k]);
          const double ro = orc_norm3(sx[k] - xo[0], sx[nm + k] - xo[1], sx[2 * nm + k] - xo[2]);
          const double rn = orc_norm3(sx[k] - xn[0], sx[nm + k] - xn[1], sx[2 * nm + k] - xn[2]);
          const double Wo = orc_W(ro / R, p->gamma), Wn = orc_W(rn / R, p->gamma);
          e3 -= G * m[a] * m[k] * (Wo / ro - Wn / rn);
          e3u -= G * m[a] * m[k] * (1.0 / ro - 1.0 / rn);
          e3h -= G * m[a] * m[k] * ((1.0 - Wo) / ro - (1.0 - Wn) / rn);
        }
      }
      eps[0] += e0; eps[1] += e1; eps[2] += e2; eps[3] += e3;
      eps[4] += e0 + e1u + e2 + e3u;
      eps[5] += e0 + e1h + e2 + e3h;
      /* the composite takes the merged state at tn */
      const int32_t cn = A < B ? A : B;
      const double Rn = orc_body_radius(M, rho);
      for (int64_t k = 0; k < nm; ++k) {
        sel[k] = 0;
        if (comp[k] != A && comp[k] != B) continue;
        sel[k] = 1;
        comp[k] = cn;
        rad[k] = Rn;
        t[k] = tn;
        for (int c = 0; c < 3; ++c) {
          x[c * nm + k] = sx[c * nm + k] = xn[c];
          v[c * nm + k] = sv[c * nm + k] = vn[c];
        }
      }
      /* its acceleration and jerk at tn from everyone's state at tn */
      err |= orc_hard_acc_jerk_range(nm, sx, sv, m, r_out, p, 0, nm, sel, comp, an_, jn_);
      orc_composite_mean(nm, m, comp, sel, an_);
      orc_composite_mean(nm, m, comp, sel, jn_);
      for (int64_t k = 0; k < nm; ++k) {
        if (!sel[k]) continue;
        for (int c = 0; c < 3; ++c) {
          a0[c * nm + k] = an_[c * nm + k];
          j0[c * nm + k] = jn_[c * nm + k];
        }
        double an = orc_norm3(an_[k], an_[nm + k], an_[2 * nm + k]);
        double jn = orc_norm3(jn_[k], jn_[nm + k], jn_[2 * nm + k]);
        double dtc = jn > 0.0 ? p->eta0 * an / jn : dt_soft;
        int kl = orc_level_for(dt_soft, dtc, p->k_max);
        if (kl > p->k_max) { err |= ORC_ERR_KMAX; kl = p->k_max; }
        while (kl < p->k_max && (tn % ((int64_t)1 << (ORC_TICK_BITS - kl))) != 0) ++kl;
        lev[k] = kl;
      }
      if (ncoll == 0) *tcoll_out = tn;
      ++ncoll;
    }
    ++nsteps;
    if (tn == T) {
      int done = 1;
      for (int64_t i = 0; i < nm; ++i) done &= (t[i] == T);
      if (done) break;
    }
    if (nsteps > 100000000) { err |= ORC_ERR_NSTEPS; break; }
  }
  *nsteps_out = nsteps;
  *ncoll_out = ncoll;
  if (dt_hard)
    for (int64_t i = 0; i < nm; ++i) dt_hard[i] = ldexp(dt_soft, -lev[i]);
  free(a0); free(j0); free(a1); free(j1); free(xp); free(vp); free(sx); free(sv); free(an_); free(jn_);
  free(rad); free(t); free(lev); free(act); free(sel);
  return err;
}

/* Batch driver of orc_hermite_collide_one (clusters as orc_hermite_clusters).
 * merged_into (n) receives, for every member, the particle index of its
 * composite's lowest slot (members are listed in ascending index, so the
 * lowest index); eps (n_clusters x 6), e0 / e1 (hard energies with the pairs
 * inside composites left out), nsteps, ncoll and tcoll (block time of the
 * first merger in ticks of dt_soft 2^-40, -1 if none) per cluster; every
 * output but merged_into is nullable. */
int orc_hermite_collide_clusters(int64_t n, int64_t n_clusters, const int32_t *cl_ptr, const int32_t *members,
                                 double *pos, double *vel, const double *m, const double *r_out, const orc_params *p,
                                 double dt_soft, double *dt_hard, double f, double rho, int32_t *merged_into,
                                 double *eps, double *e0, double *e1, int64_t *nsteps, int64_t *ncoll, int64_t *tcoll) {
  int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int64_t c = 0; c < n_clusters; ++c) {
    int64_t b = cl_ptr[c], nm = cl_ptr[c + 1] - b;
    if (nm <= 0) continue;
    double *x = (double *)malloc(sizeof(double) * 3 * nm);
    double *v = (double *)malloc(sizeof(double) * 3 * nm);
    double *mm = (double *)malloc(sizeof(double) * nm);
    double *ro = (double *)malloc(sizeof(double) * nm);
    double *dh = dt_hard ? (double *)malloc(sizeof(double) * nm) : NULL;
    int32_t *cp = (int32_t *)malloc(sizeof(int32_t) * nm);
    for (int64_t k = 0; k < nm; ++k) {
      int64_t i = members[b + k];
      for (int q = 0; q < 3; ++q) {
        x[q * nm + k] = pos[q * n + i];
        v[q * nm + k] = vel[q * n + i];
      }
      mm[k] = m[i];
      ro[k] = r_out[i];
      cp[k] = (int32_t)k;
      if (dh) dh[k] = dt_hard[i];
    }
    if (e0) e0[c] = orc_cluster_energy_comp(nm, x, v, mm, ro, p, cp);
    double ec[6] = {0, 0, 0, 0, 0, 0};
    int64_t ns = 0, nco = 0, tc = -1;
    err |= orc_hermite_collide_one(nm, x, v, mm, ro, p, dt_soft, dh, f, rho, cp, ec, &ns, &nco, &tc);
    if (eps)
      for (int q = 0; q < 6; ++q) eps[6 * c + q] = ec[q];
    if (nsteps) nsteps[c] = ns;
    if (ncoll) ncoll[c] = nco;
    if (tcoll) tcoll[c] = tc;
    if (e1) e1[c] = orc_cluster_energy_comp(nm, x, v, mm, ro, p, cp);
    for (int64_t k = 0; k < nm; ++k) {
      int64_t i = members[b + k];
      for (int q = 0; q < 3; ++q) {
        pos[q * n + i] = x[q * nm + k];
        vel[q * n + i] = v[q * nm + k];
      }
      merged_into[i] = members[b + cp[k]];
      if (dh) dt_hard[i] = dh[k];
    }
    free(x); free(v); free(mm); free(ro); free(dh); free(cp);
  }
  return err;
}

/* ------------------------------------------------------------------------ */
/* Neighbour test for one pair (Section 2.3, eq. (rsearch), eq. (rsearch1) and
 * the slow-pair clause that follows it).
 * j is a neighbour of i iff
 *   (a) r_ij < max(r_search,i, r_search,j)                     (candidate), and
 *   (b) the closest approach over the soft step, |r_ij + v_ij t_min| with
 *       t_min = clamp(-r.v / v^2, 0, dt), is <= Rsearch2 r_out,ij, or
 *   (c) |v_ij| < Rsearch3 a_ij dt / 2, a_ij = G (m_i + m_j) / r_ij^2.
 * Readings: the printed exclusion sentence is inverted relative to its own
 * explanation; pairs are kept when the closest approach does not exceed
 * Rsearch2 r_out,ij.  t_min is the minimiser of the distance (the text says
 * "maximum" but prints the minimiser).  a_ij is the mutual acceleration
 * G (m_i + m_j) / r^2, which keeps the relation symmetric.
 * The comparisons are done without square roots or divisions: the three
 * t_min cases become polynomial inequalities after multiplying through by
 * v^2 > 0 and squaring non-negative sides.  Every operation below is a single
 * IEEE FP64 operation in the order written (compiled without contraction),
 * which fixes the decision bit for bit. */
static int orc_pair_is_neighbour(double xi, double yi, double zi, double vxi, double vyi, double vzi, double mi,
                                 double roi, double rsi, double xj, double yj, double zj, double vxj, double vyj,
                                 double vzj, double mj, double roj, double rsj, const orc_params *p) {
  double dx = xi - xj, dy = yi - yj, dz = zi - zj;
  double ux = vxi - vxj, uy = vyi - vyj, uz = vzi - vzj;
  double rr = ((dx * dx) + (dy * dy)) + (dz * dz);
  double rs = rsi > rsj ? rsi : rsj;
  if (!(rr < rs * rs)) return 0;
  double rv = ((dx * ux) + (dy * uy)) + (dz * uz);
  double vv = ((ux * ux) + (uy * uy)) + (uz * uz);
  double ro = roi > roj ? roi : roj;
  double R2 = p->r_search2 * ro;
  double RR = R2 * R2;
  double dt = p->dt_soft;
  int close;
  if (vv == 0.0 || rv >= 0.0) {
    close = rr <= RR;
  } else if (-rv < dt * vv) {
    close = (rr * vv - rv * rv) <= RR * vv;
  } else {
    close = (rr + (2.0 * dt) * rv) + (dt * dt) * vv <= RR;
  }
  if (close) return 1;
  double A = (p->r_search3 * (p->G * (mi + mj))) * (0.5 * dt);
  return vv * (rr * rr) < A * A;
}

/* Neighbour rows for the particles idx[0..ni): row k lists, in ascending
 * order, every j != idx[k] that passes the test above.  row_ptr has ni + 1
 * entries.  col receives at most cap entries; the total count is returned
 * (if it exceeds cap, col is left partially filled and only row_ptr is
 * complete).  Direct O(ni * N) scan. */
int64_t orc_neighbour_rows(int64_t n, const double *pos, const double *vel, const double *m, const double *r_out,
                           const double *r_search, const orc_params *p, int64_t ni, const int64_t *idx,
                           int64_t *row_ptr, int32_t *col, int64_t cap) {
  const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
  const double *VX = vel, *VY = vel + n, *VZ = vel + 2 * n;
  int64_t *cnt = (int64_t *)calloc(ni > 0 ? ni : 1, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < ni; ++k) {
    int64_t i = idx[k], c = 0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      c += orc_pair_is_neighbour(X[i], Y[i], Z[i], VX[i], VY[i], VZ[i], m[i], r_out[i], r_search[i], X[j], Y[j],
                                 Z[j], VX[j], VY[j], VZ[j], m[j], r_out[j], r_search[j], p);
    }
    cnt[k] = c;
  }
  row_ptr[0] = 0;
  for (int64_t k = 0; k < ni; ++k) row_ptr[k + 1] = row_ptr[k] + cnt[k];
  int64_t nnz = row_ptr[ni];
  free(cnt);
  if (nnz > cap) return nnz;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < ni; ++k) {
    int64_t i = idx[k], w = row_ptr[k];
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      if (orc_pair_is_neighbour(X[i], Y[i], Z[i], VX[i], VY[i], VZ[i], m[i], r_out[i], r_search[i], X[j], Y[j],
                                Z[j], VX[j], VY[j], VZ[j], m[j], r_out[j], r_search[j], p))
        col[w++] = (int32_t)j;
    }
  }
  return nnz;
}

/* Single pair, exported for the predicate tests. */
int orc_is_neighbour(const double *pi, const double *pj, const orc_params *p) {
  /* pi, pj: x, y, z, vx, vy, vz, m, r_out, r_search */
  return orc_pair_is_neighbour(pi[0], pi[1], pi[2], pi[3], pi[4], pi[5], pi[6], pi[7], pi[8], pj[0], pj[1], pj[2],
                               pj[3], pj[4], pj[5], pj[6], pj[7], pj[8], p);
}

/* ------------------------------------------------------------------------ */
/* Neighbour-cluster labels, Section 2.3 steps i-iii: every particle starts
 * with its own index; each sweep sets a particle's index to the minimum over
 * itself and its neighbours (all from the previous sweep); sweeps repeat
 * until nothing changes.  Returns the number of sweeps. */
int orc_labels(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t *label) {
  int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) label[i] = (int32_t)i;
  int sweeps = 0;
  for (;;) {
    memcpy(prev, label, sizeof(int32_t) * n);
    int changed = 0;
    for (int64_t i = 0; i < n; ++i) {
      int32_t l = prev[i];
      for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q)
        if (prev[col[q]] < l) l = prev[col[q]];
      if (l != label[i]) { label[i] = l; changed = 1; }
    }
    ++sweeps;
    if (!changed) break;
  }
  free(prev);
  return sweeps;
}

/* ------------------------------------------------------------------------ */
/* Vector-Jacobian product of the soft acceleration of eq. (softforce) with
 * the pair cut-offs r_out,ij frozen: for L = sum_i lam_i . a_i(x, m),
 *   dL/dm_k = sum_{i != k} phi(r_ik) lam_i . (x_k - x_i)
 *   dL/dx_k = sum_{j != k} [ phi(r) w + (phi'(r) / r) d (d . w) ],
 *             d = x_j - x_k, w = m_k lam_j - m_j lam_k,
 * with phi(r) = G K(r/R) / r^3 and phi'(r) = G [K'(r/R) / (R r^3) - 3 K / r^4].
 * (Differentiating each pair term m_j phi(r_ij)(x_j - x_i) once with respect
 * to its source and once to its target.)  Direct O(N^2). */
int orc_soft_adjoint(int64_t n, const double *pos, const double *m, const double *r_out, double G, double gamma,
                     const double *lam, double *g_pos, double *g_mass) {
  const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
  const double *LX = lam, *LY = lam + n, *LZ = lam + 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < n; ++k) {
    double gx = 0.0, gy = 0.0, gz = 0.0, gm = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == k) continue;
      double dx = X[j] - X[k], dy = Y[j] - Y[k], dz = Z[j] - Z[k];
      double r2 = dx * dx + dy * dy + dz * dz;
      double r = sqrt(r2);
      double R = fmax(r_out[k], r_out[j]);
      double y = r / R;
      double K = orc_K(y, gamma);
      double Ky = orc_dKdy(y, gamma);
      double phi = G * K / (r2 * r);
      double dphi = G * (Ky / (R * r2 * r) - 3.0 * K / (r2 * r2));
      double wx = m[k] * LX[j] - m[j] * LX[k];
      double wy = m[k] * LY[j] - m[j] * LY[k];
      double wz = m[k] * LZ[j] - m[j] * LZ[k];
      double dw = dx * wx + dy * wy + dz * wz;
      gx += phi * wx + dphi / r * dx * dw;
      gy += phi * wy + dphi / r * dy * dw;
      gz += phi * wz + dphi / r * dz * dw;
      /* dL/dm_k: pair (i = j here, source k): phi lam_j . (x_k - x_j) */
      gm += phi * (LX[j] * (-dx) + LY[j] * (-dy) + LZ[j] * (-dz));
    }
    g_pos[k] = gx; g_pos[n + k] = gy; g_pos[2 * n + k] = gz;
    g_mass[k] = gm;
  }
  return 0;
}

/* Number of OpenMP threads the oracle runs on (for reporting). */
int orc_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Set the number of OpenMP threads of later calls (timing at a stated core
 * count); returns the number now in effect. */
int orc_set_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
  return orc_num_threads();
}
