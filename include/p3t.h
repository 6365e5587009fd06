/*
 * p3t.h -- C ABI of libp3t.so: the soft-force hot path of the P3T
 * (particle-particle particle-tree) scheme with individual cut-off radii
 * (Ishigaki et al. 2021, "GPLUM", PASJ 73), on one AMD MI355X (gfx950).
 *
 * Conventions for every entry point
 *   - Pointers are DEVICE pointers unless the name ends in _host.
 *   - Particle arrays are in the caller's original order, caller-owned.
 *     pos3 / vel3 / acc3 are structure-of-arrays FP64 of 3*n doubles:
 *     x row [0, n), y row [n, 2n), z row [2n, 3n).
 *   - Units: G = M_* = 1 by default, heliocentric coordinates, no indirect
 *     term (Section 2.1.1).
 *   - Calls are asynchronous on the context's HIP stream unless they return
 *     a host value (documented per call); they allocate only inside
 *     p3t_reserve or when a capacity must grow.
 *   - Every call returns a p3t_status.  Argument errors are detected on the
 *     host before any launch and leave all state unchanged.  Conditions found
 *     on the device set bits in the context's status word (P3T_FLAG_*), read
 *     with p3t_get_status.  p3t_last_error() explains the last failure.
 *   - n = 0 is a valid no-op for every per-particle call.
 */
#ifndef P3T_H
#define P3T_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct p3t_ctx p3t_ctx;

typedef enum {
  P3T_OK = 0,
  P3T_ERR_ARG = 1,      /* invalid argument (null pointer, n < 0, bad parameter) */
  P3T_ERR_CAPACITY = 2, /* caller's output buffer too small; required size returned */
  P3T_ERR_HIP = 3,      /* HIP runtime error */
  P3T_ERR_STATE = 4,    /* call order violated (e.g. force before tree) */
  P3T_ERR_NUMERIC = 5,  /* device reported NaN / coincident particles / step underflow */
  P3T_ERR_CLUSTER = 6   /* kept for compatibility; no longer returned (clusters of any size are integrated) */
} p3t_status;

/* Device status word bits (p3t_get_status). */
#define P3T_FLAG_COINCIDENT 0x01u     /* two distinct particles at the same position */
#define P3T_FLAG_NAN 0x02u            /* non-finite force or state */
#define P3T_FLAG_LIST_OVERFLOW 0x04u  /* interaction list exceeded its capacity (retried internally) */
#define P3T_FLAG_STACK_OVERFLOW 0x08u /* tree-walk stack exceeded its capacity (retried internally) */
#define P3T_FLAG_PAIR_OVERFLOW 0x10u  /* neighbour-pair buffer exceeded its capacity (retried internally) */
#define P3T_FLAG_KMAX 0x20u           /* Hermite step below dt_soft * 2^-k_max */
#define P3T_FLAG_NSTEPS 0x40u         /* Hermite block-step count limit reached */
#define P3T_FLAG_BIG_CLUSTER 0x80u    /* a cluster took the percolated-cluster path (above cluster_cap members) */
#define P3T_FLAG_UNBOUND 0x100u       /* an isolated particle's orbit is not bound (left in place; isolated = 1) */
#define P3T_FLAG_GROUP_BOUND 0x200u   /* more interaction groups than the host's bound (retried internally) */
#define P3T_FLAG_COLL_UNCHECKED 0x400u /* p3t_hard_step_collide: a cluster above 64 members was integrated
                                           without looking for collisions */

/* Parameters.  Defaults (p3t_default_params) are the paper's values where it
 * prints them (Section 3.1: eta = 0.01, eta_0 = 0.1 eta, Rsearch0..3 = 1.1,
 * 6, 2, 2; Section 2.1.3: Rcut1 = 8; G = M_* = 1) and stated readings where it
 * does not (gamma = 0.1, Rcut0 = 2, dt_soft = 2 pi / 64, theta = 0.5). */
typedef struct {
  double G, m_star;      /* gravitational constant, central mass */
  double gamma;          /* r_in / r_out of the changeover, 0 < gamma < 1 (eq. (cutfuncW)) */
  double r_cut0, r_cut1; /* eq. (routi2) */
  double r_search0, r_search1, r_search2, r_search3; /* eq. (rsearch), eq. (rsearch1) */
  double dt_soft;        /* soft step */
  double theta;          /* Barnes-Hut opening angle, >= 0 (0: exact direct sum) */
  double eta, eta0;      /* Hermite accuracy parameters (Section 3.1) */
  int32_t multipole;     /* 1: monopole cells, 2: quadrupole cells */
  int32_t precision;     /* 0: FP64 throughout, 1: mixed (FP32 far field, FP64 near pairs) */
  int32_t cutoff_mode;   /* 0: individual pair cut-off (eq. (rout2)), 1: shared (eq. (rout1)) */
  int32_t hill_length;   /* 0: Hill radius from the osculating semi-major axis, 1: from |x| */
  int32_t n_group_max;   /* max i-particles per interaction group, 1..128 */
  int32_t n_leaf_max;    /* tree nodes with at most this many particles are opened as leaves */
  int32_t vran_bins;     /* log-spaced cylindrical-radius bins for the random velocity */
  int32_t vran_min_count;/* bins with fewer members use the rms over all particles */
  int32_t k_max;         /* deepest Hermite block level (step dt_soft * 2^-k_max), <= 40 */
  int32_t cluster_cap;   /* clusters above min(cluster_cap, 1024) members take the percolated-cluster
                            path of the hard part (p3t_hermite_cluster_step); default 1024 */
  int32_t isolated;      /* clusters of one particle in the hard part: 0 Hermite with the star only,
                            1 Kepler drift as p3t_kepler_drift (Section 2.2) */
} p3t_params;

/* Counters and phase times of the last evaluation (p3t_get_stats). */
typedef struct {
  int64_t n;            /* particles in the current tree */
  int64_t n_nodes;      /* tree nodes (2n - 1) */
  int64_t n_groups;     /* interaction groups */
  int64_t n_near;       /* i-j evaluations with the changeover (self pairs excluded) */
  int64_t n_far;        /* i-j evaluations with K = 1 */
  int64_t n_cell;       /* i-cell multipole evaluations */
  int64_t n_pairs;      /* neighbour pairs found (directed, = nnz) */
  int64_t list_entries; /* total interaction-list entries (near + far + cells) */
  double ms_cutoffs, ms_tree, ms_walk, ms_force, ms_neighbour, ms_hermite; /* event-timed phases */
  /* the force phase by kernel (split form; zero for the fused kernel):
     near particles with the changeover, far particles, cells, exact
     neighbour test of the candidates */
  double ms_near, ms_far, ms_cell, ms_cand;
  int32_t timing;       /* 1 if the phase times above were measured */
  int32_t n_slow;       /* members of slow clusters in the last p3t_hard_evaluate */
  double ms_direct;     /* p3t_hard_evaluate: the direct terms of the slow members */
  /* the last hard part (p3t_hard_step, p3t_hard_evaluate, p3t_hermite_cluster_step),
     read at the next synchronising call: Hermite force evaluations of members
     due in a block step, and the pair terms among them (each member due
     evaluates every other member of its cluster) */
  int64_t n_heval, n_hpair;
  double ms_sort;       /* the radix sort inside the tree build */
  double ms_clusters;   /* neighbour CSR, labels and cluster CSR at the start of the hard part */
} p3t_stats;

/* Fill *p_host with the defaults described above. */
void p3t_default_params(p3t_params *p_host);

/* Create a context bound to the current HIP device and to hip_stream (a
 * hipStream_t; NULL = the null stream).  Validates *p_host (P3T_ERR_ARG).
 * The context owns all scratch memory; the caller owns every I/O buffer. */
p3t_status p3t_create(const p3t_params *p_host, void *hip_stream, p3t_ctx **out_host);
p3t_status p3t_destroy(p3t_ctx *ctx);
p3t_status p3t_set_stream(p3t_ctx *ctx, void *hip_stream);
/* Replace the parameters (validated).  Invalidates the tree. */
p3t_status p3t_set_params(p3t_ctx *ctx, const p3t_params *p_host);
p3t_status p3t_get_params(p3t_ctx *ctx, p3t_params *p_host);

/* Size scratch for up to n_max particles and nnz_max neighbour pairs.  Not
 * required (calls grow scratch on demand) but avoids allocation later. */
p3t_status p3t_reserve(p3t_ctx *ctx, int64_t n_max, int64_t nnz_max);

/* Cut-off and search radii (Hill radius, Section 2.1.1; eq. (routi2);
 * eq. (rsearch)):  r_out,i = max(Rcut0 r_Hill,i, Rcut1 v_ran,i dt),
 * r_search,i = Rsearch0 r_out,i + Rsearch1 v_ran,i dt, with v_ran,i the rms
 * random velocity (|v - v_Kepler|) of the particle's radial bin.  In shared
 * mode (cutoff_mode = 1, eq. (rout1); Section 2.3 for the search radius)
 * every r_out,i is then replaced by max_k r_out,k and every r_search,i by
 * max_k r_search,k, so that every pair uses the same two radii.  Outputs (n
 * doubles each) r_out, r_search, v_ran (v_ran nullable; v_ran stays the
 * particle's own bin value in both modes). */
p3t_status p3t_compute_cutoffs(p3t_ctx *ctx, int64_t n, const double *pos3, const double *vel3,
                               const double *mass, double *r_out, double *r_search, double *v_ran);

/* Build the Barnes-Hut tree over n particles (Morton order, tight bounding
 * boxes, mass, centre of mass, traceless quadrupole, max search reach per
 * node) and the interaction groups.  The pointers are read during the call
 * only (the tree keeps its own sorted copies). */
p3t_status p3t_build_tree(p3t_ctx *ctx, int64_t n, const double *pos3, const double *vel3, const double *mass,
                          const double *r_out, const double *r_search);

/* Soft acceleration of every particle of the current tree, eq. (softforce)
 * divided by m_i with the pair cut-off of eq. (rout2):
 *   a_i = sum_j G m_j K(r_ij / r_out,ij) (x_j - x_i) / r_ij^3
 * (star excluded).  Pairs within the search reach are evaluated directly in
 * FP64 with the changeover K; the rest via particles or multipole cells with
 * K = 1.  Also collects the neighbour pairs of Section 2.3 for
 * p3t_neighbour_list.  acc3: 3n doubles, written in original order. */
p3t_status p3t_compute_soft_force(p3t_ctx *ctx, double *acc3);

/* Neighbour lists (Section 2.3) of the last p3t_compute_soft_force, as CSR in
 * original indices: row_ptr (n + 1 int64), col (cap int32), rows ascending.
 * j is in row i iff r_ij < max(r_search,i, r_search,j) and the closest
 * approach over the soft step is <= Rsearch2 r_out,ij or |v_ij| <
 * Rsearch3 G (m_i + m_j) / r_ij^2 dt / 2.  Synchronises; *nnz_host = nnz.
 * If nnz > cap returns P3T_ERR_CAPACITY with *nnz_host set and col
 * untouched.  label (n int32, nullable) receives the neighbour-cluster index
 * of every particle (Section 2.3 steps i-iii: the minimum index of its
 * connected component). */
p3t_status p3t_neighbour_list(p3t_ctx *ctx, int64_t *row_ptr, int32_t *col, int64_t cap, int64_t *nnz_host,
                              int32_t *label);

/* Cluster CSR from labels (label[i] = min index of i's cluster): cl_ptr
 * (n + 1 int32, first n_clusters + 1 used), cl_members (n int32), members
 * sorted by (cluster, index).  Synchronises; *n_clusters_host set. */
p3t_status p3t_clusters(p3t_ctx *ctx, int64_t n, const int32_t *label, int32_t *cl_ptr, int32_t *cl_members,
                        int64_t *n_clusters_host);

/* Fourth-order Hermite integration of every neighbour cluster over one soft
 * step with block time steps (Section 2.1.1; Section 2.2 step (5)).  Forces:
 * central star + all intra-cluster pairs with (1 - K) (eq. (hardforce)),
 * jerk including dK/dt.  Steps dt_soft * 2^-k from Aarseth's criterion with
 * eta; the first step uses eta_0 |a|/|jerk| unless dt_hard carries one.
 * pos3 / vel3 (3n) are updated in place for the listed members.  mass, r_out
 * (n).  cl_ptr (n_clusters + 1), cl_members (indices into the n particles).
 * dt_hard (n, nullable) carries each particle's hard step in and out
 * (<= 0: initial criterion).  e_rel_err (n_clusters, nullable) receives
 * |E_end - E_start| / |E_start| of eq. (hard) restricted to the cluster;
 * n_steps (n_clusters int32, nullable) the number of block steps taken.
 * Clusters of up to 64 members share one launch (several per wavefront),
 * clusters of 65..1024 members take one workgroup each.  A cluster above
 * min(cluster_cap, 1024) members means the neighbour graph has percolated
 * (Section 3.2.3: the paper then integrates it directly on one process):
 * it is integrated with the same scheme by the percolated-cluster path,
 * member states in device memory, one wavefront per member due in a block
 * step summing its partners over the whole chip, two launches per block
 * step issued in batches by the host (the call then blocks until those
 * clusters are done), and P3T_FLAG_BIG_CLUSTER is set in the status word.
 * Malformed cl_ptr / cl_members return P3T_ERR_ARG. */
p3t_status p3t_hermite_cluster_step(p3t_ctx *ctx, int64_t n, int64_t n_clusters, const int32_t *cl_ptr,
                                    const int32_t *cl_members, double *pos3, double *vel3, const double *mass,
                                    const double *r_out, double *dt_hard, double *e_rel_err, int32_t *n_steps);

/* Soft kick, eq. (HamiltonSol): vel3 += h * acc3 (3n each). */
p3t_status p3t_kick(p3t_ctx *ctx, int64_t n, double h, const double *acc3, double *vel3);

/* Kepler drift of particles without neighbours (Section 2.2: the hard part
 * of an isolated particle is its orbit about the star, from Kepler's equation
 * solved by Newton-Raphson).  Each listed particle moves for dt on the
 * two-body orbit of mu = G * m_star of the context's parameters, its own mass
 * neglected: Newton-Raphson from dE = n dt on Kepler's equation in the
 * eccentric-anomaly difference dE, dE - e cos E0 sin dE + e sin E0 (1 - cos dE)
 * = n dt (to |step| <= 1e-15 max(1, |dE|), at most 50 iterations), then the f
 * and g functions.  FP64.  pos3, vel3 (3n, x row then y row then z row) are
 * updated in place for the listed particles only.  list (n_list int32
 * indices into the n particles, distinct; NULL: all particles, n_list must
 * then equal n).  iters (n_list int32, nullable) receives the Newton
 * iterations per list entry, -1 for an orbit that is not bound (1/a <= 0 or
 * not finite), which is left unchanged, -2 for an index outside [0, n),
 * which is skipped.  n_unbound_host (nullable): the call synchronises and
 * writes the number of orbits that were not bound; P3T_ERR_ARG then also
 * reports indices outside [0, n).  P3T_ERR_STATE when G * m_star <= 0. */
p3t_status p3t_kepler_drift(p3t_ctx *ctx, int64_t n, double dt, double *pos3, double *vel3, const int32_t *list,
                            int64_t n_list, int32_t *iters, int64_t *n_unbound_host);

/* The hard part of a soft step (Section 2.2, steps (4)-(5)) in one call,
 * from the neighbour pairs of the last p3t_compute_soft_force (or
 * p3t_evaluate): cluster labels (minimum index per connected component,
 * Section 2.3), the cluster CSR, and the Hermite integration of every
 * cluster over dt_soft (as p3t_hermite_cluster_step), all on the device with
 * one host synchronisation (the cluster-size buckets).  pos3, vel3 (3n) are
 * updated in place; mass, r_out (n) as for p3t_hermite_cluster_step; dt_hard
 * (n, nullable) carries each particle's hard step.  steps (n int32,
 * nullable) receives the block steps taken by each particle's cluster (1 for
 * a Kepler-drifted particle).  *n_clusters_host (nullable) receives the
 * number of clusters.  Conditions detected on the
 * device during the integration (P3T_FLAG_KMAX, P3T_FLAG_NSTEPS,
 * P3T_FLAG_NAN) are left in the status word for p3t_get_status or the next
 * synchronising call.  P3T_ERR_STATE without a prior force evaluation.
 * Clusters above min(cluster_cap, 1024) members take the percolated-cluster
 * path (see p3t_hermite_cluster_step). */
p3t_status p3t_hard_step(p3t_ctx *ctx, double *pos3, double *vel3, const double *mass, const double *r_out,
                         double *dt_hard, int32_t *steps, int64_t *n_clusters_host);

/* p3t_hermite_cluster_step with perfect-accretion collisions (the model
 * and readings of p3t_hard_step_collide, below) on caller-given clusters.
 * merged_into (n int32, required) receives for every particle the particle
 * at its composite's first slot in the cluster's member list (with members
 * listed in ascending index: the lowest index), its own index otherwise.
 * eps6 (6 n_clusters doubles, nullable): per cluster eps_0 .. eps_3 (with W),
 * their total with W replaced by one and with 1 - W.  e_rel_err (nullable):
 * |E_hard(end) + eps_5 - E_hard(start)| / |E_hard(start)| (the pairs inside
 * a composite left out of E_hard(end)).  n_steps as p3t_hermite_cluster_step;
 * *n_collisions_host (nullable): mergers.  Synchronises. */
p3t_status p3t_hermite_collide(p3t_ctx *ctx, int64_t n, int64_t n_clusters, const int32_t *cl_ptr,
                               const int32_t *cl_members, double *pos3, double *vel3, const double *mass,
                               const double *r_out, double *dt_hard, double f_radius, double density,
                               int32_t *merged_into, double *eps6, double *e_rel_err, int32_t *n_steps,
                               int64_t *n_collisions_host);

/* The hard part with perfect-accretion collisions (Section 2.5.1): as
 * p3t_hard_step, and two bodies of a cluster collide when their distance is
 * below f_radius (R_i + R_j), R = (3 m / (4 pi density))^(1/3) in code units
 * (density > 0, f_radius >= 0, both finite; f_radius = 0 never collides).  The
 * colliding bodies become a composite that keeps the centre of mass and the
 * momentum; inside the hard part its parts stay separate particles (each
 * with its own r_out) that exchange no force and move with the mass-weighted
 * mean of their hard accelerations and jerks, and the dissipations of
 * eq. (e0) ... eq. (e3) are booked.  Readings: collisions are looked for at
 * every block step among the pairs evaluated there (at least one body due,
 * predicted states); the first pair in (lower, higher) slot order merges
 * after the corrector, one merger per block step; the composite's next step
 * comes from eta_0 and divides the block time; the neighbours of eq. (e3)
 * are the cluster's other members.  Clusters of 2..64 members look for
 * collisions (one wavefront each); larger clusters are integrated without
 * and set P3T_FLAG_COLL_UNCHECKED.
 * merged_into (n int32, device, required) receives for every particle the
 * lowest index of its composite (its own index if it did not merge).
 * eps_host (6 doubles, host, nullable): sums over all mergers of eps_0,
 * eps_1, eps_2, eps_3 (eq. (e0) ... eq. (e3), with W), of their total with
 * W replaced by one (the Newtonian energy lost, neighbours only) and with
 * 1 - W (the hard energy lost).  *n_collisions_host (nullable): number of
 * mergers.  Synchronises.  Pass the result to p3t_merge_bodies before the
 * next evaluation: the parts of a composite share one position. */
p3t_status p3t_hard_step_collide(p3t_ctx *ctx, double *pos3, double *vel3, const double *mass, const double *r_out,
                                 double *dt_hard, int32_t *steps, double f_radius, double density,
                                 int32_t *merged_into, double *eps_host, int64_t *n_collisions_host,
                                 int64_t *n_clusters_host);

/* Perfect accretion after p3t_hard_step_collide (Section 2.5.1): every
 * composite becomes one particle.  The part at the lowest index keeps the
 * shared state and takes the composite's mass (summed in index order); the
 * other parts are removed and the arrays are compacted in index order, in
 * place: afterwards pos3 / vel3 hold (3, n_new) with row stride n_new in
 * their first 3 n_new entries, mass, dt_hard (nullable) and steps (nullable)
 * their first n_new.  *n_new_host (required) receives the new count.
 * merged_into (n) must map every particle to the lowest index of its
 * composite, which maps to itself; anything else is P3T_ERR_ARG (checked
 * before anything is moved).  Invalidates the tree: the next call is an
 * evaluation with cut-off radii of the new set (Section 2.2, step (9)).
 * Synchronises. */
p3t_status p3t_merge_bodies(p3t_ctx *ctx, int64_t n, const int32_t *merged_into, double *pos3, double *vel3,
                            double *mass, double *dt_hard, int32_t *steps, int64_t *n_new_host);

/* p3t_build_tree followed by p3t_compute_soft_force in one call.  With
 * use_graph = 1 the whole device sequence (bounding box, Morton keys, radix
 * sort, gather, radix tree, moments, groups, walk, longest-first group order,
 * force kernels, neighbour candidates) is captured once into a hipGraph on a
 * private stream and replayed on later calls with the same n, pointers,
 * parameters and launch shapes; the counts that vary between calls (groups,
 * list lengths) stay on the device.  The call then synchronises once to read
 * the counters.  If a list, stack or pair buffer overflowed, the buffers grow
 * (which also retires the graph) and the force is redone eagerly, so the
 * result is always complete.  Phase times (p3t_get_stats) cover the graph as
 * a whole (ms_force) when timing is on.  Same arguments, ownership and errors
 * as the two calls it replaces; with use_graph = 0 it is exactly those. */
p3t_status p3t_evaluate(p3t_ctx *ctx, int64_t n, const double *pos3, const double *vel3, const double *mass,
                        const double *r_out, const double *r_search, double *acc3, int32_t use_graph);

/* p3t_hard_step followed by p3t_evaluate (Section 2.2, steps (4)-(7)), with
 * the long-running clusters taken off the critical path.  Every cluster of
 * up to min(cluster_cap, 1024) members that is still running after
 * 2^slow_log2 block steps saves its block-step state and stops ("parks"),
 * as long as the parked members fit in 1024 (otherwise all of them finish
 * before the evaluation, which is then the ordinary one; a percolated
 * cluster never parks); the parked members form S.  The
 * parked clusters then finish on a second stream, continuing exactly where
 * they stopped, while the tree, walk and soft force of Section 2.2 run at
 * the new state with the members of S given zero mass; after both finish,
 * S's final positions and velocities go into pos3 and vel3 and the soft
 * terms between S and every particle (eq. (softforce) with the changeover
 * at the pair cut-off, eq. (rout2)) are summed directly in FP64, with the
 * neighbour test of Section 2.3 for every pair that involves S.
 *   pos3, vel3 (3n, in/out), mass (n): as for p3t_hard_step; the state
 *     after the call is the one p3t_hard_step leaves, bit for bit.
 *   r_out_hard (n): the cut-offs of the hard part (those of the evaluation
 *     whose pairs form the clusters); r_out, r_search (n): those of the new
 *     evaluation (they may be the same arrays).
 *   dt_hard (n, in/out, nullable): carried hard steps, as for p3t_hard_step.
 *   steps (n, int32, out, nullable): block steps taken by each particle's
 *     cluster.
 *   acc3 (3n, out): the soft acceleration at the new state.  The neighbour
 *     pairs (p3t_neighbour_list) equal those of p3t_evaluate bit for bit; the
 *     forces differ from it only in that the terms involving S are exact
 *     rather than tree terms.
 *   slow_log2 <= 0: no budget, exactly p3t_hard_step + p3t_evaluate.
 *   use_graph: as for p3t_evaluate.  *n_clusters_host, *n_slow_host
 *     (nullable) receive the cluster count and |S|.
 * Errors as p3t_hard_step and p3t_evaluate; the state is advanced whenever
 * the hard part succeeded.  n is that of the last evaluation. */
p3t_status p3t_hard_evaluate(p3t_ctx *ctx, double *pos3, double *vel3, const double *mass, const double *r_out_hard,
                             double *dt_hard, int32_t *steps, const double *r_out, const double *r_search,
                             double *acc3, int32_t slow_log2, int32_t use_graph, int64_t *n_clusters_host,
                             int64_t *n_slow_host);

/* Total energy of the particles about the star, eq. (soft) + eq. (hard)
 * over all particles (Section 3.2.1 measures an integration's error by its
 * relative change).  The changeover weights of a pair add up to one, so this
 * is the Newtonian energy
 *   E = sum_i [m_i |v_i|^2 / 2 - G M_* m_i / |x_i|] - sum_{i<j} G m_i m_j / r_ij,
 * summed directly, O(N^2), in FP64 with compensated sums in a fixed order
 * (a diagnostic for runs of modest N; about 1e8 pairs per millisecond).
 * pos3, vel3 (3n), mass (n): device memory.  Synchronises and writes
 * *energy_host. */
p3t_status p3t_total_energy(p3t_ctx *ctx, int64_t n, const double *pos3, const double *vel3, const double *mass,
                            double *energy_host);

/* Soft force over the CURRENT tree topology and interaction lists at new
 * positions pos3 (3n) and masses mass (n), in the caller's order, with the
 * pair cut-offs of the last p3t_build_tree: the sorted positions and masses
 * are replaced, the cell moments recomputed, and every group is evaluated
 * over its existing lists (eq. (softforce), eq. (rout2)).  This is the
 * function whose derivative p3t_soft_kick_adjoint returns; it exists so that
 * finite differences and checkpointed recomputation see exactly the lists of
 * the forward pass.  Writes acc3 (3n).  Neighbour pairs are not collected:
 * p3t_neighbour_list keeps returning those of the last
 * p3t_compute_soft_force.  P3T_ERR_STATE without a prior
 * p3t_compute_soft_force. */
p3t_status p3t_soft_force_frozen(p3t_ctx *ctx, const double *pos3, const double *mass, double *acc3);

/* Vector-Jacobian product of the soft kick v' = v + h a(x, m) (eq.
 * (HamiltonSol), eq. (softforce)) at the state of the last force evaluation
 * (p3t_compute_soft_force or p3t_soft_force_frozen), with its interaction lists
 * and pair cut-offs r_out,ij held fixed.  For the cotangent lam_v3 (3n) of v'
 * it WRITES g_pos3 (3n) = h d(lam . a)/dx and g_mass (n) = h d(lam . a)/dm,
 * all in the caller's order (the cotangent of v itself is lam_v3 unchanged).
 * Cells enter as monopoles: the call returns P3T_ERR_STATE if the evaluation
 * used quadrupole cells (multipole = 2 with theta > 0).  Device memory; the
 * library allocates its scratch on the first call for a given size. */
p3t_status p3t_soft_kick_adjoint(p3t_ctx *ctx, double h, const double *lam_v3, double *g_pos3, double *g_mass);

/* Enable (1) / disable (0) event timing of the phases (p3t_stats). */
p3t_status p3t_set_timing(p3t_ctx *ctx, int32_t on);

/* Launch shapes of the soft-force kernels.  None of them changes what is
   computed beyond the order of floating-point summation; they exist so that an
   autotuner can pick the fastest shape for a workload.
     force_split      1: one kernel per interaction class (near with the
                      changeover and neighbour candidates, far particles,
                      cells) plus an exact-test kernel over the candidates;
                      0: one fused kernel.
     force_unroll     j-loop unroll of the split kernels: 1, 2, 4 or 8.
     force_persistent 1: persistent grids that take groups from a queue in
                      longest-list-first order; 0: one workgroup per group.
     waves_per_cu     persistent grid of the split kernels in wavefronts per
                      compute unit (1..64; capped by the kernel's occupancy).
     walk_waves_per_cu persistent grid of the walk (1..64).
     direct_pair_cap  capacity (pairs) of the neighbour-pair buffer of the
                      parked members' direct terms in p3t_hard_evaluate;
                      0 keeps the current one (initially 65,536).  When a
                      call finds more pairs, the buffer grows and the
                      evaluation is redone, so the result does not depend on
                      it; a small value lets a test reach that path.
     top_slots        entries of the LDS hash table that holds the arrival
                      counters of the tree's top climb (a power of two,
                      1..4096; 0 keeps the current one, initially 4096).
                      Nodes that find no free entry within 32 probes use a
                      counter in device memory; the moments do not depend on
                      the choice.
   Host memory; p3t_set_kernel_config rejects values outside these ranges
   with P3T_ERR_ARG and leaves the previous shape in place.  Zero-filled
   fields of a struct from p3t_get_kernel_config keep their meaning. */
typedef struct {
  int32_t force_split, force_unroll, force_persistent, waves_per_cu, walk_waves_per_cu;
  int32_t direct_pair_cap, top_slots;
  int32_t reserved[1];
} p3t_kernel_config;
p3t_status p3t_set_kernel_config(p3t_ctx *ctx, const p3t_kernel_config *cfg_host);
p3t_status p3t_get_kernel_config(p3t_ctx *ctx, p3t_kernel_config *cfg_host);
/* Counters and phase times of the last evaluation, as the host read them
 * when that call finished; does not wait for the device.  The time of a
 * p3t_compute_cutoffs still running is reported by a later call. */
p3t_status p3t_get_stats(p3t_ctx *ctx, p3t_stats *out_host);
/* Read and clear the device status word.  Synchronises. */
p3t_status p3t_get_status(p3t_ctx *ctx, uint32_t *flags_host);
/* Text of the last error on this context (static storage of the context);
 * with ctx = NULL, of the last failed p3t_compute_cutoffs_noalloc on the
 * calling thread. */
const char *p3t_last_error(p3t_ctx *ctx);

/* p3t_compute_cutoffs without a context and without allocating: for callers
 * that cannot call hipMalloc (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same radii as
 * p3t_compute_cutoffs with the same parameters, bit for bit: the passes
 * recompute each particle's cylindrical radius, random velocity and Hill
 * radius where they need them instead of keeping them in scratch, so the
 * only scratch (range partials, per-chunk bin sums, bin values) lives in a
 * file-scope device array of 8 MiB that every GPU the library runs on holds
 * until the process ends.
 *   p_host: parameters (validated as by p3t_create; host memory).
 *   pos3, vel3 (3n), mass (n): inputs; r_out, r_search (n), v_ran (n,
 *     nullable): outputs.  Device memory, caller-owned.
 *   hip_stream: a hipStream_t (NULL = the null stream); the call only
 *     enqueues kernels on it (no synchronisation, no memset).
 * Limit: the per-chunk bin sums take 2 ceil(n / 1024) vran_bins doubles;
 * inputs that need more than the 8 MiB (n above about 8.3 million at 64
 * bins) return P3T_ERR_CAPACITY and launch nothing.  The first call on a
 * device (n = 0 included) looks the array's address up with
 * hipGetSymbolAddress; make that call before capturing a graph.  All calls
 * on one GPU share its array: calls that overlap on one GPU (other streams,
 * other threads) race and give wrong radii.  Errors: P3T_ERR_ARG (null
 * parameters or pointers, invalid parameters, n < 0), P3T_ERR_CAPACITY,
 * P3T_ERR_HIP; text through p3t_last_error(NULL). */
p3t_status p3t_compute_cutoffs_noalloc(const p3t_params *p_host, int64_t n, const double *pos3, const double *vel3,
                                       const double *mass, double *r_out, double *r_search, double *v_ran,
                                       void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* P3T_H */
