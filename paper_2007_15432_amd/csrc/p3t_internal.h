// p3t_internal.h -- internal declarations of libp3t (not part of the ABI).
//
// Device layout (all library-owned scratch lives in one arena per context):
//   particles in Morton order, structure of arrays, FP64:
//     sx sy sz | svx svy svz | sm | sro (r_out) | sinv (1/r_out) | sreach (max(r_search, r_out)) | srs
//     sid (int32, original index)
//   tree: 2n-1 nodes (internal 0..n-2, leaf of sorted particle k = n-1+k)
//     WalkNode (AoS, 96 B): tight bbox, centre of mass, max reach, first, count, left, right
//     CellMom  (AoS, 80 B): centre of mass, mass, traceless quadrupole
//   groups: node ids of the interaction groups
//   lists: per group offsets into one pool of int32 entries (cells | near | far)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/p3t.h"

namespace p3t {

constexpr int WAVE = 64;

// ---------------------------------------------------------------- records
struct WalkNode {
  double lo[3];
  double hi[3];
  double com[3];
  double reach;  // max over members of max(r_search, r_out)
  int32_t first, count, left, right;
};
static_assert(sizeof(WalkNode) == 96, "WalkNode layout");

struct CellMom {
  double com[3];
  double mass;
  double q[6];  // xx, yy, zz, xy, xz, yz of sum m (3 s s^T - |s|^2 I), s about com
};
static_assert(sizeof(CellMom) == 80, "CellMom layout");

// per-group list descriptor
struct GroupList {
  int64_t off;      // offset of the group's entries in the pool
  int32_t n_cell;   // cells, then near particles, then far particles
  int32_t n_near;
  int32_t n_far;
  int32_t node;     // group node id
};
static_assert(sizeof(GroupList) == 24, "GroupList layout");

// device-side counters (one small struct in the arena)
struct DevCounters {
  unsigned int status;      // P3T_FLAG_* bits
  unsigned int status_d;    // bits of the parked members' direct terms (second stream, merged after the join)
  unsigned long long pool_cursor;  // list pool allocation cursor
  unsigned long long n_pairs;      // neighbour pairs appended
  unsigned long long n_groups;     // interaction groups
  unsigned long long walk_queue;   // persistent walk kernel queue head
  unsigned long long force_queue;  // persistent force kernel queue head
  unsigned long long n_near, n_far, n_cell;  // interaction counts
  unsigned long long n_clusters;
  unsigned long long n_chunks;     // subtree roots of the bottom-up moment pass
  unsigned long long queue[3];    // persistent queues of the split force kernels
  unsigned long long n_cand;      // neighbour candidates appended (split force)
  unsigned long long n_pairs_d;   // pairs of the parked members' direct terms (p3t_hard_evaluate)
  unsigned long long n_unbound;   // orbits that are not bound (p3t_kepler_drift)
  unsigned long long n_bad_index; // list entries outside [0, n) (p3t_kepler_drift)
  unsigned long long n_heval;     // Hermite: evaluations of members due in a block step (last hard part)
  unsigned long long n_hpair;     // Hermite: pair terms of those evaluations
  unsigned long long n_coll;      // Hermite: mergers of the last hard part with collisions
};

// ---------------------------------------------------------------- device helpers
// 1/sqrt(x) for a finite, positive, normal x: the hardware estimate
// (relative error below 2^-22) and one third-order correction
// y (1 + e/2 + 3e^2/8), e = 1 - x y^2, which leaves an error below an ulp.
// The library rsqrt adds selects for zero, infinite and denormal x; callers
// of this one never pass such an x (a non-finite input gives a NaN).
__device__ __forceinline__ double rsqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

__device__ __forceinline__ int popc_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0));
}

__device__ __forceinline__ void set_flag(DevCounters *c, unsigned bits) { atomicOr(&c->status, bits); }

// Wave-uniform values that steer loops (queue indices, list lengths, stack
// tops) must live in scalar registers.  A value broadcast with a shuffle is
// uniform at run time but not provably so to the compiler, which then
// compiles the loop exit as divergent and may re-enter the broadcast with its
// source lane switched off.  readfirstlane / readlane make uniformity explicit
// and turn such exits into scalar branches.
__device__ __forceinline__ int uniform_first(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int uniform_lane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ long long uniform_first64(long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v & 0xffffffffll));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ long long uniform_lane64(long long v, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)v >> 32), l);
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// The old value of *p after adding v (wave-uniform) once for the whole
// wavefront, returned to every lane.  Lane `from` alone issues the atomic:
// an atomic that every lane executes (the others adding zero) is expanded
// by the compiler into a scalar loop over the 64 lanes before the single
// memory operation.  Every lane of the wavefront must call it, with lane
// `from` active.
__device__ __forceinline__ unsigned long long wave_fetch_add(unsigned long long *p, unsigned long long v,
                                                             int from = 0) {
  unsigned long long r = 0;
  if ((int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)) == from) r = atomicAdd(p, v);
  return (unsigned long long)uniform_lane64((long long)r, from);
}

// inclusive wave scan of int
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int t = __shfl_up(v, o, WAVE);
    if (l >= o) v += t;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    T t = __shfl_xor(v, o, WAVE);
    v = t < v ? t : v;
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    T t = __shfl_xor(v, o, WAVE);
    v = t > v ? t : v;
  }
  return v;
}

// Hermite bucket-count words (hermite.hip): [0, 11) the buckets, [11, 21)
// the parked clusters of buckets 0..9, the parked member count, [22, 25)
// the clusters of buckets 1..3 with a close pair (listed at the end of
// their bucket's list, apart from the others), then the cluster count and
// the malformed-input flag.
constexpr int HERM_BC_PARK0 = 11, HERM_BC_PARKED = 21, HERM_BC_CLOSE0 = 22, HERM_BC_NC = 28, HERM_BC_BAD = 29,
              HERM_BC_WORDS = 32;
constexpr int HERM_N_BUCKETS = 11;
// A neighbour pair counts as close when its free-fall time scale
// sqrt(r^3 / G(m_i + m_j)) is below dt_soft / CLOSE_RATIO: nearly every
// cluster that takes hundreds of Hermite block steps holds one (mostly
// bound pairs), so the hard part dispatches such clusters first.  Only the
// order of the work depends on it.
constexpr double CLOSE_RATIO = 0.5;
// parked members of one p3t_hard_evaluate call at most, and the chunks of
// the direct sum over all particles for each of them
constexpr int SLOW_CAP = 1024, SLOW_CHUNKS = 2048;

// ---------------------------------------------------------------- context
struct Arena {
  char *base = nullptr;
  size_t size = 0, used = 0;
  template <typename T>
  T *take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (used + bytes > size) return nullptr;
    T *p = reinterpret_cast<T *>(base + used);
    used += bytes;
    return p;
  }
};

}  // namespace p3t

struct p3t_ctx {
  p3t_params P;
  hipStream_t stream = nullptr;
  int device = 0;
  int n_cu = 256;
  std::string last_error;
  int timing = 0;
  hipEvent_t ev[24] = {};
  p3t_stats stats = {};

  // capacities
  int64_t n_cap = 0;         // particles the arena is sized for
  int64_t pair_cap = 0;      // neighbour-pair buffer capacity
  int64_t pool_cap = 0;      // list pool entries
  int64_t slot_cap_list = 0; // per-slot temp list capacity (each of cells/near/far)
  int64_t slot_cap_stack = 0;
  int walk_slots = 0;

  // arena (particles, tree, groups, scratch) and separately grown buffers
  p3t::Arena arena;
  int32_t *pool = nullptr;          // list pool
  int32_t *slot_lists = nullptr;    // walk temp lists (walk_slots * 3 * slot_cap_list)
  int32_t *slot_stack = nullptr;    // walk stacks (walk_slots * slot_cap_stack)
  int2 *pairs = nullptr;            // neighbour pairs (i_orig, j_orig)
  int2 *cands = nullptr;            // neighbour candidates (sorted indices)
  int64_t cand_cap = 0;
  // The clusters of the next hard part (labels, cluster CSR, buckets) are
  // prepared on aux_stream right behind an evaluation's kernels, beside the
  // host's read of its counters and the kicks that follow; prep_state 2 =
  // enqueued before the counters were read, 1 = the evaluation needed no
  // retry and the preparation is valid for prep_n particles.  Every other
  // call first makes the main stream wait for it (the scratch is shared)
  // and drops it.
  int prep_state = 0;
  int prep_timed = 0;              // the preparation recorded its timing events
  int cut_timing_pending = 0;      // events 0 / 1 of p3t_compute_cutoffs not read yet
  int park_flags_valid = 0;        // slow_flag holds the members parked in the last hard part
  int64_t prep_n = 0;
  hipEvent_t prep_ev[2] = {};      // fork (main stream), done (aux stream)
  int32_t *hc_pinned = nullptr;    // bucket words, pinned host memory
  // collisions: per-cluster dissipations (6 per cluster) and their sums (6);
  // merging: staging rows (9 n) and int scratch (2 n + 1)
  double *coll_buf = nullptr;
  int64_t coll_cap = 0;
  double *merge_st = nullptr;
  int32_t *merge_i32 = nullptr;
  int64_t merge_cap = 0;

  // state
  int64_t n = 0;
  int64_t n_groups = 0;
  int64_t n_pairs = 0;
  bool tree_valid = false, force_valid = false;
  unsigned host_status = 0;   // accumulated device status bits (cleared by p3t_get_status)
  int force_slots = 0;        // persistent force grid
  int force_persistent = 1;
  int walk_waves_per_cu = 8;  // persistent walk grid
  int top_slots = 4096;       // LDS hash entries of the tree's top climb (power of two <= 4096)
  int64_t groups_hint = 0;    // group count of the last evaluation (bounds the next one's grids)
  int tree_timing_pending = 0;  // the last tree build recorded its events
  int graphed = 0;            // the last evaluation replayed the captured graph
  struct {
    int split = 1;         // 1: one kernel per interaction class, 0: the fused kernel
    int unroll = 4;        // j-loop unroll of the split kernels (1, 2, 4, 8)
    int waves_per_cu = 8;  // persistent grid of the split kernels: waves per CU (capped by occupancy)
  } fcfg;
  int32_t *herm_bcount = nullptr;  // Hermite bucket counts (p3t::HERM_BC_WORDS)
  int32_t *herm_blists = nullptr;  // Hermite bucket lists (11 * n_cap)
  int32_t *herm_clbk = nullptr;    // bucket of each cluster (n_cap)
  uint8_t *slow_flag = nullptr;    // member of a slow cluster (n_cap), p3t_hard_evaluate

  // arena pointers
  p3t::DevCounters *cnt = nullptr;
  double *bbox = nullptr;       // 6 doubles (+ partials)
  double *bbox_part = nullptr;
  double *sx = nullptr, *sy = nullptr, *sz = nullptr, *svx = nullptr, *svy = nullptr, *svz = nullptr;
  double *sm = nullptr, *sro = nullptr, *sinv = nullptr, *sreach = nullptr, *srs = nullptr;
  int32_t *sid = nullptr;
  uint64_t *keys = nullptr, *keys_alt = nullptr;
  int32_t *perm = nullptr, *perm_alt = nullptr;
  uint32_t *radix_hist = nullptr;
  int64_t radix_hist_cap = 0;
  int32_t *parent = nullptr;
  int32_t *visit = nullptr;
  p3t::WalkNode *wnode = nullptr;
  p3t::CellMom *cmom = nullptr;
  int32_t *group_flag = nullptr;
  int64_t *node_scan = nullptr;     // exclusive scan over nodes (2n)
  int32_t *group_node = nullptr;
  p3t::GroupList *glist = nullptr;
  int32_t *group_order = nullptr;   // groups sorted by work (longest first)
  int64_t *scan_tmp = nullptr;
  int64_t scan_tmp_cap = 0;
  int32_t *row_cnt = nullptr;       // per-particle counters (n)
  int64_t *csr_ptr = nullptr;       // internal CSR row pointer (n + 1)
  int32_t *csr_col = nullptr;       // internal CSR columns (pair_cap)
  int32_t *uf_parent = nullptr;     // union-find parents (n)
  int64_t uf_early = 0;             // n if uf_parent holds the first pass of labels_pairs_early, else 0
  uint64_t *cl_keys = nullptr, *cl_keys_alt = nullptr;  // cluster sort keys (n)
  double *cut_part = nullptr;       // cut-off bin partial sums
  uint8_t *close_flag = nullptr;    // per particle: in a close neighbour pair at the last evaluation
  int32_t *cut_bin = nullptr;       // cut-off radial bin of each particle (n; the cluster
                                    // preparation may use row_cnt at the same time)
  double *tmp_d = nullptr;          // per-particle FP64 scratch (3n)
  double *acc_s = nullptr;          // soft acceleration in sorted order (3n)
  // second stream for the big Hermite clusters, fork / join events
  hipStream_t aux_stream = nullptr;
  hipEvent_t aux_ev[2] = {};
  // captured evaluation graph (p3t_evaluate with use_graph = 1)
  hipStream_t cap_stream = nullptr;
  hipGraph_t g_graph = nullptr;
  hipGraphExec_t g_exec = nullptr;
  uint64_t g_key = 0;
  int32_t *hs_label = nullptr;      // p3t_hard_step: labels (n), cluster CSR (n + 1, n)
  int32_t *hs_cl_ptr = nullptr;
  int32_t *hs_cl_mem = nullptr;
  double *adj_buf = nullptr;        // soft-kick adjoint scratch (adjoint_buf_need(adj_cap))
  int64_t adj_cap = 0;
  // p3t_hard_evaluate: clusters parked by the step budget finish on
  // slow_stream while the tree of everyone else is evaluated on the main stream
  int slow_active = 0;              // force kernels leave pairs with a parked member alone
  hipStream_t slow_stream = nullptr;
  hipEvent_t slow_ev[3] = {};
  char *ov_buf = nullptr;           // one allocation for the pointers below
  int64_t ov_n_cap = 0;
  double *pk_x = nullptr, *pk_v = nullptr, *pk_a = nullptr, *pk_j = nullptr;  // parked state (3 n_cap each)
  int64_t *pk_t = nullptr;          // parked members' times (n_cap)
  int32_t *pk_lev = nullptr;        // parked members' levels (n_cap)
  int32_t *pk_nst = nullptr;        // parked clusters' step counts (n_cap)
  double *pk_e0 = nullptr;          // parked clusters' initial energies (n_cap)
  int32_t *pk_lists = nullptr;      // parked clusters per bucket (10 * n_cap)
  double *m_eff = nullptr;          // masses with the parked members at zero (n_cap)
  int32_t *slow_list = nullptr;     // parked members (SLOW_CAP)
  double *slow_part = nullptr;      // partial sums of the forces on the parked members
  double *acc_d = nullptr;          // the parked members' direct terms (3 n_cap)
  char *huge_buf = nullptr;         // member states of the percolated-cluster path (hermite.hip)
  size_t huge_bytes = 0;
  int2 *pairs_d = nullptr;          // their neighbour pairs (pairs_d_cap used of pairs_d_alloc)
  int64_t pairs_d_cap = 0, pairs_d_alloc = 0;
};

// ---------------------------------------------------------------- launchers
namespace p3t {

// util.hip
hipError_t scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, int64_t *tmp, int64_t tmp_cap,
                           hipStream_t s);  // out has n + 1 entries (exclusive, out[n] = total)
int64_t scan_tmp_need(int64_t n);
void reset_queues(p3t_ctx *c);  // queue heads and per-evaluation counters
hipError_t tree_moments(p3t_ctx *c, int64_t n);
hipError_t refresh_tree(p3t_ctx *c, const double *pos3, const double *mass);
hipError_t soft_kick_adjoint(p3t_ctx *c, double h, const double *lam_v3, double *g_pos3, double *g_mass);
int64_t adjoint_buf_need(int64_t n_cap);

// timing events of the context (recorded only when timing is on)
void ev_record(p3t_ctx *c, int k);
double ev_ms(p3t_ctx *c, int a, int b);
void cut_timing_read(p3t_ctx *c);

hipError_t radix_sort_pairs(uint64_t *&keys, int32_t *&vals, uint64_t *&keys_alt, int32_t *&vals_alt, int64_t n_static,
                            const unsigned long long *n_dev, int bit_lo, int bit_hi, uint32_t *hist, int64_t hist_cap,
                            int64_t *tmp, int64_t tmp_cap, hipStream_t s);
int64_t radix_hist_need(int64_t n);
hipError_t fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t fill_f64(double *p, double v, int64_t n, hipStream_t s);
hipError_t iota_i32(int32_t *p, int64_t n, hipStream_t s);
hipError_t bbox_reduce(const double *pos3, int64_t n, double *part, double *out, hipStream_t s);
hipError_t kick(int64_t n, double h, const double *acc3, double *vel3, hipStream_t s);
hipError_t kepler_drift(int64_t n, int64_t n_list, const int32_t *list, double mu, double dt, double *pos3,
                        double *vel3, int32_t *iters, DevCounters *cnt, hipStream_t s);
hipError_t kepler_singles(int64_t n, int32_t count, const int32_t *blist, const int32_t *cl_ptr,
                          const int32_t *members, double mu, double dt, double *pos3, double *vel3, double *dt_hard,
                          int32_t *msteps, double *e_rel, int32_t *nsteps, DevCounters *cnt, hipStream_t s);

// energy.hip: total energy into out[0] (share: n doubles of scratch)
hipError_t total_energy(int64_t n, const double *pos3, const double *vel3, const double *mass, double G, double GM,
                        double *share, double *out, hipStream_t s);

// cutoff.hip
int64_t cut_part_need(int64_t n_cap);
const char *noalloc_last_error();  // last failure of p3t_compute_cutoffs_noalloc on this thread
hipError_t compute_cutoffs(p3t_ctx *c, int64_t n, const double *pos3, const double *vel3, const double *mass,
                           double *r_out, double *r_search, double *v_ran);
hipError_t cutoffs_run(const p3t_params &P, int64_t n, const double *pos3, const double *vel3, const double *mass,
                       double *r_out, double *r_search, double *v_ran, double *tmp, int32_t *bin, double *part,
                       hipStream_t s);

// api.hip
const char *params_error(const p3t_params &P);  // why P is invalid, or nullptr
bool bad_ptr(const void *p, int64_t n);         // p is null while n > 0

// tree.hip
hipError_t build_tree(p3t_ctx *c, int64_t n, const double *pos3, const double *vel3, const double *mass,
                      const double *r_out, const double *r_search);

// walk.hip
hipError_t walk_groups(p3t_ctx *c, int64_t n_groups);

// force.hip
// frozen: no neighbour pairs or candidates are kept (evaluation over existing lists)
hipError_t soft_force(p3t_ctx *c, int64_t n_groups, double *acc3, bool frozen = false);

// nbr.hip
hipError_t build_csr(p3t_ctx *c, int64_t n, int64_t n_pairs);
hipError_t labels_cc(p3t_ctx *c, int64_t n, int32_t *label);
hipError_t labels_pairs(p3t_ctx *c, int64_t n, int32_t *label);
hipError_t labels_pairs_early(p3t_ctx *c, int64_t n);
hipError_t clusters_csr(p3t_ctx *c, int64_t n, const int32_t *label, int32_t *cl_ptr, int32_t *cl_members,
                        int64_t *n_clusters);
hipError_t clusters_csr_dev(p3t_ctx *c, int64_t n, const int32_t *label, int32_t *cl_ptr, int32_t *cl_members,
                            bool keys_ready = false);

// hermite.hip
// nc_dev (nullable): the cluster count on the device, nc then only bounds it
// Clusters of 2..8 members holding a member flagged in either array
// (nullable) are dispatched first (see CLOSE_RATIO).
struct CloseSrc {
  const uint8_t *a = nullptr, *b = nullptr;
};
hipError_t herm_bucket(p3t_ctx *c, int64_t n, int64_t nc, const int32_t *cl_ptr, const int32_t *cl_members,
                       const int64_t *nc_dev, int32_t *hc, const CloseSrc &close = CloseSrc());
// perfect-accretion collisions in the hard part (hermite.hip, wave path)
struct HermColl {
  double f;          // radius enhancement factor
  double r3;         // 3 / (4 pi rho): body radius = cbrt(r3 m)
  int32_t *merged;   // per particle: lowest index of its composite (identity on entry)
  double *ceps;      // per cluster: six dissipation sums (zeroed on entry)
};
// reset_work: also zero the Hermite work counters (n_heval, n_hpair,
// n_coll); a preparation enqueued before the last evaluation's counters are
// read leaves them, and herm_reset_work zeroes them when the hard part starts
hipError_t herm_bucket_enqueue(p3t_ctx *c, hipStream_t s, int64_t n, int64_t nc, const int32_t *cl_ptr,
                               const int32_t *cl_members, const int64_t *nc_dev, int32_t *hc, bool reset_work = true,
                               const CloseSrc &close = CloseSrc());
hipError_t herm_reset_work(p3t_ctx *c, hipStream_t s);
hipError_t herm_launch(p3t_ctx *c, int64_t n, int64_t stride, const int32_t *cl_ptr, const int32_t *cl_members,
                       double *pos3, double *vel3, const double *mass, const double *r_out, double *dt_hard,
                       double *e_rel_err, int32_t *n_steps, int32_t *steps_out, const int32_t *hc, int budget,
                       int resume, hipStream_t s, hipStream_t s_big, hipEvent_t ev_fork, hipEvent_t ev_join,
                       const HermColl *coll = nullptr);
// merge.hip: the composites of a hard part with collisions become single
// particles (see p3t_merge_bodies)
hipError_t merge_bodies(p3t_ctx *c, int64_t n, const int32_t *merged, double *pos3, double *vel3, double *mass,
                        double *dt_hard, int32_t *steps, int64_t *n_new);
hipError_t sum_rows6(int64_t nc, const double *rows, double *out6, hipStream_t s);
hipError_t aux_streams(p3t_ctx *c);
// slow.hip: the direct terms of the parked members after their integration
// the direct terms of S on stream s, into acc_d / pairs_d (pos3, vel3: the
// state of everyone else; S's from the park buffers)
hipError_t slow_direct(p3t_ctx *c, const double *pos3, const double *vel3, const double *mass, const double *r_out,
                       const double *r_search, int ns, hipStream_t s);
// after the join, on the main stream: S's state into pos3 / vel3, and (acc3
// not null) the direct terms into acc3 and their pairs behind the others
hipError_t slow_merge(p3t_ctx *c, double *pos3, double *vel3, double *acc3, int ns);
// the parked members' list in ascending order, before the direct terms
hipError_t slow_sort(p3t_ctx *c, int ns, hipStream_t s);
hipError_t slow_prepare(p3t_ctx *c, const double *mass, int ns);
hipError_t hermite_clusters(p3t_ctx *c, int64_t n, int64_t nc, const int32_t *cl_ptr, const int32_t *cl_members,
                            double *pos3, double *vel3, const double *mass, const double *r_out, double *dt_hard,
                            double *e_rel_err, int32_t *n_steps, const int64_t *nc_dev = nullptr,
                            int64_t *nc_out = nullptr, int32_t *steps_out = nullptr, const HermColl *coll = nullptr);

}  // namespace p3t
