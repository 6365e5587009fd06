// api.hip -- the C ABI of libp3t (declared in include/p3t.h): context and
// scratch management, argument checking, capacity growth and retry, phase
// timing and status reporting.  All compute runs in the kernels of the other
// translation units; this file only orders launches on the context's stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <new>

#include "p3t_internal.h"

using namespace p3t;

namespace {

constexpr unsigned NUMERIC_BITS =
    P3T_FLAG_COINCIDENT | P3T_FLAG_NAN | P3T_FLAG_KMAX | P3T_FLAG_NSTEPS | P3T_FLAG_UNBOUND;
constexpr unsigned RETRY_BITS =
    P3T_FLAG_LIST_OVERFLOW | P3T_FLAG_STACK_OVERFLOW | P3T_FLAG_PAIR_OVERFLOW | P3T_FLAG_GROUP_BOUND;

p3t_status fail(p3t_ctx *c, p3t_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
p3t_status fail(p3t_ctx *c, p3t_status st, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->last_error = buf;
  }
  return st;
}

#define HIP_OK(c, expr)                                                                              \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess) return fail((c), P3T_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

const char *check_params(const p3t_params &P) {
  if (!(P.gamma > 0.0 && P.gamma < 1.0)) return "gamma must lie in (0, 1)";
  if (!(P.G >= 0.0) || !(P.m_star >= 0.0)) return "G and m_star must be >= 0";
  if (!(P.r_cut0 >= 0.0) || !(P.r_cut1 >= 0.0)) return "r_cut0, r_cut1 must be >= 0";
  if (!(P.r_search0 >= 0.0) || !(P.r_search1 >= 0.0) || !(P.r_search2 >= 0.0) || !(P.r_search3 >= 0.0))
    return "r_search0..3 must be >= 0";
  if (!(P.dt_soft > 0.0) || !std::isfinite(P.dt_soft)) return "dt_soft must be > 0";
  if (!(P.theta >= 0.0) || !std::isfinite(P.theta)) return "theta must be >= 0";
  if (!(P.eta > 0.0) || !(P.eta0 > 0.0)) return "eta, eta0 must be > 0";
  if (P.multipole != 1 && P.multipole != 2) return "multipole must be 1 or 2";
  if (P.precision != 0 && P.precision != 1) return "precision must be 0 or 1";
  if (P.cutoff_mode != 0 && P.cutoff_mode != 1) return "cutoff_mode must be 0 or 1";
  if (P.hill_length != 0 && P.hill_length != 1) return "hill_length must be 0 or 1";
  if (P.n_group_max < 1 || P.n_group_max > 128) return "n_group_max must be in [1, 128]";
  if (P.n_leaf_max < 1 || P.n_leaf_max > 256) return "n_leaf_max must be in [1, 256]";
  if (P.vran_bins < 1 || P.vran_bins > 256) return "vran_bins must be in [1, 256]";
  if (P.vran_min_count < 1) return "vran_min_count must be >= 1";
  if (P.k_max < 0 || P.k_max > 40) return "k_max must be in [0, 40]";
  if (P.cluster_cap < 1) return "cluster_cap must be >= 1";
  if (P.isolated != 0 && P.isolated != 1) return "isolated must be 0 or 1";
  return nullptr;
}

template <typename T>
hipError_t dev_alloc(T *&p, int64_t count) {
  if (p) {
    hipError_t e = hipFree(p);
    p = nullptr;
    if (e != hipSuccess) return e;
  }
  if (count <= 0) count = 1;
  return hipMalloc((void **)&p, (size_t)count * sizeof(T));
}

// (re)allocate the arena for n_cap particles
p3t_status alloc_arena(p3t_ctx *c, int64_t n_cap) {
  if (n_cap < 1024) n_cap = 1024;
  const int64_t n2 = 2 * n_cap;
  auto bytes = [](int64_t count, size_t sz) { return ((size_t)count * sz + 255) & ~size_t(255); };
  const int64_t hist = radix_hist_need(n_cap);
  const int64_t stmp = scan_tmp_need(std::max<int64_t>(n2 + 1, hist));
  size_t total = 0;
  total += bytes(1, sizeof(DevCounters));
  total += bytes(8 + 6 * 1024, sizeof(double));
  total += 11 * bytes(n_cap, sizeof(double));
  total += bytes(n_cap, sizeof(int32_t));                          // sid
  total += 2 * bytes(n_cap, sizeof(uint64_t)) + 2 * bytes(n_cap, sizeof(int32_t));  // keys, perm
  total += bytes(hist, sizeof(uint32_t));
  total += bytes(stmp, sizeof(int64_t));
  total += bytes(n2, sizeof(int32_t)) + bytes(n_cap, sizeof(int32_t));  // parent, visit
  total += bytes(n2, sizeof(WalkNode)) + bytes(n2, sizeof(CellMom));
  total += bytes(n2, sizeof(int32_t)) + bytes(n2 + 1, sizeof(int64_t));  // group_flag, node_scan
  total += bytes(n_cap, sizeof(int32_t));                               // group_node
  total += bytes(n_cap, sizeof(GroupList));
  total += bytes(n_cap, sizeof(int32_t));                                           // group order
  total += bytes(n_cap, sizeof(int32_t)) + bytes(n_cap + 1, sizeof(int64_t));       // row_cnt, csr_ptr
  total += bytes(n_cap, sizeof(int32_t)) + 2 * bytes(n_cap, sizeof(uint64_t));      // uf, cl keys
  total += bytes(cut_part_need(n_cap), sizeof(double)) + bytes(n_cap, sizeof(int32_t));  // cut-off bins
  total += bytes(n_cap + 4, sizeof(uint8_t));                                                // close flags
  total += 2 * bytes(3 * n_cap, sizeof(double));
  total += bytes(HERM_BC_WORDS, sizeof(int32_t)) + bytes(HERM_N_BUCKETS * n_cap, sizeof(int32_t));  // buckets
  total += bytes(n_cap, sizeof(int32_t)) + bytes(n_cap, sizeof(uint8_t));  // cluster buckets, slow flags
  total += 3 * bytes(n_cap + 1, sizeof(int32_t));                             // hard-step labels, clusters
  total += 4096;
  if (c->prep_state) {  // a cluster preparation may still use the old arena
    HIP_OK(c, hipEventSynchronize(c->prep_ev[1]));
    c->prep_state = 0;
  }
  if (c->arena.base) {
    HIP_OK(c, hipFree(c->arena.base));
    c->arena.base = nullptr;
  }
  HIP_OK(c, hipMalloc((void **)&c->arena.base, total));
  c->arena.size = total;
  c->arena.used = 0;
  Arena &A = c->arena;
  c->cnt = A.take<DevCounters>(1);
  c->bbox = A.take<double>(8 + 6 * 1024);
  c->bbox_part = c->bbox + 8;
  double **soa[11] = {&c->sx, &c->sy, &c->sz, &c->svx, &c->svy, &c->svz, &c->sm, &c->sro, &c->sinv, &c->sreach, &c->srs};
  for (auto p : soa) *p = A.take<double>(n_cap);
  c->sid = A.take<int32_t>(n_cap);
  c->keys = A.take<uint64_t>(n_cap);
  c->keys_alt = A.take<uint64_t>(n_cap);
  c->perm = A.take<int32_t>(n_cap);
  c->perm_alt = A.take<int32_t>(n_cap);
  c->radix_hist = A.take<uint32_t>(hist);
  c->radix_hist_cap = hist;
  c->scan_tmp = A.take<int64_t>(stmp);
  c->scan_tmp_cap = stmp;
  c->parent = A.take<int32_t>(n2);
  c->visit = A.take<int32_t>(n_cap);
  c->wnode = A.take<WalkNode>(n2);
  c->cmom = A.take<CellMom>(n2);
  c->group_flag = A.take<int32_t>(n2);
  c->node_scan = A.take<int64_t>(n2 + 1);
  c->group_node = A.take<int32_t>(n_cap);
  c->glist = A.take<GroupList>(n_cap);
  c->group_order = A.take<int32_t>(n_cap);
  c->row_cnt = A.take<int32_t>(n_cap);
  c->csr_ptr = A.take<int64_t>(n_cap + 1);
  c->uf_parent = A.take<int32_t>(n_cap);
  c->cl_keys = A.take<uint64_t>(n_cap);
  c->cl_keys_alt = A.take<uint64_t>(n_cap);
  c->cut_part = A.take<double>(cut_part_need(n_cap));
  c->cut_bin = A.take<int32_t>(n_cap);
  c->close_flag = A.take<uint8_t>(n_cap + 4);
  c->tmp_d = A.take<double>(3 * n_cap);
  c->acc_s = A.take<double>(3 * n_cap);
  c->herm_bcount = A.take<int32_t>(HERM_BC_WORDS);
  c->herm_blists = A.take<int32_t>(HERM_N_BUCKETS * n_cap);
  c->herm_clbk = A.take<int32_t>(n_cap);
  c->slow_flag = A.take<uint8_t>(n_cap);
  c->hs_label = A.take<int32_t>(n_cap + 1);
  c->hs_cl_ptr = A.take<int32_t>(n_cap + 1);
  c->hs_cl_mem = A.take<int32_t>(n_cap + 1);
  if (!c->hs_cl_mem) return fail(c, P3T_ERR_HIP, "arena layout overflow (internal)");
  HIP_OK(c, hipMemsetAsync(c->cnt, 0, sizeof(DevCounters), c->stream));
  c->n_cap = n_cap;
  c->tree_valid = c->force_valid = false;
  c->park_flags_valid = 0;
  return P3T_OK;
}

p3t_status ensure_n(p3t_ctx *c, int64_t n) {
  if (n <= c->n_cap) return P3T_OK;
  return alloc_arena(c, std::max<int64_t>(n, c->n_cap + c->n_cap / 2));
}

p3t_status ensure_lists(p3t_ctx *c, int64_t n) {
  if (!c->pool || c->pool_cap < std::max<int64_t>(1 << 20, 32 * n)) {
    const int64_t cap = std::max<int64_t>(1 << 20, 64 * n);
    HIP_OK(c, dev_alloc(c->pool, cap));
    c->pool_cap = cap;
  }
  if (!c->slot_lists) {
    c->walk_slots = c->n_cu * c->walk_waves_per_cu;
    if (c->slot_cap_list == 0) c->slot_cap_list = 16384;
    if (c->slot_cap_stack == 0) c->slot_cap_stack = 8192;
    HIP_OK(c, dev_alloc(c->slot_lists, (int64_t)c->walk_slots * 3 * c->slot_cap_list));
    HIP_OK(c, dev_alloc(c->slot_stack, (int64_t)c->walk_slots * c->slot_cap_stack));
  }
  if (!c->pairs) {
    const int64_t cap = std::max<int64_t>(1 << 16, 2 * n);
    HIP_OK(c, dev_alloc(c->pairs, cap));
    HIP_OK(c, dev_alloc(c->csr_col, cap));
    c->pair_cap = cap;
  }
  if (!c->cands) {
    const int64_t cap = std::max<int64_t>(1 << 16, 8 * n);
    HIP_OK(c, dev_alloc(c->cands, cap));
    c->cand_cap = cap;
  }
  return P3T_OK;
}

p3t_status sync_counters(p3t_ctx *c, DevCounters *h) {
  HIP_OK(c, hipMemcpyAsync(h, c->cnt, sizeof(DevCounters), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return P3T_OK;
}

// Makes the main stream wait for a pending cluster preparation (its scratch
// is shared with every other call) and drops it.
void prep_join(p3t_ctx *c) {
  if (c->prep_state) {
    // if the stream cannot be made to wait, the host waits instead
    if (hipStreamWaitEvent(c->stream, c->prep_ev[1], 0) != hipSuccess) (void)hipEventSynchronize(c->prep_ev[1]);
    c->prep_state = 0;
  }
}

// Waits (host) for a pending cluster preparation and drops it: before
// scratch it reads is grown or freed.
void prep_drop_sync(p3t_ctx *c) {
  if (c->prep_state) {
    (void)hipEventSynchronize(c->prep_ev[1]);
    c->prep_state = 0;
  }
}

// The member flags of the close-first dispatch order (close pairs of the
// last evaluation, members parked in the last hard part).
CloseSrc close_src(p3t_ctx *c) {
  CloseSrc f;
  f.a = c->close_flag;
  f.b = c->park_flags_valid ? c->slow_flag : nullptr;
  return f;
}

// Enqueues on aux_stream, right behind the evaluation just enqueued on the
// main stream and before its counters are read, the clusters of the next
// hard part: labels straight from the pair list (its length read on the
// device), the cluster CSR and the bucket words (copied to pinned host
// memory).  It runs while the host reads the counters and enqueues the
// kicks and radii that follow; eval_finish keeps it (prep_confirm) when the
// evaluation needs no retry.  p3t_hard_step / p3t_hard_evaluate take the
// result instead of computing it.
p3t_status prep_enqueue(p3t_ctx *c) {
  const int64_t n = c->n;
  if (c->prep_state) prep_join(c);
  if (n <= 0 || !c->pairs) return P3T_OK;
  HIP_OK(c, aux_streams(c));
  if (!c->prep_ev[0])
    for (auto &ev : c->prep_ev) HIP_OK(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  if (!c->hc_pinned) HIP_OK(c, hipHostMalloc((void **)&c->hc_pinned, sizeof(int32_t) * HERM_BC_WORDS));
  HIP_OK(c, hipEventRecord(c->prep_ev[0], c->stream));
  HIP_OK(c, hipStreamWaitEvent(c->aux_stream, c->prep_ev[0], 0));
  struct Swap {  // the cluster functions enqueue on c->stream
    p3t_ctx *c;
    hipStream_t main;
    ~Swap() { c->stream = main; }
  } swap{c, c->stream};
  c->stream = c->aux_stream;
  ev_record(c, 20);
  HIP_OK(c, labels_pairs(c, n, c->hs_label));
  HIP_OK(c, clusters_csr_dev(c, n, c->hs_label, c->hs_cl_ptr, c->hs_cl_mem, true));
  // clusters with a close pair at this evaluation, or with a member parked
  // in the last hard part, are dispatched first
  const CloseSrc close = close_src(c);
  // the work counters of the hard part just finished are read after this
  // is enqueued: prep_take zeroes them instead
  HIP_OK(c, herm_bucket_enqueue(c, c->aux_stream, n, n, c->hs_cl_ptr, c->hs_cl_mem, c->node_scan + n, c->hc_pinned,
                                false, close));
  ev_record(c, 21);
  HIP_OK(c, hipEventRecord(c->prep_ev[1], c->aux_stream));
  c->prep_state = 2;
  c->prep_n = n;
  c->prep_timed = c->timing;
  return P3T_OK;
}

// The prepared clusters for n particles, if any: the main stream waits for
// them, the work counters of the new hard part are zeroed and hc receives
// the bucket words (returns false otherwise, after dropping a preparation
// that does not apply).
bool prep_take(p3t_ctx *c, int64_t n, int32_t *hc) {
  if (c->prep_state != 1 || c->prep_n != n) {
    prep_join(c);
    return false;
  }
  // the host waits for the preparation (it reads the bucket words), which
  // also orders everything enqueued after this behind it
  if (hipEventSynchronize(c->prep_ev[1]) != hipSuccess || herm_reset_work(c, c->stream) != hipSuccess) {
    c->prep_state = 0;
    return false;
  }
  for (int k = 0; k < HERM_BC_WORDS; ++k) hc[k] = c->hc_pinned[k];
  c->prep_state = 0;
  c->stats.ms_clusters = (c->timing && c->prep_timed) ? ev_ms(c, 20, 21) : 0.0;
  return true;
}

// atomic: a kernel on another stream may be setting bits at the same time
__global__ void k_clear_bits(DevCounters *cnt, unsigned bits) { atomicAnd(&cnt->status, ~bits); }

// move numeric bits from the device word into the host-side word
p3t_status harvest_status(p3t_ctx *c, unsigned *new_bits) {
  DevCounters h;
  p3t_status st = sync_counters(c, &h);
  if (st != P3T_OK) return st;
  const unsigned bits = h.status;
  c->stats.n_heval = (int64_t)h.n_heval;
  c->stats.n_hpair = (int64_t)h.n_hpair;
  if (bits) hipLaunchKernelGGL(k_clear_bits, dim3(1), dim3(1), 0, c->stream, c->cnt, bits);
  c->host_status |= bits;
  if (new_bits) *new_bits = bits;
  return P3T_OK;
}

}  // namespace

namespace p3t {
void ev_record(p3t_ctx *c, int k) {
  if (c->timing) (void)hipEventRecord(c->ev[k], c->stream);  // timing only: a failure costs a phase time
}
double ev_ms(p3t_ctx *c, int a, int b) {
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) != hipSuccess) {
    (void)hipGetLastError();  // an event not recorded: no time, and no error left behind for the next check
    return 0.0;
  }
  return ms;
}

// The cut-off radii's event time, once their end event has completed (a
// later call picks it up otherwise).
void cut_timing_read(p3t_ctx *c) {
  if (!c->cut_timing_pending || !c->ev[1]) return;
  if (hipEventQuery(c->ev[1]) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  c->stats.ms_cutoffs = ev_ms(c, 0, 1);
  c->cut_timing_pending = 0;
}

bool bad_ptr(const void *p, int64_t n) { return n > 0 && p == nullptr; }

const char *params_error(const p3t_params &P) { return check_params(P); }

}  // namespace p3t

extern "C" {

void p3t_default_params(p3t_params *P) {
  if (!P) return;
  std::memset(P, 0, sizeof(*P));
  P->G = 1.0;
  P->m_star = 1.0;
  P->gamma = 0.1;
  P->r_cut0 = 2.0;
  P->r_cut1 = 8.0;
  P->r_search0 = 1.1;
  P->r_search1 = 6.0;
  P->r_search2 = 2.0;
  P->r_search3 = 2.0;
  P->dt_soft = 2.0 * M_PI / 64.0;
  P->theta = 0.5;
  P->eta = 0.01;
  P->eta0 = 0.001;
  P->multipole = 2;
  P->precision = 0;
  P->cutoff_mode = 0;
  P->hill_length = 0;
  P->n_group_max = 128;
  P->n_leaf_max = 16;
  P->vran_bins = 64;
  P->vran_min_count = 8;
  P->k_max = 40;
  P->cluster_cap = 1024;
  P->isolated = 0;
}

namespace {

void drop_graph(p3t_ctx *c) {
  if (c->g_exec) (void)hipGraphExecDestroy(c->g_exec);
  if (c->g_graph) (void)hipGraphDestroy(c->g_graph);
  c->g_exec = nullptr;
  c->g_graph = nullptr;
  c->g_key = 0;
}

uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
  return h;
}

// Everything a captured evaluation bakes into its kernel arguments.
uint64_t graph_key(const p3t_ctx *c, int64_t n, const void *const *ptrs, int np) {
  uint64_t h = mix(0x51ed270b27a1c3ull, (uint64_t)n);
  for (int k = 0; k < np; ++k) h = mix(h, (uint64_t)(uintptr_t)ptrs[k]);
  const void *own[] = {c->arena.base, c->pool, c->slot_lists, c->slot_stack, c->pairs, c->cands, c->csr_col};
  for (const void *q : own) h = mix(h, (uint64_t)(uintptr_t)q);
  const int64_t caps[] = {c->n_cap, c->pool_cap, c->slot_cap_list, c->slot_cap_stack, c->pair_cap, c->cand_cap,
                          c->walk_slots, c->fcfg.split, c->fcfg.unroll, c->fcfg.waves_per_cu, c->force_persistent,
                          c->top_slots};
  for (int64_t v : caps) h = mix(h, (uint64_t)v);
  h = mix(h, (uint64_t)c->slow_active);
  const unsigned char *pb = reinterpret_cast<const unsigned char *>(&c->P);
  for (size_t k = 0; k < sizeof(p3t_params); ++k) h = mix(h, pb[k]);
  return h;
}

}  // namespace

p3t_status p3t_create(const p3t_params *p, void *stream, p3t_ctx **out) {
  if (!p || !out) return P3T_ERR_ARG;
  *out = nullptr;
  const char *why = check_params(*p);
  if (why) return P3T_ERR_ARG;
  p3t_ctx *c = new (std::nothrow) p3t_ctx();
  if (!c) return P3T_ERR_HIP;
  c->P = *p;
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return P3T_ERR_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess && prop.multiProcessorCount > 0)
    c->n_cu = prop.multiProcessorCount;
  c->force_slots = c->n_cu * 16;
  c->force_persistent = 1;
  for (auto &e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      delete c;
      return P3T_ERR_HIP;
    }
  if (alloc_arena(c, 1024) != P3T_OK) {
    delete c;
    return P3T_ERR_HIP;
  }
  *out = c;
  return P3T_OK;
}

p3t_status p3t_destroy(p3t_ctx *c) {
  if (!c) return P3T_ERR_ARG;
  // teardown: errors are ignored, every resource is released regardless
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->aux_stream) (void)hipStreamSynchronize(c->aux_stream);
  if (c->aux_stream) (void)hipStreamDestroy(c->aux_stream);
  for (auto &ev : c->aux_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (c->slow_stream) (void)hipStreamSynchronize(c->slow_stream);
  if (c->slow_stream) (void)hipStreamDestroy(c->slow_stream);
  for (auto &ev : c->slow_ev)
    if (ev) (void)hipEventDestroy(ev);
  void *bufs[] = {c->arena.base, c->pool,    c->slot_lists, c->slot_stack, c->pairs,
                  c->csr_col,    c->cands,   c->adj_buf,    c->ov_buf,     c->pairs_d,
                  c->huge_buf,   c->coll_buf, c->merge_st,  c->merge_i32};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  for (auto &e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : c->prep_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->hc_pinned) (void)hipHostFree(c->hc_pinned);
  delete c;
  return P3T_OK;
}

p3t_status p3t_set_stream(p3t_ctx *c, void *stream) {
  if (!c) return P3T_ERR_ARG;
  // a pending cluster preparation stays valid: every later call makes the
  // (new) stream wait for it before using its scratch
  c->stream = (hipStream_t)stream;
  return P3T_OK;
}

p3t_status p3t_set_params(p3t_ctx *c, const p3t_params *p) {
  if (!c || !p) return fail(c, P3T_ERR_ARG, "null argument");
  prep_join(c);
  const char *why = check_params(*p);
  if (why) return fail(c, P3T_ERR_ARG, "%s", why);
  c->P = *p;
  c->tree_valid = c->force_valid = false;
  return P3T_OK;
}

p3t_status p3t_get_params(p3t_ctx *c, p3t_params *p) {
  if (!c || !p) return P3T_ERR_ARG;
  *p = c->P;
  return P3T_OK;
}

p3t_status p3t_reserve(p3t_ctx *c, int64_t n_max, int64_t nnz_max) {
  if (!c || n_max < 0 || nnz_max < 0) return fail(c, P3T_ERR_ARG, "reserve: bad argument");
  prep_join(c);
  p3t_status st = ensure_n(c, n_max);
  if (st != P3T_OK) return st;
  if ((st = ensure_lists(c, n_max)) != P3T_OK) return st;
  if (nnz_max > c->pair_cap) {
    HIP_OK(c, dev_alloc(c->pairs, nnz_max));
    HIP_OK(c, dev_alloc(c->csr_col, nnz_max));
    c->pair_cap = nnz_max;
    c->force_valid = false;
  }
  return P3T_OK;
}

p3t_status p3t_compute_cutoffs(p3t_ctx *c, int64_t n, const double *pos3, const double *vel3, const double *mass,
                               double *r_out, double *r_search, double *v_ran) {
  if (!c) return P3T_ERR_ARG;
  if (n < 0 || n > (int64_t(1) << 30)) return fail(c, P3T_ERR_ARG, "compute_cutoffs: n out of range");
  if (bad_ptr(pos3, n) || bad_ptr(vel3, n) || bad_ptr(mass, n) || bad_ptr(r_out, n) || bad_ptr(r_search, n))
    return fail(c, P3T_ERR_ARG, "compute_cutoffs: null pointer");
  if (n == 0) return P3T_OK;
  p3t_status st = ensure_n(c, n);
  if (st != P3T_OK) return st;
  ev_record(c, 0);
  HIP_OK(c, compute_cutoffs(c, n, pos3, vel3, mass, r_out, r_search, v_ran));
  ev_record(c, 1);
  // read once the radii are done (cut_timing_read), not waited for here:
  // the host goes on to enqueue what follows
  if (c->timing) c->cut_timing_pending = 1;
  return P3T_OK;
}

p3t_status p3t_build_tree(p3t_ctx *c, int64_t n, const double *pos3, const double *vel3, const double *mass,
                          const double *r_out, const double *r_search) {
  if (!c) return P3T_ERR_ARG;
  prep_join(c);
  if (n < 0 || n > (int64_t(1) << 30)) return fail(c, P3T_ERR_ARG, "build_tree: n out of range");
  if (bad_ptr(pos3, n) || bad_ptr(vel3, n) || bad_ptr(mass, n) || bad_ptr(r_out, n) || bad_ptr(r_search, n))
    return fail(c, P3T_ERR_ARG, "build_tree: null pointer");
  c->tree_valid = c->force_valid = false;
  c->n = n;
  if (n == 0) {
    c->tree_valid = true;
    return P3T_OK;
  }
  p3t_status st = ensure_n(c, n);
  if (st != P3T_OK) return st;
  if ((st = ensure_lists(c, n)) != P3T_OK) return st;
  ev_record(c, 2);
  HIP_OK(c, build_tree(c, n, pos3, vel3, mass, r_out, r_search));
  ev_record(c, 3);
  // No synchronisation: the group count stays on the device.  The host
  // keeps a bound for the grid sizes (twice the last count, or n); a larger
  // count sets P3T_FLAG_GROUP_BOUND and the walk and force are redone.
  c->n_groups = c->groups_hint > 0 ? std::min<int64_t>(n, 2 * c->groups_hint + 1024) : n;
  c->tree_timing_pending = c->timing;
  c->stats.n = n;
  c->stats.n_nodes = 2 * n - 1;
  c->tree_valid = true;
  return P3T_OK;
}

// Clears the retry bits and grows whatever overflowed in the last walk/force.
p3t_status grow_for_retry(p3t_ctx *c, const DevCounters &h) {
  const unsigned retry = h.status & RETRY_BITS;
  hipLaunchKernelGGL(k_clear_bits, dim3(1), dim3(1), 0, c->stream, c->cnt, RETRY_BITS);
  if (retry & P3T_FLAG_LIST_OVERFLOW) {
    if ((int64_t)h.pool_cursor > c->pool_cap) {
      const int64_t cap = (int64_t)h.pool_cursor + (int64_t)h.pool_cursor / 4 + 1024;
      HIP_OK(c, dev_alloc(c->pool, cap));
      c->pool_cap = cap;
    } else {
      c->slot_cap_list *= 2;
      HIP_OK(c, dev_alloc(c->slot_lists, (int64_t)c->walk_slots * 3 * c->slot_cap_list));
    }
  }
  if (retry & P3T_FLAG_STACK_OVERFLOW) {
    c->slot_cap_stack *= 2;
    HIP_OK(c, dev_alloc(c->slot_stack, (int64_t)c->walk_slots * c->slot_cap_stack));
  }
  if (retry & P3T_FLAG_GROUP_BOUND) {  // more groups than the bound: every group this time
    c->n_groups = c->n;
    c->groups_hint = 0;
  }
  if (retry & P3T_FLAG_PAIR_OVERFLOW) {
    if ((int64_t)h.n_pairs > c->pair_cap) {
      const int64_t cap = (int64_t)h.n_pairs + (int64_t)h.n_pairs / 4 + 1024;
      HIP_OK(c, dev_alloc(c->pairs, cap));
      HIP_OK(c, dev_alloc(c->csr_col, cap));
      c->pair_cap = cap;
    }
    if ((int64_t)h.n_cand > c->cand_cap) {
      const int64_t cap = (int64_t)h.n_cand + (int64_t)h.n_cand / 4 + 1024;
      HIP_OK(c, dev_alloc(c->cands, cap));
      c->cand_cap = cap;
    }
  }
  return P3T_OK;
}

namespace {
bool eval_finish(p3t_ctx *c, const DevCounters &h, unsigned *num, p3t_status *st);
}

p3t_status p3t_compute_soft_force(p3t_ctx *c, double *acc3) {
  if (!c) return P3T_ERR_ARG;
  prep_join(c);
  c->uf_early = 0;  // a new pair list
  if (!c->tree_valid) return fail(c, P3T_ERR_STATE, "compute_soft_force: no tree (call p3t_build_tree)");
  if (bad_ptr(acc3, c->n)) return fail(c, P3T_ERR_ARG, "compute_soft_force: null pointer");
  c->force_valid = false;
  if (c->n == 0) {
    c->n_pairs = 0;
    c->force_valid = true;
    return P3T_OK;
  }
  p3t_status st;
  for (int attempt = 0; attempt < 8; ++attempt) {
    ev_record(c, 4);
    HIP_OK(c, walk_groups(c, c->n_groups));
    ev_record(c, 5);
    HIP_OK(c, soft_force(c, c->n_groups, acc3));
    ev_record(c, 6);
    c->graphed = 0;
    if ((st = prep_enqueue(c)) != P3T_OK) return st;
    DevCounters h;
    if ((st = sync_counters(c, &h)) != P3T_OK) return st;
    unsigned num = 0;
    if (eval_finish(c, h, &num, &st)) {
      if (st != P3T_OK) return st;
      continue;  // grown: walk and force again over the same tree
    }
    if (num)
      return fail(c, P3T_ERR_NUMERIC, "compute_soft_force: device status 0x%x (coincident particles or NaN)", num);
    return st;  // the cluster preparation's status
  }
  return fail(c, P3T_ERR_CAPACITY, "compute_soft_force: scratch still too small after repeated growth");
}

namespace {

// Tree, walk and soft force enqueued on the context's stream, eagerly or by
// replaying the captured graph, with no host synchronisation; the caller
// reads the counters once the work is done and hands them to eval_finish.
p3t_status eval_enqueue(p3t_ctx *c, int64_t n, const double *pos3, const double *vel3, const double *mass,
                        const double *r_out, const double *r_search, double *acc3, int32_t use_graph) {
  p3t_status st;
  c->uf_early = 0;  // a new pair list
  if (!use_graph) {
    if ((st = p3t_build_tree(c, n, pos3, vel3, mass, r_out, r_search)) != P3T_OK) return st;
    ev_record(c, 4);
    HIP_OK(c, walk_groups(c, c->n_groups));
    ev_record(c, 5);
    HIP_OK(c, soft_force(c, c->n_groups, acc3));
    ev_record(c, 6);
    c->graphed = 0;
    return P3T_OK;
  }
  c->tree_valid = c->force_valid = false;
  c->n = n;
  if ((st = ensure_n(c, n)) != P3T_OK) return st;
  if ((st = ensure_lists(c, n)) != P3T_OK) return st;
  const void *ptrs[] = {pos3, vel3, mass, r_out, r_search, acc3};
  const uint64_t key = graph_key(c, n, ptrs, 6);
  if (!c->g_exec || key != c->g_key) {
    drop_graph(c);
    if (!c->cap_stream) HIP_OK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    const hipStream_t user = c->stream;
    const int timing = c->timing;
    c->stream = c->cap_stream;
    c->timing = 0;  // no event records inside the graph
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      // n bounds the group count; every group-sized loop reads the count on the device
      hipError_t e1 = build_tree(c, n, pos3, vel3, mass, r_out, r_search);
      if (e1 == hipSuccess) e1 = walk_groups(c, n);
      if (e1 == hipSuccess) e1 = soft_force(c, n, acc3);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(c->cap_stream, &g);
      if (e == hipSuccess) e = e1;
      c->g_graph = g;
      if (e == hipSuccess) e = hipGraphInstantiate(&c->g_exec, c->g_graph, nullptr, nullptr, 0);
    }
    c->stream = user;
    c->timing = timing;
    if (e != hipSuccess) {
      drop_graph(c);
      return fail(c, P3T_ERR_HIP, "evaluate: graph capture failed: %s", hipGetErrorString(e));
    }
    c->g_key = key;
  }
  ev_record(c, 2);
  HIP_OK(c, hipGraphLaunch(c->g_exec, c->stream));
  ev_record(c, 6);
  c->n_groups = n;
  c->tree_valid = true;
  c->stats.n = n;
  c->stats.n_nodes = 2 * n - 1;
  c->graphed = 1;
  return P3T_OK;
}

// The counters h of a finished enqueued evaluation.  A buffer that
// overflowed is grown (returns true: the evaluation must be redone);
// otherwise the pair count, groups and statistics are taken over and the
// numeric bits (coincident pairs, NaN) are left in *num.
bool eval_finish(p3t_ctx *c, const DevCounters &h, unsigned *num, p3t_status *st) {
  *st = P3T_OK;
  *num = 0;
  if (h.status & RETRY_BITS) {
    prep_drop_sync(c);  // it read a pair list that is redone
    *st = grow_for_retry(c, h);
    return true;
  }
  c->n_pairs = (int64_t)h.n_pairs;
  c->n_groups = c->groups_hint = (int64_t)h.n_groups;
  c->stats.n_groups = c->n_groups;
  c->stats.n_heval = (int64_t)h.n_heval;
  c->stats.n_hpair = (int64_t)h.n_hpair;
  c->stats.n_near = (int64_t)h.n_near;
  c->stats.n_far = (int64_t)h.n_far;
  c->stats.n_cell = (int64_t)h.n_cell;
  c->stats.n_pairs = c->n_pairs;
  c->stats.list_entries = (int64_t)h.pool_cursor;
  cut_timing_read(c);
  if (c->timing) {
    if (c->graphed) {
      c->stats.ms_tree = c->stats.ms_walk = c->stats.ms_sort = 0.0;
      c->stats.ms_force = ev_ms(c, 2, 6);  // the whole captured evaluation
      c->stats.ms_near = c->stats.ms_far = c->stats.ms_cell = c->stats.ms_cand = 0.0;
    } else {
      if (c->tree_timing_pending) {  // the tree of this evaluation was timed
        c->stats.ms_tree = ev_ms(c, 2, 3);
        c->stats.ms_sort = ev_ms(c, 17, 18);
      }
      c->stats.ms_walk = ev_ms(c, 4, 5);
      c->stats.ms_force = ev_ms(c, 5, 6);
      if (c->fcfg.split) {
        c->stats.ms_near = ev_ms(c, 5, 11);
        c->stats.ms_far = ev_ms(c, 11, 12);
        c->stats.ms_cell = ev_ms(c, 12, 13);
        c->stats.ms_cand = ev_ms(c, 13, 14);
      } else {
        c->stats.ms_near = c->stats.ms_far = c->stats.ms_cell = c->stats.ms_cand = 0.0;
      }
    }
    c->tree_timing_pending = 0;
  }
  *num = h.status & NUMERIC_BITS;
  c->host_status |= h.status;
  if (h.status) hipLaunchKernelGGL(k_clear_bits, dim3(1), dim3(1), 0, c->stream, c->cnt, h.status);
  c->force_valid = true;
  if (c->prep_state == 2) {
    if (*num)
      prep_join(c);
    else
      c->prep_state = 1;  // the preparation enqueued behind this evaluation holds
  }
  return false;
}

}  // namespace

p3t_status p3t_evaluate(p3t_ctx *c, int64_t n, const double *pos3, const double *vel3, const double *mass,
                        const double *r_out, const double *r_search, double *acc3, int32_t use_graph) {
  if (!c) return P3T_ERR_ARG;
  if (!use_graph || n == 0) {
    p3t_status st = p3t_build_tree(c, n, pos3, vel3, mass, r_out, r_search);
    if (st != P3T_OK) return st;
    return p3t_compute_soft_force(c, acc3);
  }
  if (n < 0 || n > (int64_t(1) << 30)) return fail(c, P3T_ERR_ARG, "evaluate: n out of range");
  if (bad_ptr(pos3, n) || bad_ptr(vel3, n) || bad_ptr(mass, n) || bad_ptr(r_out, n) || bad_ptr(r_search, n) ||
      bad_ptr(acc3, n))
    return fail(c, P3T_ERR_ARG, "evaluate: null pointer");
  prep_join(c);
  p3t_status st = eval_enqueue(c, n, pos3, vel3, mass, r_out, r_search, acc3, 1);
  if (st != P3T_OK) return st;
  if ((st = prep_enqueue(c)) != P3T_OK) return st;
  DevCounters h;
  if ((st = sync_counters(c, &h)) != P3T_OK) return st;
  unsigned num = 0;
  if (eval_finish(c, h, &num, &st)) {
    // a buffer overflowed: grown (the key changes with it); finish eagerly
    if (st != P3T_OK) return st;
    return p3t_compute_soft_force(c, acc3);
  }
  if (num) return fail(c, P3T_ERR_NUMERIC, "evaluate: device status 0x%x (coincident particles or NaN)", num);
  return st;
}

p3t_status p3t_neighbour_list(p3t_ctx *c, int64_t *row_ptr, int32_t *col, int64_t cap, int64_t *nnz_host,
                              int32_t *label) {
  if (!c) return P3T_ERR_ARG;
  prep_join(c);
  if (!c->force_valid) return fail(c, P3T_ERR_STATE, "neighbour_list: call p3t_compute_soft_force first");
  if (!nnz_host || !row_ptr || cap < 0) return fail(c, P3T_ERR_ARG, "neighbour_list: bad argument");
  const int64_t n = c->n, np = c->n_pairs;
  *nnz_host = np;
  if (n == 0) {
    HIP_OK(c, hipMemsetAsync(row_ptr, 0, sizeof(int64_t), c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return P3T_OK;
  }
  ev_record(c, 7);
  HIP_OK(c, build_csr(c, n, np));
  if (np > cap) {
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return fail(c, P3T_ERR_CAPACITY, "neighbour_list: nnz %lld exceeds cap %lld", (long long)np, (long long)cap);
  }
  if (np > 0 && !col) return fail(c, P3T_ERR_ARG, "neighbour_list: null col");
  HIP_OK(c, hipMemcpyAsync(row_ptr, c->csr_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, c->stream));
  if (np > 0) HIP_OK(c, hipMemcpyAsync(col, c->csr_col, sizeof(int32_t) * np, hipMemcpyDeviceToDevice, c->stream));
  if (label) HIP_OK(c, labels_cc(c, n, label));
  ev_record(c, 8);
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (c->timing) c->stats.ms_neighbour = ev_ms(c, 7, 8);
  return P3T_OK;
}

p3t_status p3t_clusters(p3t_ctx *c, int64_t n, const int32_t *label, int32_t *cl_ptr, int32_t *cl_members,
                        int64_t *n_clusters_host) {
  if (!c) return P3T_ERR_ARG;
  prep_join(c);
  if (n < 0 || n > (int64_t(1) << 30) || !n_clusters_host) return fail(c, P3T_ERR_ARG, "clusters: bad argument");
  if (bad_ptr(label, n) || bad_ptr(cl_ptr, n) || bad_ptr(cl_members, n)) return fail(c, P3T_ERR_ARG, "clusters: null");
  *n_clusters_host = 0;
  if (n == 0) return P3T_OK;
  p3t_status st = ensure_n(c, n);
  if (st != P3T_OK) return st;
  int64_t nc = 0;
  HIP_OK(c, clusters_csr(c, n, label, cl_ptr, cl_members, &nc));
  *n_clusters_host = nc;
  return P3T_OK;
}

p3t_status p3t_hermite_cluster_step(p3t_ctx *c, int64_t n, int64_t n_clusters, const int32_t *cl_ptr,
                                    const int32_t *cl_members, double *pos3, double *vel3, const double *mass,
                                    const double *r_out, double *dt_hard, double *e_rel_err, int32_t *n_steps) {
  if (!c) return P3T_ERR_ARG;
  prep_join(c);
  if (n < 0 || n_clusters < 0 || n > (int64_t(1) << 30) || n_clusters > (int64_t(1) << 30))
    return fail(c, P3T_ERR_ARG, "hermite_cluster_step: size out of range");
  if (n_clusters == 0) return P3T_OK;
  if (!cl_ptr || !cl_members || bad_ptr(pos3, n) || bad_ptr(vel3, n) || bad_ptr(mass, n) || bad_ptr(r_out, n))
    return fail(c, P3T_ERR_ARG, "hermite_cluster_step: null pointer");
  p3t_status st = ensure_n(c, std::max(n, n_clusters));
  if (st != P3T_OK) return st;
  ev_record(c, 9);
  hipError_t e =
      hermite_clusters(c, n, n_clusters, cl_ptr, cl_members, pos3, vel3, mass, r_out, dt_hard, e_rel_err, n_steps);
  if (e == hipErrorInvalidDevicePointer)
    return fail(c, P3T_ERR_ARG, "hermite_cluster_step: cl_ptr not non-decreasing or a member outside [0, n)");
  HIP_OK(c, e);
  ev_record(c, 10);
  unsigned bits = 0;
  if ((st = harvest_status(c, &bits)) != P3T_OK) return st;
  if (c->timing) c->stats.ms_hermite = ev_ms(c, 9, 10);
  if (bits & NUMERIC_BITS)
    return fail(c, P3T_ERR_NUMERIC, "hermite_cluster_step: device status 0x%x", bits & NUMERIC_BITS);
  return P3T_OK;
}

p3t_status p3t_hermite_collide(p3t_ctx *c, int64_t n, int64_t n_clusters, const int32_t *cl_ptr,
                               const int32_t *cl_members, double *pos3, double *vel3, const double *mass,
                               const double *r_out, double *dt_hard, double f_radius, double density,
                               int32_t *merged_into, double *eps6, double *e_rel_err, int32_t *n_steps,
                               int64_t *n_collisions_host) {
  if (!c) return P3T_ERR_ARG;
  prep_join(c);
  if (n_collisions_host) *n_collisions_host = 0;
  if (n < 0 || n_clusters < 0 || n > (int64_t(1) << 30) || n_clusters > (int64_t(1) << 30))
    return fail(c, P3T_ERR_ARG, "hermite_collide: size out of range");
  if (!(f_radius >= 0.0) || !std::isfinite(f_radius)) return fail(c, P3T_ERR_ARG, "hermite_collide: f_radius < 0");
  if (!(density > 0.0) || !std::isfinite(density)) return fail(c, P3T_ERR_ARG, "hermite_collide: density <= 0");
  if (n_clusters == 0) return P3T_OK;
  if (!cl_ptr || !cl_members || bad_ptr(pos3, n) || bad_ptr(vel3, n) || bad_ptr(mass, n) || bad_ptr(r_out, n) ||
      bad_ptr(merged_into, n))
    return fail(c, P3T_ERR_ARG, "hermite_collide: null pointer");
  p3t_status st = ensure_n(c, std::max(n, n_clusters));
  if (st != P3T_OK) return st;
  if (!eps6 && c->coll_cap < 6 * n_clusters + 6) {
    HIP_OK(c, dev_alloc(c->coll_buf, 6 * c->n_cap + 6));
    c->coll_cap = 6 * c->n_cap + 6;
  }
  double *ceps = eps6 ? eps6 : c->coll_buf;
  HIP_OK(c, iota_i32(merged_into, n, c->stream));
  HIP_OK(c, fill_f64(ceps, 0.0, 6 * n_clusters, c->stream));
  HermColl hc;
  hc.f = f_radius;
  hc.r3 = 3.0 / (4.0 * M_PI * density);
  hc.merged = merged_into;
  hc.ceps = ceps;
  ev_record(c, 9);
  hipError_t e = hermite_clusters(c, n, n_clusters, cl_ptr, cl_members, pos3, vel3, mass, r_out, dt_hard, e_rel_err,
                                  n_steps, nullptr, nullptr, nullptr, &hc);
  if (e == hipErrorInvalidDevicePointer)
    return fail(c, P3T_ERR_ARG, "hermite_collide: cl_ptr not non-decreasing or a member outside [0, n)");
  HIP_OK(c, e);
  ev_record(c, 10);
  DevCounters h;
  if ((st = sync_counters(c, &h)) != P3T_OK) return st;
  if (n_collisions_host) *n_collisions_host = (int64_t)h.n_coll;
  unsigned bits = 0;
  if ((st = harvest_status(c, &bits)) != P3T_OK) return st;
  if (c->timing) c->stats.ms_hermite = ev_ms(c, 9, 10);
  if (bits & NUMERIC_BITS)
    return fail(c, P3T_ERR_NUMERIC, "hermite_collide: device status 0x%x", bits & NUMERIC_BITS);
  return P3T_OK;
}

p3t_status p3t_kick(p3t_ctx *c, int64_t n, double h, const double *acc3, double *vel3) {
  if (!c) return P3T_ERR_ARG;
  if (n < 0 || bad_ptr(acc3, n) || bad_ptr(vel3, n) || !std::isfinite(h)) return fail(c, P3T_ERR_ARG, "kick: bad argument");
  HIP_OK(c, kick(n, h, acc3, vel3, c->stream));
  return P3T_OK;
}

p3t_status p3t_kepler_drift(p3t_ctx *c, int64_t n, double dt, double *pos3, double *vel3, const int32_t *list,
                            int64_t n_list, int32_t *iters, int64_t *n_unbound_host) {
  if (!c) return P3T_ERR_ARG;
  prep_join(c);
  if (n < 0 || n_list < 0 || bad_ptr(pos3, n) || bad_ptr(vel3, n) || !std::isfinite(dt))
    return fail(c, P3T_ERR_ARG, "kepler_drift: bad argument");
  if (n_list > 0 && !list && n_list != n) return fail(c, P3T_ERR_ARG, "kepler_drift: without a list n_list must equal n");
  if (n_list > 0 && n == 0) return fail(c, P3T_ERR_ARG, "kepler_drift: list given for n = 0");
  const double mu = c->P.G * c->P.m_star;
  if (!(mu > 0.0) || !std::isfinite(mu)) return fail(c, P3T_ERR_STATE, "kepler_drift: G m_star must be > 0");
  const size_t off = offsetof(DevCounters, n_unbound);
  HIP_OK(c, hipMemsetAsync((char *)c->cnt + off, 0, 2 * sizeof(unsigned long long), c->stream));
  HIP_OK(c, kepler_drift(n, n_list, list, mu, dt, pos3, vel3, iters, c->cnt, c->stream));
  if (n_unbound_host) {
    DevCounters h;
    p3t_status st;
    if ((st = sync_counters(c, &h)) != P3T_OK) return st;
    *n_unbound_host = (int64_t)h.n_unbound;
    if (h.n_bad_index) return fail(c, P3T_ERR_ARG, "kepler_drift: %llu list entries outside [0, n)", h.n_bad_index);
  }
  return P3T_OK;
}

p3t_status p3t_hard_step(p3t_ctx *c, double *pos3, double *vel3, const double *mass, const double *r_out,
                         double *dt_hard, int32_t *steps, int64_t *n_clusters_host) {
  if (!c) return P3T_ERR_ARG;
  if (!c->force_valid) return fail(c, P3T_ERR_STATE, "hard_step: no neighbour pairs (call p3t_compute_soft_force)");
  const int64_t n = c->n;
  if (bad_ptr(pos3, n) || bad_ptr(vel3, n) || bad_ptr(mass, n) || bad_ptr(r_out, n))
    return fail(c, P3T_ERR_ARG, "hard_step: null pointer");
  if (n_clusters_host) *n_clusters_host = 0;
  if (n == 0) {
    prep_join(c);
    return P3T_OK;
  }
  int32_t hc[HERM_BC_WORDS];
  const bool prepared = prep_take(c, n, hc);
  ev_record(c, 9);
  if (!prepared) {
    HIP_OK(c, build_csr(c, n, c->n_pairs));
    HIP_OK(c, labels_cc(c, n, c->hs_label));
    HIP_OK(c, clusters_csr_dev(c, n, c->hs_label, c->hs_cl_ptr, c->hs_cl_mem));
  }
  ev_record(c, 19);
  hipError_t e = prepared ? (hc[HERM_BC_BAD] ? hipErrorInvalidDevicePointer : hipSuccess)
                          : herm_bucket(c, n, n, c->hs_cl_ptr, c->hs_cl_mem, c->node_scan + n, hc, close_src(c));
  HIP_OK(c, e);
  HIP_OK(c, aux_streams(c));
  HIP_OK(c, herm_launch(c, n, n, c->hs_cl_ptr, c->hs_cl_mem, pos3, vel3, mass, r_out, dt_hard, nullptr, nullptr,
                        steps, hc, 0, 0, c->stream, c->aux_stream, c->aux_ev[0], c->aux_ev[1]));
  ev_record(c, 10);
  if (n_clusters_host) *n_clusters_host = hc[HERM_BC_NC];
  if (c->timing) {
    HIP_OK(c, hipStreamSynchronize(c->stream));
    c->stats.ms_hermite = ev_ms(c, 9, 10);
    if (!prepared) c->stats.ms_clusters = ev_ms(c, 9, 19);
  }
  return P3T_OK;
}

p3t_status p3t_hard_step_collide(p3t_ctx *c, double *pos3, double *vel3, const double *mass, const double *r_out,
                                 double *dt_hard, int32_t *steps, double f_radius, double density,
                                 int32_t *merged_into, double *eps_host, int64_t *n_collisions_host,
                                 int64_t *n_clusters_host) {
  if (!c) return P3T_ERR_ARG;
  if (!c->force_valid)
    return fail(c, P3T_ERR_STATE, "hard_step_collide: no neighbour pairs (call p3t_compute_soft_force)");
  const int64_t n = c->n;
  if (bad_ptr(pos3, n) || bad_ptr(vel3, n) || bad_ptr(mass, n) || bad_ptr(r_out, n) || bad_ptr(merged_into, n))
    return fail(c, P3T_ERR_ARG, "hard_step_collide: null pointer");
  if (!(f_radius >= 0.0) || !std::isfinite(f_radius)) return fail(c, P3T_ERR_ARG, "hard_step_collide: f_radius < 0");
  if (!(density > 0.0) || !std::isfinite(density)) return fail(c, P3T_ERR_ARG, "hard_step_collide: density <= 0");
  if (n_clusters_host) *n_clusters_host = 0;
  if (n_collisions_host) *n_collisions_host = 0;
  if (eps_host)
    for (int q = 0; q < 6; ++q) eps_host[q] = 0.0;
  if (n == 0) return P3T_OK;
  if (c->coll_cap < 6 * n + 6) {
    HIP_OK(c, dev_alloc(c->coll_buf, 6 * c->n_cap + 6));
    c->coll_cap = 6 * c->n_cap + 6;
  }
  int32_t hcw[HERM_BC_WORDS];
  const bool prepared = prep_take(c, n, hcw);
  ev_record(c, 9);
  if (!prepared) {
    HIP_OK(c, build_csr(c, n, c->n_pairs));
    HIP_OK(c, labels_cc(c, n, c->hs_label));
    HIP_OK(c, clusters_csr_dev(c, n, c->hs_label, c->hs_cl_ptr, c->hs_cl_mem));
  }
  ev_record(c, 19);
  HIP_OK(c, iota_i32(merged_into, n, c->stream));
  HIP_OK(c, fill_f64(c->coll_buf, 0.0, 6 * n, c->stream));
  HermColl hc;
  hc.f = f_radius;
  hc.r3 = 3.0 / (4.0 * M_PI * density);
  hc.merged = merged_into;
  hc.ceps = c->coll_buf;
  hipError_t e = prepared ? (hcw[HERM_BC_BAD] ? hipErrorInvalidDevicePointer : hipSuccess)
                          : herm_bucket(c, n, n, c->hs_cl_ptr, c->hs_cl_mem, c->node_scan + n, hcw, close_src(c));
  HIP_OK(c, e);
  HIP_OK(c, aux_streams(c));
  HIP_OK(c, herm_launch(c, n, n, c->hs_cl_ptr, c->hs_cl_mem, pos3, vel3, mass, r_out, dt_hard, nullptr, nullptr,
                        steps, hcw, 0, 0, c->stream, c->aux_stream, c->aux_ev[0], c->aux_ev[1], &hc));
  ev_record(c, 10);
  const int64_t nc = hcw[HERM_BC_NC];
  if (n_clusters_host) *n_clusters_host = nc;
  HIP_OK(c, sum_rows6(nc, c->coll_buf, c->coll_buf + 6 * n, c->stream));
  double sums[6];
  HIP_OK(c, hipMemcpyAsync(sums, c->coll_buf + 6 * n, sizeof(sums), hipMemcpyDeviceToHost, c->stream));
  DevCounters h;
  p3t_status st = sync_counters(c, &h);  // synchronises the stream
  if (st != P3T_OK) return st;
  if (eps_host)
    for (int q = 0; q < 6; ++q) eps_host[q] = sums[q];
  if (n_collisions_host) *n_collisions_host = (int64_t)h.n_coll;
  if (c->timing) {
    c->stats.ms_hermite = ev_ms(c, 9, 10);
    if (!prepared) c->stats.ms_clusters = ev_ms(c, 9, 19);
  }
  return P3T_OK;
}

p3t_status p3t_merge_bodies(p3t_ctx *c, int64_t n, const int32_t *merged_into, double *pos3, double *vel3,
                            double *mass, double *dt_hard, int32_t *steps, int64_t *n_new_host) {
  if (!c || !n_new_host) return P3T_ERR_ARG;
  prep_join(c);
  *n_new_host = n;
  if (n < 0 || n > (int64_t(1) << 30)) return fail(c, P3T_ERR_ARG, "merge_bodies: n out of range");
  if (n == 0) return P3T_OK;
  if (bad_ptr(merged_into, n) || bad_ptr(pos3, n) || bad_ptr(vel3, n) || bad_ptr(mass, n))
    return fail(c, P3T_ERR_ARG, "merge_bodies: null pointer");
  p3t_status st = ensure_n(c, n);  // node_scan (n + 1) and the scan scratch
  if (st != P3T_OK) return st;
  if (c->merge_cap < n) {
    HIP_OK(c, dev_alloc(c->merge_st, 9 * c->n_cap));
    HIP_OK(c, dev_alloc(c->merge_i32, 2 * c->n_cap + 1));
    c->merge_cap = c->n_cap;
  }
  c->tree_valid = c->force_valid = false;  // the particle set changes
  hipError_t e = merge_bodies(c, n, merged_into, pos3, vel3, mass, dt_hard, steps, n_new_host);
  if (e == hipErrorInvalidValue)
    return fail(c, P3T_ERR_ARG, "merge_bodies: merged_into is not a composite map (each entry the lowest index "
                                "of its composite, which maps to itself)");
  HIP_OK(c, e);
  return P3T_OK;
}

namespace {

// pair buffer of the parked members' direct terms (its own allocation, grown
// when the count after a join exceeds it)
p3t_status ensure_pairs_d(p3t_ctx *c, int64_t cap) {
  if (c->pairs_d && c->pairs_d_alloc >= cap) {
    c->pairs_d_cap = cap;
    return P3T_OK;
  }
  HIP_OK(c, dev_alloc(c->pairs_d, cap));
  c->pairs_d_alloc = c->pairs_d_cap = cap;
  return P3T_OK;
}

// buffers of p3t_hard_evaluate's slow split, sized for n_cap particles
p3t_status ensure_overlap(p3t_ctx *c) {
  if (!c->slow_ev[0])
    for (auto &ev : c->slow_ev) HIP_OK(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  const int64_t pcap = c->pairs_d_cap > 0 ? c->pairs_d_cap : 64 * SLOW_CAP;
  if (c->ov_buf && c->ov_n_cap >= c->n_cap) return ensure_pairs_d(c, pcap);
  const int64_t nc = c->n_cap;
  auto bytes = [](int64_t count, size_t sz) { return ((size_t)count * sz + 255) & ~size_t(255); };
  const size_t total = 4 * bytes(3 * nc, sizeof(double)) + bytes(nc, sizeof(int64_t)) + 2 * bytes(nc, sizeof(int32_t)) +
                       2 * bytes(nc, sizeof(double)) + bytes(10 * nc, sizeof(int32_t)) + bytes(nc, sizeof(int32_t)) +
                       bytes((int64_t)SLOW_CAP * SLOW_CHUNKS * 3, sizeof(double)) + bytes(3 * nc, sizeof(double));
  c->ov_n_cap = 0;
  c->pk_x = nullptr;
  HIP_OK(c, dev_alloc(c->ov_buf, (int64_t)total));
  Arena A;
  A.base = c->ov_buf;
  A.size = total;
  c->pk_x = A.take<double>(3 * nc);
  c->pk_v = A.take<double>(3 * nc);
  c->pk_a = A.take<double>(3 * nc);
  c->pk_j = A.take<double>(3 * nc);
  c->pk_t = A.take<int64_t>(nc);
  c->pk_lev = A.take<int32_t>(nc);
  c->pk_nst = A.take<int32_t>(nc);
  c->pk_e0 = A.take<double>(nc);
  c->m_eff = A.take<double>(nc);
  c->pk_lists = A.take<int32_t>(10 * nc);
  c->slow_list = A.take<int32_t>(nc);
  c->slow_part = A.take<double>((int64_t)SLOW_CAP * SLOW_CHUNKS * 3);
  c->acc_d = A.take<double>(3 * nc);
  if (!c->acc_d) return fail(c, P3T_ERR_HIP, "overlap buffer layout overflow (internal)");
  c->ov_n_cap = nc;
  return ensure_pairs_d(c, pcap);
}

}  // namespace

p3t_status p3t_hard_evaluate(p3t_ctx *c, double *pos3, double *vel3, const double *mass, const double *r_out_hard,
                             double *dt_hard, int32_t *steps, const double *r_out, const double *r_search, double *acc3,
                             int32_t slow_log2, int32_t use_graph, int64_t *n_clusters_host, int64_t *n_slow_host) {
  if (!c) return P3T_ERR_ARG;
  if (n_clusters_host) *n_clusters_host = 0;
  if (n_slow_host) *n_slow_host = 0;
  if (!c->force_valid)
    return fail(c, P3T_ERR_STATE, "hard_evaluate: no neighbour pairs (call p3t_compute_soft_force)");
  const int64_t n = c->n;
  if (bad_ptr(pos3, n) || bad_ptr(vel3, n) || bad_ptr(mass, n) || bad_ptr(r_out_hard, n) || bad_ptr(r_out, n) ||
      bad_ptr(r_search, n) || bad_ptr(acc3, n))
    return fail(c, P3T_ERR_ARG, "hard_evaluate: null pointer");
  c->stats.n_slow = 0;
  c->stats.ms_direct = 0.0;
  if (n == 0) return p3t_evaluate(c, 0, pos3, vel3, mass, r_out, r_search, acc3, use_graph);
  const bool split = slow_log2 > 0;
  p3t_status st;
  int32_t hc[HERM_BC_WORDS];
  const bool prepared = prep_take(c, n, hc);
  if (split && (st = ensure_overlap(c)) != P3T_OK) return st;
  ev_record(c, 9);
  if (!prepared) {
    HIP_OK(c, build_csr(c, n, c->n_pairs));
    HIP_OK(c, labels_cc(c, n, c->hs_label));
    HIP_OK(c, clusters_csr_dev(c, n, c->hs_label, c->hs_cl_ptr, c->hs_cl_mem));
  }
  ev_record(c, 19);
  hipError_t e = prepared ? (hc[HERM_BC_BAD] ? hipErrorInvalidDevicePointer : hipSuccess)
                          : herm_bucket(c, n, n, c->hs_cl_ptr, c->hs_cl_mem, c->node_scan + n, hc, close_src(c));
  if (n_clusters_host) *n_clusters_host = hc[HERM_BC_NC];
  HIP_OK(c, e);
  HIP_OK(c, aux_streams(c));
  const int budget = split ? (slow_log2 < 30 ? 1 << slow_log2 : 1 << 30) : 0;
  if (split) {
    HIP_OK(c, hipMemsetAsync(c->slow_flag, 0, (size_t)n, c->stream));
    c->park_flags_valid = 1;
  }
  HIP_OK(c, herm_launch(c, n, n, c->hs_cl_ptr, c->hs_cl_mem, pos3, vel3, mass, r_out_hard, dt_hard, nullptr, nullptr,
                        steps, hc, budget, 0, c->stream, c->aux_stream, c->aux_ev[0], c->aux_ev[1]));
  ev_record(c, 10);
  if (!split) {
    st = p3t_evaluate(c, n, pos3, vel3, mass, r_out, r_search, acc3, use_graph);
    if (c->timing) {
      c->stats.ms_hermite = ev_ms(c, 9, 10);
      if (!prepared) c->stats.ms_clusters = ev_ms(c, 9, 19);
    }
    return st;
  }
  // the clusters parked by the step budget finish on their own stream
  HIP_OK(c, hipMemcpyAsync(hc + HERM_BC_PARK0, c->herm_bcount + HERM_BC_PARK0,
                           sizeof(int32_t) * (HERM_BC_PARKED + 1 - HERM_BC_PARK0), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  int ns = hc[HERM_BC_PARKED];
  if (ns > SLOW_CAP) {
    // too many for the direct sums: finish them here, then evaluate as usual
    HIP_OK(c, herm_launch(c, n, n, c->hs_cl_ptr, c->hs_cl_mem, pos3, vel3, mass, r_out_hard, dt_hard, nullptr,
                          nullptr, steps, hc, 0, 1, c->stream, c->aux_stream, c->aux_ev[0], c->aux_ev[1]));
    HIP_OK(c, slow_merge(c, pos3, vel3, nullptr, ns));  // copies the state back only
    HIP_OK(c, hipMemsetAsync(c->slow_flag, 0, (size_t)n, c->stream));
    if (c->timing) {
      ev_record(c, 10);
      HIP_OK(c, hipStreamSynchronize(c->stream));
      c->stats.ms_hermite = ev_ms(c, 9, 10);
      if (!prepared) c->stats.ms_clusters = ev_ms(c, 9, 19);
    }
    c->stats.n_slow = 0;
    return p3t_evaluate(c, n, pos3, vel3, mass, r_out, r_search, acc3, use_graph);
  }
  if (ns > 0) {
    // resume, then (issued below, after the evaluation's launches) the
    // direct terms of S, both beside the evaluation
    HIP_OK(c, hipEventRecord(c->slow_ev[0], c->stream));
    HIP_OK(c, hipStreamWaitEvent(c->slow_stream, c->slow_ev[0], 0));
    HIP_OK(c, slow_sort(c, ns, c->slow_stream));  // while the chip is free, not behind the tree's kernels
    HIP_OK(c, herm_launch(c, n, n, c->hs_cl_ptr, c->hs_cl_mem, pos3, vel3, mass, r_out_hard, dt_hard, nullptr, nullptr,
                          steps, hc, 0, 1, c->slow_stream, c->aux_stream, c->aux_ev[0], c->aux_ev[1]));
    // the direct terms' pair counter and status word, cleared on the main
    // stream while the resume runs
    HIP_OK(c, hipMemsetAsync(&c->cnt->n_pairs_d, 0, sizeof(unsigned long long), c->stream));
    HIP_OK(c, hipMemsetAsync(&c->cnt->status_d, 0, sizeof(unsigned int), c->stream));
    HIP_OK(c, hipEventRecord(c->slow_ev[2], c->stream));
  }
  // everyone else: tree, walk and force at the new state, S massless (with
  // S empty too, so that a captured evaluation keeps its arguments)
  HIP_OK(c, slow_prepare(c, mass, ns));
  c->slow_active = 1;
  st = eval_enqueue(c, n, pos3, vel3, c->m_eff, r_out, r_search, acc3, use_graph);
  c->slow_active = 0;
  if (ns > 0) {
    HIP_OK(c, hipStreamWaitEvent(c->slow_stream, c->slow_ev[2], 0));
    HIP_OK(c, slow_direct(c, pos3, vel3, mass, r_out, r_search, ns, c->slow_stream));
    HIP_OK(c, hipEventRecord(c->slow_ev[1], c->slow_stream));
  }
  // the next hard part's union-find over the pairs written so far, while
  // the main stream would wait for the second one anyway
  if (ns > 0 && st == P3T_OK) HIP_OK(c, labels_pairs_early(c, n));
  // join: S's new state into pos3 / vel3, its terms into acc3
  if (ns > 0) HIP_OK(c, hipStreamWaitEvent(c->stream, c->slow_ev[1], 0));
  ev_record(c, 15);
  if (st != P3T_OK) {
    // nothing of the evaluation ran: the state is that of p3t_hard_step
    if (ns > 0) HIP_OK(c, slow_merge(c, pos3, vel3, nullptr, ns));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    c->force_valid = false;
    return st;
  }
  if (ns > 0) HIP_OK(c, slow_merge(c, pos3, vel3, acc3, ns));
  ev_record(c, 16);
  if ((st = prep_enqueue(c)) != P3T_OK) return st;
  // the one synchronisation of the evaluation: its counters, the direct
  // terms' pair count and the second stream's status bits
  DevCounters h;
  if ((st = sync_counters(c, &h)) != P3T_OK) return st;
  if (c->timing) {
    c->stats.ms_hermite = ev_ms(c, 9, 10);
    if (!prepared) c->stats.ms_clusters = ev_ms(c, 9, 19);
    c->stats.ms_direct = ev_ms(c, 15, 16);
  }
  c->stats.n_slow = ns;
  if (n_slow_host) *n_slow_host = ns;
  // the second stream's bits (coincident pairs, NaN) join the status here
  const unsigned bits_d = ns > 0 ? h.status_d & NUMERIC_BITS : 0u;
  const bool direct_overflow = ns > 0 && (int64_t)h.n_pairs_d > c->pairs_d_cap;
  if ((h.status & RETRY_BITS) || direct_overflow) {
    // a buffer was too small: grow it, and evaluate again at the final
    // state (an ordinary evaluation, every term from the tree)
    prep_drop_sync(c);  // it read an incomplete pair list
    c->host_status |= bits_d;
    if (direct_overflow) {
      const int64_t need = (int64_t)h.n_pairs_d;
      if ((st = ensure_pairs_d(c, need + need / 4 + 1024)) != P3T_OK) return st;
    }
    if ((h.status & RETRY_BITS) && (st = grow_for_retry(c, h)) != P3T_OK) return st;
    return p3t_evaluate(c, n, pos3, vel3, mass, r_out, r_search, acc3, 0);
  }
  unsigned num = 0;
  eval_finish(c, h, &num, &st);  // no retry bits here
  num |= bits_d;
  c->host_status |= bits_d;
  if (num)
    return fail(c, P3T_ERR_NUMERIC, "hard_evaluate: device status 0x%x (coincident particles or NaN)", num);
  return st;
}

p3t_status p3t_total_energy(p3t_ctx *c, int64_t n, const double *pos3, const double *vel3, const double *mass,
                            double *energy_host) {
  if (!c) return P3T_ERR_ARG;
  prep_join(c);
  if (n < 0 || n > (int64_t(1) << 30) || !energy_host) return fail(c, P3T_ERR_ARG, "total_energy: bad argument");
  if (bad_ptr(pos3, n) || bad_ptr(vel3, n) || bad_ptr(mass, n)) return fail(c, P3T_ERR_ARG, "total_energy: null pointer");
  *energy_host = 0.0;
  if (n == 0) return P3T_OK;
  p3t_status st = ensure_n(c, n);
  if (st != P3T_OK) return st;
  double *share = c->tmp_d, *out = c->tmp_d + n;  // 3 n_cap doubles of scratch
  HIP_OK(c, total_energy(n, pos3, vel3, mass, c->P.G, c->P.G * c->P.m_star, share, out, c->stream));
  HIP_OK(c, hipMemcpyAsync(energy_host, out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return P3T_OK;
}

p3t_status p3t_soft_force_frozen(p3t_ctx *c, const double *pos3, const double *mass, double *acc3) {
  if (!c) return P3T_ERR_ARG;
  prep_join(c);
  if (!c->force_valid) return fail(c, P3T_ERR_STATE, "soft_force_frozen: no interaction lists (call p3t_compute_soft_force)");
  if (bad_ptr(pos3, c->n) || bad_ptr(mass, c->n) || bad_ptr(acc3, c->n))
    return fail(c, P3T_ERR_ARG, "soft_force_frozen: null pointer");
  if (c->n == 0) return P3T_OK;
  HIP_OK(c, refresh_tree(c, pos3, mass));
  reset_queues(c);
  HIP_OK(c, soft_force(c, c->n_groups, acc3, true));
  // no pair or candidate buffer was offered: their overflow bits mean nothing here
  hipLaunchKernelGGL(k_clear_bits, dim3(1), dim3(1), 0, c->stream, c->cnt, (unsigned)P3T_FLAG_PAIR_OVERFLOW);
  return P3T_OK;
}

p3t_status p3t_soft_kick_adjoint(p3t_ctx *c, double h, const double *lam_v3, double *g_pos3, double *g_mass) {
  if (!c) return P3T_ERR_ARG;
  prep_join(c);
  if (!c->force_valid) return fail(c, P3T_ERR_STATE, "soft_kick_adjoint: no interaction lists (call p3t_compute_soft_force)");
  if (bad_ptr(lam_v3, c->n) || bad_ptr(g_pos3, c->n) || bad_ptr(g_mass, c->n))
    return fail(c, P3T_ERR_ARG, "soft_kick_adjoint: null pointer");
  if (c->P.multipole != 1 && c->stats.n_cell > 0)
    return fail(c, P3T_ERR_STATE, "soft_kick_adjoint: cells must be monopoles (multipole = 1) or absent (theta = 0)");
  if (c->n == 0) return P3T_OK;
  if (c->adj_cap < c->n) {
    HIP_OK(c, hipStreamSynchronize(c->stream));
    HIP_OK(c, dev_alloc(c->adj_buf, adjoint_buf_need(c->n_cap)));
    c->adj_cap = c->n_cap;
  }
  HIP_OK(c, soft_kick_adjoint(c, h, lam_v3, g_pos3, g_mass));
  return P3T_OK;
}

p3t_status p3t_set_timing(p3t_ctx *c, int32_t on) {
  if (!c) return P3T_ERR_ARG;
  c->timing = on ? 1 : 0;
  c->stats.timing = c->timing;
  return P3T_OK;
}

p3t_status p3t_set_kernel_config(p3t_ctx *c, const p3t_kernel_config *k) {
  if (!c || !k) return P3T_ERR_ARG;
  prep_join(c);
  const int u = k->force_unroll;
  if ((k->force_split != 0 && k->force_split != 1) || (u != 1 && u != 2 && u != 4 && u != 8) ||
      (k->force_persistent != 0 && k->force_persistent != 1) || k->waves_per_cu < 1 || k->waves_per_cu > 64 ||
      k->walk_waves_per_cu < 1 || k->walk_waves_per_cu > 64 || k->direct_pair_cap < 0 || k->top_slots < 0 ||
      k->top_slots > 4096 || (k->top_slots & (k->top_slots - 1)) != 0)
    return fail(c, P3T_ERR_ARG, "set_kernel_config: value out of range");
  if (k->direct_pair_cap > 0) c->pairs_d_cap = k->direct_pair_cap;  // allocated (or grown) when next needed
  if (k->top_slots > 0) c->top_slots = k->top_slots;
  c->fcfg.split = k->force_split;
  c->fcfg.unroll = u;
  c->fcfg.waves_per_cu = k->waves_per_cu;
  c->force_persistent = k->force_persistent;
  if (c->walk_waves_per_cu != k->walk_waves_per_cu) {
    c->walk_waves_per_cu = k->walk_waves_per_cu;
    if (c->slot_lists) {  // the walk's per-slot scratch follows the grid
      HIP_OK(c, hipStreamSynchronize(c->stream));
      c->walk_slots = c->n_cu * c->walk_waves_per_cu;
      HIP_OK(c, dev_alloc(c->slot_lists, (int64_t)c->walk_slots * 3 * c->slot_cap_list));
      HIP_OK(c, dev_alloc(c->slot_stack, (int64_t)c->walk_slots * c->slot_cap_stack));
    }
  }
  return P3T_OK;
}

p3t_status p3t_get_kernel_config(p3t_ctx *c, p3t_kernel_config *k) {
  if (!c || !k) return P3T_ERR_ARG;
  *k = p3t_kernel_config{};
  k->force_split = c->fcfg.split;
  k->force_unroll = c->fcfg.unroll;
  k->force_persistent = c->force_persistent;
  k->waves_per_cu = c->fcfg.waves_per_cu;
  k->walk_waves_per_cu = c->walk_waves_per_cu;
  k->direct_pair_cap = (int32_t)std::min<int64_t>(c->pairs_d_cap > 0 ? c->pairs_d_cap : 64 * SLOW_CAP, INT32_MAX);
  k->top_slots = c->top_slots;
  return P3T_OK;
}

p3t_status p3t_get_stats(p3t_ctx *c, p3t_stats *out) {
  if (!c || !out) return P3T_ERR_ARG;
  cut_timing_read(c);
  *out = c->stats;
  return P3T_OK;
}

p3t_status p3t_get_status(p3t_ctx *c, uint32_t *flags) {
  if (!c || !flags) return P3T_ERR_ARG;
  prep_join(c);
  unsigned bits = 0;
  p3t_status st = harvest_status(c, &bits);
  if (st != P3T_OK) return st;
  *flags = c->host_status;
  c->host_status = 0;
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return P3T_OK;
}

const char *p3t_last_error(p3t_ctx *c) { return c ? c->last_error.c_str() : noalloc_last_error(); }

}  // extern "C"
