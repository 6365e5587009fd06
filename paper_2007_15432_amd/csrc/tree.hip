// tree.hip -- Barnes-Hut tree over the particles (the paper uses the tree of
// its particle framework, Section 2.1.1; its construction is not specified
// there).  Built here for one GPU, fully in parallel:
//   1. bounding box; 48-bit Morton keys on a cube over the box (16 bits/axis,
//      cells of 2^-16 of the box, far below the leaf scale; the thin disk
//      then splits in x/y first and in z only at small scales);
//   2. stable radix sort of (key, index); gather of a Morton-ordered SoA copy;
//   3. binary radix tree over the sorted keys (one thread per internal node,
//      Karras 2012), ties broken by the sorted position;
//   4. bottom-up pass (one thread per leaf, second arrival combines): tight
//      bounding box, mass, centre of mass, traceless quadrupole, max reach;
//   5. interaction groups: nodes with at most n_group_max particles whose
//      parent has more.
#include "p3t_internal.h"

namespace p3t {

// bit k of v (k < 21) to bit 3k
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

// bits per axis of the Morton keys: 3 MORTON_BITS = 48 key bits, six 8-bit
// radix passes
constexpr int MORTON_BITS = 16;

__global__ void k_morton(int64_t n, const double *__restrict__ pos, const double *__restrict__ box,
                         uint64_t *__restrict__ keys, int32_t *__restrict__ perm) {
  const double lx = box[0], ly = box[1], lz = box[2];
  const double ext = fmax(fmax(box[3] - lx, box[4] - ly), box[5] - lz);
  const double qmax = (double)((1 << MORTON_BITS) - 1);
  const double scale = ext > 0.0 ? qmax / ext : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double q[3] = {(pos[i] - lx) * scale, (pos[n + i] - ly) * scale, (pos[2 * n + i] - lz) * scale};
    uint32_t u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = (uint32_t)fmin(fmax(q[c], 0.0), qmax);
    keys[i] = (spread3(u[0]) << 2) | (spread3(u[1]) << 1) | spread3(u[2]);
    perm[i] = (int32_t)i;
  }
}

// The caller's rows packed into one 72-B record per particle (coalesced on
// both sides), so that the gather below reads one record per particle where
// it would read nine 8-B elements from nine scattered rows.
constexpr int PACK = 9;

__global__ void k_pack(int64_t n, const double *__restrict__ pos, const double *__restrict__ vel,
                       const double *__restrict__ m, const double *__restrict__ ro, const double *__restrict__ rs,
                       double *__restrict__ rec) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double *r = rec + PACK * i;
    r[0] = pos[i];
    r[1] = pos[n + i];
    r[2] = pos[2 * n + i];
    r[3] = vel[i];
    r[4] = vel[n + i];
    r[5] = vel[2 * n + i];
    r[6] = m[i];
    r[7] = ro[i];
    r[8] = rs[i];
  }
}

__global__ void k_gather(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ rec,
                         double *__restrict__ sx, double *__restrict__ sy, double *__restrict__ sz,
                         double *__restrict__ svx, double *__restrict__ svy, double *__restrict__ svz,
                         double *__restrict__ sm, double *__restrict__ sro, double *__restrict__ sinv,
                         double *__restrict__ sreach, double *__restrict__ srs, int32_t *__restrict__ sid,
                         unsigned long long *__restrict__ n_chunks) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_chunks = 0;  // the radix tree that follows lists the chunk roots
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = perm[k];
    const double *r = rec + PACK * i;
    sx[k] = r[0];
    sy[k] = r[1];
    sz[k] = r[2];
    svx[k] = r[3];
    svy[k] = r[4];
    svz[k] = r[5];
    sm[k] = r[6];
    const double o = r[7], s = r[8];
    sro[k] = o;
    sinv[k] = 1.0 / o;
    sreach[k] = fmax(o, s);
    srs[k] = s;
    sid[k] = (int32_t)i;
  }
}

// new positions and masses into the sorted arrays of the current order
__global__ void k_regather_xm(int64_t n, const int32_t *__restrict__ sid, const double *__restrict__ pos,
                              const double *__restrict__ m, double *__restrict__ sx, double *__restrict__ sy,
                              double *__restrict__ sz, double *__restrict__ sm) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = sid[k];
    sx[k] = pos[i];
    sy[k] = pos[n + i];
    sz[k] = pos[2 * n + i];
    sm[k] = m[i];
  }
}

// leaves per subtree of the bottom-up moments' first phase (see below)
constexpr int CHUNK = 1024;

// common-prefix length of sorted keys i and j (positions break ties)
__device__ __forceinline__ int prefix_len(const uint64_t *__restrict__ k, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  const uint64_t a = k[i], b = k[j];
  if (a == b) return 64 + __clz((unsigned)(i ^ j));
  return __clzll(a ^ b);
}

// Internal node i of the binary radix tree: its key range and split.
// Also lists the chunk roots of the moments pass (nodes of at most CHUNK
// leaves whose parent has more; the root if it has at most CHUNK; each is
// appended by its parent, the root by node 0's thread, n_chunks zeroed
// before the launch; their order does not matter) and clears the arrival
// counter of every internal node.
__global__ void k_radix_tree(int n, const uint64_t *__restrict__ k, p3t::WalkNode *__restrict__ wn,
                             int32_t *__restrict__ parent, int32_t *__restrict__ chunk_list,
                             unsigned long long *__restrict__ n_chunks, int32_t *__restrict__ visit) {
  const int leaf0 = n - 1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n - 1; i += gridDim.x * blockDim.x) {
    const int d = (prefix_len(k, n, i, i + 1) - prefix_len(k, n, i, i - 1)) > 0 ? 1 : -1;
    const int dmin = prefix_len(k, n, i, i - d);
    int lmax = 2;
    while (prefix_len(k, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
      if (prefix_len(k, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = prefix_len(k, n, i, j);
    int s = 0, t = l;
    do {
      t = (t + 1) >> 1;
      if (prefix_len(k, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int split = i + s * d + (d < 0 ? -1 : 0);
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    const int left = (lo == split) ? leaf0 + split : split;
    const int right = (hi == split + 1) ? leaf0 + split + 1 : split + 1;
    wn[i].left = left;
    wn[i].right = right;
    wn[i].first = lo;
    wn[i].count = hi - lo + 1;
    parent[left] = i;
    parent[right] = i;
    if (i == 0) parent[0] = -1;  // node 0 is the root and never a child
    visit[i] = 0;
    const int count = hi - lo + 1;
    const int cl = (lo == split) ? 1 : split - lo + 1, cr = (hi == split + 1) ? 1 : hi - split;
    if (count > CHUNK) {
      if (cl <= CHUNK) chunk_list[atomicAdd(n_chunks, 1ull)] = left;
      if (cr <= CHUNK) chunk_list[atomicAdd(n_chunks, 1ull)] = right;
    } else if (i == 0) {
      chunk_list[atomicAdd(n_chunks, 1ull)] = 0;
    }
  }
}

__device__ __forceinline__ void quad_shift(double q[6], double m, double dx, double dy, double dz) {
  // add m (3 d d^T - |d|^2 I) for a point mass m at offset d from the new centre
  const double d2 = dx * dx + dy * dy + dz * dz;
  q[0] += m * (3.0 * dx * dx - d2);
  q[1] += m * (3.0 * dy * dy - d2);
  q[2] += m * (3.0 * dz * dz - d2);
  q[3] += m * 3.0 * dx * dy;
  q[4] += m * 3.0 * dx * dz;
  q[5] += m * 3.0 * dy * dz;
}

// Internal node from its two children: tight box, mass, centre of mass,
// traceless quadrupole about the centre of mass (parallel-axis shift of each
// child's moment), max reach.  Fixed order (left, right): deterministic.
__device__ __forceinline__ void combine_node(int node, p3t::WalkNode *wn, p3t::CellMom *cm) {
  const int a = wn[node].left, b = wn[node].right;
  const p3t::WalkNode wa = wn[a], wb = wn[b];
  const p3t::CellMom ca = cm[a], cb = cm[b];
  p3t::WalkNode o;
  p3t::CellMom co;
  const double M = ca.mass + cb.mass;
  co.mass = M;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    o.lo[d] = fmin(wa.lo[d], wb.lo[d]);
    o.hi[d] = fmax(wa.hi[d], wb.hi[d]);
    co.com[d] = M > 0.0 ? (ca.mass * ca.com[d] + cb.mass * cb.com[d]) / M : 0.5 * (o.lo[d] + o.hi[d]);
    o.com[d] = co.com[d];
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) co.q[q] = ca.q[q] + cb.q[q];
  quad_shift(co.q, ca.mass, ca.com[0] - co.com[0], ca.com[1] - co.com[1], ca.com[2] - co.com[2]);
  quad_shift(co.q, cb.mass, cb.com[0] - co.com[0], cb.com[1] - co.com[1], cb.com[2] - co.com[2]);
  o.reach = fmax(wa.reach, wb.reach);
  // range and children are already in the record (and may be read meanwhile)
  p3t::WalkNode &w = wn[node];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    w.lo[d] = o.lo[d];
    w.hi[d] = o.hi[d];
    w.com[d] = o.com[d];
  }
  w.reach = o.reach;
  cm[node] = co;
}

// Bottom-up moments in two phases so that every hand-over between threads
// stays inside one workgroup (workgroup-scope fences only; device-scope
// fences would write back and invalidate the L2 of every XCD per level).
//   chunk roots: nodes with <= CHUNK leaves whose parent has more;
//   phase 1: one workgroup per chunk writes the leaf records and climbs to the
//            chunk root (second arrival at a node combines its children);
//   phase 2: one workgroup climbs from every chunk root to the tree root.
// (CHUNK is defined with the radix tree, which flags the chunk roots.)

__global__ void k_chunk_flag(int n, const p3t::WalkNode *__restrict__ wn, const int32_t *__restrict__ parent,
                             int32_t *__restrict__ flag) {
  const int n_nodes = 2 * n - 1, leaf0 = n - 1;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n_nodes; g += gridDim.x * blockDim.x) {
    const int c = g >= leaf0 ? 1 : wn[g].count;
    const int p = (g == 0) ? -1 : parent[g];
    flag[g] = (c <= CHUNK && (p < 0 || wn[p].count > CHUNK)) ? 1 : 0;
  }
}

__global__ void k_chunk_compact(int n_nodes, const int32_t *__restrict__ flag, const int64_t *__restrict__ pos,
                                int32_t *__restrict__ chunk, p3t::DevCounters *cnt) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n_nodes; g += gridDim.x * blockDim.x)
    if (flag[g]) chunk[pos[g]] = g;
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt->n_chunks = (unsigned long long)pos[n_nodes];
}

// What a parent needs of a child: box, centre of mass, mass, quadrupole,
// reach (136 B).  The chunk's internal nodes keep theirs in LDS while the
// climb runs; a leaf's comes from the particle arrays.
struct NodeRec {
  double lo[3], hi[3], com[3];
  double mass, reach;
  double q[6];
};
static_assert(sizeof(NodeRec) == 136, "NodeRec layout");

// Bottom-up within one chunk, the records of its internal nodes in LDS: a
// subtree of the radix tree over leaves [first, first + count) numbers its
// count - 1 internal nodes inside [first, first + count), so node - first
// indexes a slot.  Same arithmetic, in the same order, as combine_node.
//
// Only the records that something reads are written to device memory: the
// walk stops at the first node of at most n_leaf particles, so it reads a
// node (box, centre, reach, range) only if the node's parent holds more than
// n_leaf particles, and the force kernels read the moments of such nodes
// when they are accepted as cells; the chunk roots are read by the top
// climb.  Below that level the climb keeps its records in LDS only (most of
// the 2n - 1 nodes: about 90% at n_leaf = 16).  A particle's moment record
// is needed only when it is a chunk root itself.
constexpr int MOM_T = 1024;

__global__ __launch_bounds__(MOM_T) void k_moments_local(int n, const double *__restrict__ sx,
                                                         const double *__restrict__ sy, const double *__restrict__ sz,
                                                         const double *__restrict__ sm,
                                                         const double *__restrict__ sreach, p3t::WalkNode *wn,
                                                         p3t::CellMom *cm, const int32_t *__restrict__ parent,
                                                         int32_t *visit, const int32_t *__restrict__ chunk,
                                                         p3t::DevCounters *cnt, int n_leaf) {
  __shared__ __align__(16) NodeRec rec[CHUNK];
  __shared__ int lvisit[CHUNK];
  __shared__ int tleft[CHUNK], tright[CHUNK], tpar[CHUNK];  // the chunk's topology
  __shared__ unsigned char wide[CHUNK];  // internal node first + t holds more than n_leaf particles
  const int leaf0 = n - 1;
  const int nch = (int)cnt->n_chunks;
  auto child = [&](int c, int first, int count, NodeRec &o) -> bool {
    if (c >= leaf0) {
      const int k = c - leaf0;
      o.lo[0] = o.hi[0] = o.com[0] = sx[k];
      o.lo[1] = o.hi[1] = o.com[1] = sy[k];
      o.lo[2] = o.hi[2] = o.com[2] = sz[k];
      o.mass = sm[k];
      o.reach = sreach[k];
#pragma unroll
      for (int q = 0; q < 6; ++q) o.q[q] = 0.0;
      return true;
    }
    const unsigned off = (unsigned)(c - first);
    if (off >= (unsigned)count) return false;
    o = rec[off];
    return true;
  };
  for (int ci = blockIdx.x; ci < nch; ci += gridDim.x) {
    const int r = chunk[ci];
    const int first = r >= leaf0 ? r - leaf0 : wn[r].first;
    const int count = r >= leaf0 ? 1 : min(wn[r].count, CHUNK);
    for (int t = threadIdx.x; t < CHUNK; t += blockDim.x) lvisit[t] = 0;
    for (int t = threadIdx.x; t < count; t += blockDim.x) {
      const int node = first + t;
      if (node < leaf0) {  // one index of the range may be a node outside the subtree: loaded, never used
        tleft[t] = wn[node].left;
        tright[t] = wn[node].right;
        tpar[t] = parent[node];
        wide[t] = wn[node].count > n_leaf ? 1 : 0;
      }
    }
    __syncthreads();
    // is the record of node c (in this chunk) read later: the chunk root,
    // or a node whose parent (then inside the chunk) is wider than a leaf
    auto needed = [&](int c, int par) -> bool {
      if (c == r) return true;
      const unsigned po = (unsigned)(par - first);
      return po < (unsigned)count && wide[po];
    };
    // leaf records, staged in the (still unused) record slots and written
    // out as consecutive 16-B words: 96-B and 80-B records stored lane by
    // lane would leave every store instruction on scattered partial lines
    static_assert(CHUNK * sizeof(p3t::WalkNode) <= sizeof(rec) && CHUNK * sizeof(p3t::CellMom) <= sizeof(rec),
                  "leaf records exceed the staging area");
    p3t::WalkNode *lw = reinterpret_cast<p3t::WalkNode *>(rec);
    const uint4 *stage = reinterpret_cast<const uint4 *>(rec);
    // the leaves whose walk record is read (staged, then written as 16-B words)
    for (int t = threadIdx.x; t < count; t += blockDim.x) {
      const int k = first + t;
      const int leaf = leaf0 + k;
      lvisit[t] = needed(leaf, leaf == r ? -1 : parent[leaf]) ? 1 : 0;  // reset below, before the climb
      p3t::WalkNode w;
      w.lo[0] = w.hi[0] = w.com[0] = sx[k];
      w.lo[1] = w.hi[1] = w.com[1] = sy[k];
      w.lo[2] = w.hi[2] = w.com[2] = sz[k];
      w.reach = sreach[k];
      w.first = k;
      w.count = 1;
      w.left = -1;
      w.right = -1;
      lw[t] = w;
    }
    __syncthreads();
    {
      uint4 *dst = reinterpret_cast<uint4 *>(wn + leaf0 + first);
      constexpr int WPR = (int)(sizeof(p3t::WalkNode) / sizeof(uint4));
      const int words = count * WPR;
      for (int q = threadIdx.x; q < words; q += blockDim.x)
        if (lvisit[q / WPR]) dst[q] = stage[q];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < count; t += blockDim.x) lvisit[t] = 0;
    if (r >= leaf0 && threadIdx.x == 0) {  // a chunk of one particle: the top climb reads its moments
      const int k = r - leaf0;
      p3t::CellMom c;
      c.com[0] = sx[k];
      c.com[1] = sy[k];
      c.com[2] = sz[k];
      c.mass = sm[k];
#pragma unroll
      for (int q = 0; q < 6; ++q) c.q[q] = 0.0;
      cm[r] = c;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < count; t += blockDim.x) {
      const int leaf = leaf0 + first + t;
      int node = (leaf == r) ? -1 : parent[leaf];
      while (node >= 0) {
        const unsigned off = (unsigned)(node - first);
        if (off >= (unsigned)count) {  // not a radix subtree: reported, never indexed
          p3t::set_flag(cnt, P3T_FLAG_NAN);
          break;
        }
        // first arrival: the sibling will finish; only the second arrival
        // combines (a third would mean a malformed tree: stop, never loop)
        if (atomicAdd(&lvisit[off], 1) != 1) break;
        // the sibling's record is in LDS: order LDS only (the global
        // records are read by later kernels)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        const int a = tleft[off], b = tright[off];
        NodeRec ra, rb;
        if (!child(a, first, count, ra) || !child(b, first, count, rb)) {
          p3t::set_flag(cnt, P3T_FLAG_NAN);
          break;
        }
        NodeRec o;
        const double M = ra.mass + rb.mass;
        o.mass = M;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          o.lo[d] = fmin(ra.lo[d], rb.lo[d]);
          o.hi[d] = fmax(ra.hi[d], rb.hi[d]);
          o.com[d] = M > 0.0 ? (ra.mass * ra.com[d] + rb.mass * rb.com[d]) / M : 0.5 * (o.lo[d] + o.hi[d]);
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) o.q[q] = ra.q[q] + rb.q[q];
        quad_shift(o.q, ra.mass, ra.com[0] - o.com[0], ra.com[1] - o.com[1], ra.com[2] - o.com[2]);
        quad_shift(o.q, rb.mass, rb.com[0] - o.com[0], rb.com[1] - o.com[1], rb.com[2] - o.com[2]);
        o.reach = fmax(ra.reach, rb.reach);
        rec[off] = o;
        if (needed(node, tpar[off])) {
          // the node's range and children are already in its record
          p3t::WalkNode &wo = wn[node];
          p3t::CellMom co;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            wo.lo[d] = o.lo[d];
            wo.hi[d] = o.hi[d];
            wo.com[d] = o.com[d];
            co.com[d] = o.com[d];
          }
          wo.reach = o.reach;
          co.mass = M;
#pragma unroll
          for (int q = 0; q < 6; ++q) co.q[q] = o.q[q];
          cm[node] = co;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        if (node == r) break;
        node = tpar[off];
      }
    }
    __syncthreads();
  }
}

constexpr int TOP_SLOTS = 4096;  // power of two
constexpr int TOP_PROBES = 32;   // probes per node before it falls back to its counter in device memory

// Workgroup 0 climbs from every chunk root to the root; the other
// workgroups meanwhile flag the interaction groups, which need only the node
// counts (group g: count(g) <= ng and g is the root or count(parent) > ng).
__global__ __launch_bounds__(1024) void k_moments_top(p3t::WalkNode *wn, p3t::CellMom *cm,
                                                      const int32_t *__restrict__ parent, int32_t *visit,
                                                      const int32_t *__restrict__ chunk, const p3t::DevCounters *cnt,
                                                      int n_nodes, int ng, int32_t *__restrict__ flag,
                                                      int slots) {
  if (blockIdx.x > 0) {
    // (a particle's record may not be written: its count is 1)
    const int leaf0 = (n_nodes - 1) / 2;
    for (int g = (blockIdx.x - 1) * blockDim.x + threadIdx.x; g < n_nodes; g += (gridDim.x - 1) * blockDim.x) {
      const int c = g >= leaf0 ? 1 : wn[g].count;
      const int p = (g == 0) ? -1 : parent[g];
      flag[g] = (c <= ng && (p < 0 || wn[p].count > ng)) ? 1 : 0;
    }
    return;
  }
  // Arrival counters of the top nodes in an LDS hash table of `slots`
  // entries (a power of two <= TOP_SLOTS; open addressing on the node id).
  // A node that finds neither its key nor a free entry within TOP_PROBES
  // probes uses its counter in device memory.  Keys are never removed, so the
  // entries a node probes only ever fill: both arrivals at a node see the
  // same probe sequence and make the same choice (the second finds the key
  // the first stored, or the same entries taken by other nodes).
  __shared__ int hkey[TOP_SLOTS], hcnt[TOP_SLOTS];
  const unsigned mask = (unsigned)slots - 1u;
  const int probes = slots < TOP_PROBES ? slots : TOP_PROBES;
  for (int q = threadIdx.x; q < slots; q += blockDim.x) {
    hkey[q] = -1;
    hcnt[q] = 0;
  }
  __syncthreads();
  const int nch = (int)cnt->n_chunks;
  for (int ci = threadIdx.x; ci < nch; ci += blockDim.x) {
    const int r = chunk[ci];
    int node = r == 0 ? -1 : parent[r];
    while (node >= 0) {
      unsigned h = ((unsigned)node * 2654435761u) & mask;
      int slot = -1;
      for (int probe = 0; probe < probes; ++probe) {
        const int k = atomicCAS(&hkey[h], -1, node);
        if (k == -1 || k == node) {
          slot = (int)h;
          break;
        }
        h = (h + 1) & mask;
      }
      const int prev = slot >= 0 ? atomicAdd(&hcnt[slot], 1) : atomicAdd(&visit[node], 1);
      if (prev != 1) break;
      __threadfence_block();
      combine_node(node, wn, cm);
      __threadfence_block();
      node = parent[node];
    }
  }
}

__global__ void k_group_compact(int n_nodes, const int32_t *__restrict__ flag, const int64_t *__restrict__ pos,
                                int32_t *__restrict__ group_node, p3t::DevCounters *cnt) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n_nodes; g += gridDim.x * blockDim.x)
    if (flag[g]) group_node[pos[g]] = g;
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt->n_groups = (unsigned long long)pos[n_nodes];
}

static inline unsigned g1d(int64_t n, int64_t cap = 65536) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

static hipError_t moments_pass(p3t_ctx *c, int64_t n, bool chunks_ready);

hipError_t build_tree(p3t_ctx *c, int64_t n, const double *pos3, const double *vel3, const double *mass,
                      const double *r_out, const double *r_search) {
  hipStream_t s = c->stream;
  hipError_t e;
  if ((e = bbox_reduce(pos3, n, c->bbox_part, c->bbox, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_morton, dim3(g1d(n)), dim3(256), 0, s, n, pos3, c->bbox, c->keys, c->perm);
  uint64_t *k = c->keys, *ka = c->keys_alt;
  int32_t *v = c->perm, *va = c->perm_alt;
  ev_record(c, 17);
  if ((e = radix_sort_pairs(k, v, ka, va, n, nullptr, 0, 3 * MORTON_BITS, c->radix_hist, c->radix_hist_cap, c->scan_tmp,
                            c->scan_tmp_cap, s)) != hipSuccess)
    return e;
  ev_record(c, 18);
  // after an even number of passes the result is back in keys / perm.  The
  // node records are rebuilt below, so their storage (96 B per node, 2n - 1
  // nodes) holds the packed rows until then.
  static_assert(PACK * sizeof(double) <= 2 * sizeof(WalkNode), "packed rows exceed the node storage");
  double *rec = reinterpret_cast<double *>(c->wnode);
  hipLaunchKernelGGL(k_pack, dim3(g1d(n)), dim3(256), 0, s, n, pos3, vel3, mass, r_out, r_search, rec);
  hipLaunchKernelGGL(k_gather, dim3(g1d(n)), dim3(256), 0, s, n, v, rec, c->sx, c->sy, c->sz, c->svx, c->svy, c->svz,
                     c->sm, c->sro, c->sinv, c->sreach, c->srs, c->sid,
                     &c->cnt->n_chunks);
  if (n > 1) {
    hipLaunchKernelGGL(k_radix_tree, dim3(g1d(n - 1)), dim3(256), 0, s, (int)n, k, c->wnode, c->parent,
                       c->group_node, &c->cnt->n_chunks, c->visit);
  }
  return moments_pass(c, n, n > 1);
}

// Moments, boxes and groups of the current topology (the bottom-up pass);
// chunks_ready: the radix tree has just listed the chunk roots and cleared
// the arrival counters.
static hipError_t moments_pass(p3t_ctx *c, int64_t n, bool chunks_ready) {
  hipStream_t s = c->stream;
  hipError_t e;
  const int64_t n_nodes = 2 * n - 1;
  if (!chunks_ready) {
    if ((e = fill_i32(c->visit, 0, n > 1 ? n - 1 : 1, s)) != hipSuccess) return e;
    // chunk roots (into group_node / node_scan, both free until the groups are formed)
    hipLaunchKernelGGL(k_chunk_flag, dim3(g1d(n_nodes)), dim3(256), 0, s, (int)n, c->wnode, c->parent, c->group_flag);
    if ((e = scan_i32_to_i64(c->group_flag, c->node_scan, n_nodes, c->scan_tmp, c->scan_tmp_cap, s)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_chunk_compact, dim3(g1d(n_nodes)), dim3(256), 0, s, (int)n_nodes, c->group_flag,
                       c->node_scan, c->group_node, c->cnt);
  }
  hipLaunchKernelGGL(k_moments_local, dim3(c->n_cu * 2), dim3(MOM_T), 0, s, (int)n, c->sx, c->sy, c->sz, c->sm,
                     c->sreach, c->wnode, c->cmom, c->parent, c->visit, c->group_node, c->cnt, c->P.n_leaf_max);
  const unsigned gflag = (unsigned)std::max<int64_t>(1, std::min<int64_t>(2048, (n_nodes + 1023) / 1024));
  hipLaunchKernelGGL(k_moments_top, dim3(1 + gflag), dim3(1024), 0, s, c->wnode, c->cmom, c->parent, c->visit,
                     c->group_node, c->cnt, (int)n_nodes, c->P.n_group_max, c->group_flag, c->top_slots);
  if ((e = scan_i32_to_i64(c->group_flag, c->node_scan, n_nodes, c->scan_tmp, c->scan_tmp_cap, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_group_compact, dim3(g1d(n_nodes)), dim3(256), 0, s, (int)n_nodes, c->group_flag, c->node_scan,
                     c->group_node, c->cnt);
  return hipGetLastError();
}

// the bottom-up pass over the current topology (its chunk roots flagged anew)
hipError_t tree_moments(p3t_ctx *c, int64_t n) { return moments_pass(c, n, false); }

// Same topology, same lists: positions and masses replaced, moments redone.
hipError_t refresh_tree(p3t_ctx *c, const double *pos3, const double *mass) {
  const int64_t n = c->n;
  hipLaunchKernelGGL(k_regather_xm, dim3(g1d(n)), dim3(256), 0, c->stream, n, c->sid, pos3, mass, c->sx, c->sy, c->sz,
                     c->sm);
  return tree_moments(c, n);
}

}  // namespace p3t
