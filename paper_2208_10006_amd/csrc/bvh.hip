// bvh.hip -- BVH over primitive boxes, built on the GPU.  Both builders
// start from 30-bit Morton codes of the primitive centroids, stably radix
// sorted (ties keep primitive order, so the key (code, index) is unique):
//  * up to kPlocMax primitives: PLOC clustering in one workgroup (Meister and
//    Bittner 2018), which gives surface-area-aware trees;
//  * beyond: the linear BVH of Karras 2012 ("Maximizing Parallelism in the
//    Construction of BVHs, Octrees, and k-d Trees"): one thread per internal
//    node finds its key range and split from the longest common prefix, then
//    a bottom-up box refit where the second thread to reach a node (atomic
//    counter, acquire/release) merges its two children.
//
// Node layout (64 B, four float4): both child boxes inline so one node fetch
// serves the two slab tests of the traversal:
//   [0] Llo.x Llo.y Llo.z Lhi.x  [1] Lhi.y Lhi.z Rlo.x Rlo.y
//   [2] Rlo.z Rhi.x Rhi.y Rhi.z  [3] childL childR (int; leaf = ~sorted index)
// The root is node 0.  Leaf boxes are widened by one float ulp on each side
// so that they also contain the FP64 geometry the FP32 vertices were rounded
// from.
#include "sbr_device.hpp"
#include "sbr_internal.hpp"
#include "lds_sort.hpp"

namespace sbr {
namespace {

__device__ inline uint32_t spread10(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// 30-bit Morton code of primitive i's box centre, quantised to 1024 cells per
// axis of the scene box slo + [0, 1/inv_ext]
__device__ inline uint32_t morton_code(const float* __restrict__ lo, const float* __restrict__ hi, int64_t i,
                                       float3 slo, float3 inv_ext) {
  const float cx = 0.5f * (lo[3 * i] + hi[3 * i]);
  const float cy = 0.5f * (lo[3 * i + 1] + hi[3 * i + 1]);
  const float cz = 0.5f * (lo[3 * i + 2] + hi[3 * i + 2]);
  auto q = [](float c, float l, float ie) {
    float u = (c - l) * ie;
    u = fminf(fmaxf(u, 0.0f), 1.0f);
    return (uint32_t)fminf(u * 1024.0f, 1023.0f);
  };
  return (spread10(q(cx, slo.x, inv_ext.x)) << 2) | (spread10(q(cy, slo.y, inv_ext.y)) << 1) |
         spread10(q(cz, slo.z, inv_ext.z));
}

// Quantised centroid positions in the scene box slo + [0, 1/inv_ext]; with
// bounds (device lo xyz, hi xyz) the box comes from there, by the same float
// operations the host uses.
__global__ void k_morton(const float* __restrict__ lo, const float* __restrict__ hi, int64_t n, float3 slo,
                         float3 inv_ext, const float* __restrict__ bounds, uint64_t* __restrict__ code,
                         uint32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (bounds) {
    slo = make_float3(bounds[0], bounds[1], bounds[2]);
    inv_ext.x = bounds[3] > bounds[0] ? 1.0f / (bounds[3] - bounds[0]) : 0.0f;
    inv_ext.y = bounds[4] > bounds[1] ? 1.0f / (bounds[4] - bounds[1]) : 0.0f;
    inv_ext.z = bounds[5] > bounds[2] ? 1.0f / (bounds[5] - bounds[2]) : 0.0f;
  }
  code[i] = morton_code(lo, hi, i, slo, inv_ext);
  idx[i] = (uint32_t)i;
}

__device__ inline int delta(const uint64_t* code, int64_t n, int64_t i, int64_t j) {
  if (j < 0 || j >= n) return -1;
  const uint64_t a = code[i], b = code[j];
  if (a == b) return 64 + __clz((uint32_t)(i ^ j));
  return __clzll(a ^ b);
}

// Children of internal node i of the Karras hierarchy over n sorted codes
// (unique as (code, index)): its key range from the longest common prefix,
// then the split; a child is a leaf (~index) when its range is one key.
__device__ inline void karras_node(const uint64_t* code, int64_t n, int64_t i, int32_t& cl, int32_t& cr) {
  const int d = (delta(code, n, i, i + 1) - delta(code, n, i, i - 1)) >= 0 ? 1 : -1;
  const int dmin = delta(code, n, i, i - d);
  int64_t lmax = 2;
  while (delta(code, n, i, i + lmax * d) > dmin) lmax <<= 1;
  int64_t l = 0;
  for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
    if (delta(code, n, i, i + (l + t) * d) > dmin) l += t;
  const int64_t j = i + l * d;
  const int dnode = delta(code, n, i, j);
  int64_t s = 0, t = l;
  do {
    t = (t + 1) >> 1;
    if (delta(code, n, i, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  const int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
  const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
  cl = lo == gamma ? ~(int32_t)gamma : (int32_t)gamma;
  cr = hi == gamma + 1 ? ~(int32_t)(gamma + 1) : (int32_t)(gamma + 1);
}

__global__ void k_karras(const uint64_t* __restrict__ code, int64_t n, float4* __restrict__ nodes,
                         int32_t* __restrict__ parent_int, int32_t* __restrict__ parent_leaf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  int32_t cl, cr;
  karras_node(code, n, i, cl, cr);
  if (cl < 0) parent_leaf[~cl] = (int32_t)i;
  else parent_int[cl] = (int32_t)i;
  if (cr < 0) parent_leaf[~cr] = (int32_t)i;
  else parent_int[cr] = (int32_t)i;
  nodes[4 * i + 3] = make_float4(__int_as_float(cl), __int_as_float(cr), 0.0f, 0.0f);
  if (i == 0) parent_int[0] = -1;
}

// write a child box into its parent's slot (component-wise: the sibling may
// be writing the other half of the same float4 concurrently)
__device__ inline void put_box(float4* nodes, int64_t p, bool right, const float* b /* lo3 hi3 */) {
  float* f = reinterpret_cast<float*>(nodes + 4 * p);
  const int off = right ? 6 : 0;
  for (int k = 0; k < 6; ++k) f[off + k] = b[k];
}

__global__ void k_refit(const float* __restrict__ lo, const float* __restrict__ hi, const uint32_t* __restrict__ order,
                        int64_t n, float4* nodes, const int32_t* __restrict__ parent_int,
                        const int32_t* __restrict__ parent_leaf, uint32_t* flags, float* root_box) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t prim = order[i];
  float b[6];
  for (int k = 0; k < 3; ++k) {
    b[k] = nextafterf(lo[3 * prim + k], -INFINITY);
    b[3 + k] = nextafterf(hi[3 * prim + k], INFINITY);
  }
  int64_t p = parent_leaf[i];
  {
    const float4 c = nodes[4 * p + 3];
    put_box(nodes, p, __float_as_int(c.y) == ~(int32_t)i, b);
  }
  while (true) {
    const uint32_t old = __hip_atomic_fetch_add(&flags[p], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (old == 0) return;  // the sibling subtree is not finished yet; it will continue
    const float* f = reinterpret_cast<const float*>(nodes + 4 * p);
    float u[6];
    for (int k = 0; k < 3; ++k) {
      u[k] = fminf(__hip_atomic_load(&f[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                   __hip_atomic_load(&f[6 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      u[3 + k] = fmaxf(__hip_atomic_load(&f[3 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                       __hip_atomic_load(&f[9 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    if (p == 0) {
      for (int k = 0; k < 6; ++k) root_box[k] = u[k];
      return;
    }
    const int64_t pp = parent_int[p];
    const float4 c = nodes[4 * pp + 3];
    put_box(nodes, pp, __float_as_int(c.y) == (int32_t)p, u);
    p = pp;
  }
}

__global__ void k_depth(const int32_t* __restrict__ parent_int, const int32_t* __restrict__ parent_leaf, int64_t n,
                        uint32_t* depth) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t d = 1;
  int64_t p = parent_leaf[i];
  while (p > 0) {
    p = parent_int[p];
    ++d;
  }
  atomicMax(depth, d);
}

// Small linear trees (receiver sets, small scenes) in one workgroup: the
// same Morton codes, stable sort, hierarchy and boxes as the multi-kernel
// path (so the same tree), with codes, links and node boxes in LDS.  The
// refit climbs from every leaf; an LDS counter per node lets the second
// arrival merge it (its sibling's box and height were stored before the
// sibling's release-increment), and node heights give the depth: the
// number of internal nodes on the longest root-to-leaf path.
__global__ __launch_bounds__(kSmallThreads) void k_lbvh_small(const float* __restrict__ lo,
                                                            const float* __restrict__ hi, int n, float3 slo,
                                                            float3 inv_ext, const float* __restrict__ bounds,
                                                            float4* __restrict__ nodes,
                                                            uint32_t* __restrict__ order, float* __restrict__ root_box,
                                                            uint32_t* __restrict__ depth) {
  if (bounds) {  // scene box from the device, by the same float operations as the host
    slo = make_float3(bounds[0], bounds[1], bounds[2]);
    inv_ext.x = bounds[3] > bounds[0] ? 1.0f / (bounds[3] - bounds[0]) : 0.0f;
    inv_ext.y = bounds[4] > bounds[1] ? 1.0f / (bounds[4] - bounds[1]) : 0.0f;
    inv_ext.z = bounds[5] > bounds[2] ? 1.0f / (bounds[5] - bounds[2]) : 0.0f;
  }
  __shared__ uint64_t lk[kLbvhSmall];
  __shared__ uint32_t lv[kLbvhSmall];
  __shared__ uint16_t hist[kSmallWaves][256];
  __shared__ uint32_t dsum[kSmallWaves / 4];
  __shared__ int32_t ch[kLbvhSmall][2];
  __shared__ int32_t par_int[kLbvhSmall], par_leaf[kLbvhSmall];
  __shared__ float nbox[kLbvhSmall][6];
  __shared__ uint32_t ht[kLbvhSmall], arrive[kLbvhSmall];
  const int t = threadIdx.x;
  for (int i = t; i < n; i += kSmallThreads) {
    lk[i] = morton_code(lo, hi, i, slo, inv_ext);
    lv[i] = (uint32_t)i;
    arrive[i] = 0;
  }
  __syncthreads();
  lds_radix_sort_pairs<kLbvhSmall / kSmallThreads>(lk, lv, hist, dsum, n, 0, 30);
  for (int i = t; i < n - 1; i += kSmallThreads) {
    int32_t cl, cr;
    karras_node(lk, n, i, cl, cr);
    ch[i][0] = cl, ch[i][1] = cr;
    if (cl < 0) par_leaf[~cl] = i;
    else par_int[cl] = i;
    if (cr < 0) par_leaf[~cr] = i;
    else par_int[cr] = i;
  }
  for (int i = t; i < n; i += kSmallThreads) order[i] = lv[i];
  __syncthreads();
  auto leaf_box = [&](int leaf, float* b) {
    const uint32_t prim = lv[leaf];
    for (int k = 0; k < 3; ++k) {
      b[k] = nextafterf(lo[3 * prim + k], -INFINITY);
      b[3 + k] = nextafterf(hi[3 * prim + k], INFINITY);
    }
  };
  for (int i = t; i < n; i += kSmallThreads) {
    int32_t p = par_leaf[i];
    while (true) {
      const uint32_t old = __hip_atomic_fetch_add(&arrive[p], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (old == 0) break;  // the other child is not finished; its climb continues here
      float b[2][6];
      uint32_t h = 0;
      for (int c = 0; c < 2; ++c) {
        const int32_t x = ch[p][c];
        if (x < 0) {
          leaf_box(~x, b[c]);
        } else {
          for (int k = 0; k < 6; ++k) b[c][k] = nbox[x][k];
          h = max(h, ht[x]);
        }
      }
      float u[6];
      for (int k = 0; k < 3; ++k) u[k] = fminf(b[0][k], b[1][k]), u[3 + k] = fmaxf(b[0][3 + k], b[1][3 + k]);
      for (int k = 0; k < 6; ++k) nbox[p][k] = u[k];
      ht[p] = h + 1;
      float4* o = nodes + 4 * (int64_t)p;
      o[0] = make_float4(b[0][0], b[0][1], b[0][2], b[0][3]);
      o[1] = make_float4(b[0][4], b[0][5], b[1][0], b[1][1]);
      o[2] = make_float4(b[1][2], b[1][3], b[1][4], b[1][5]);
      o[3] = make_float4(__int_as_float(ch[p][0]), __int_as_float(ch[p][1]), 0.0f, 0.0f);
      if (p == 0) {
        for (int k = 0; k < 6; ++k) root_box[k] = u[k];
        *depth = h + 1;
        break;
      }
      p = par_int[p];
    }
  }
}

__global__ void k_single_leaf(const float* __restrict__ lo, const float* __restrict__ hi, float4* nodes,
                              uint32_t* order, float* root_box) {
  float b[6];
  for (int k = 0; k < 3; ++k) {
    b[k] = nextafterf(lo[k], -INFINITY);
    b[3 + k] = nextafterf(hi[k], INFINITY);
  }
  float* f = reinterpret_cast<float*>(nodes);
  for (int k = 0; k < 6; ++k) f[k] = b[k];
  for (int k = 0; k < 3; ++k) {  // empty right box: never intersected
    f[6 + k] = INFINITY;
    f[9 + k] = -INFINITY;
  }
  nodes[3] = make_float4(__int_as_float(~0), __int_as_float(~0), 0.0f, 0.0f);
  order[0] = 0;
  for (int k = 0; k < 6; ++k) root_box[k] = b[k];
}

// ---------------------------------------------------------------------------
// PLOC (Meister and Bittner 2018, "Parallel Locally-Ordered Clustering for
// Bounding Volume Hierarchy Construction"), one workgroup.  The clusters start
// as the Morton-ordered leaves.  Each pass, every cluster finds its nearest
// neighbour among the kPlocR clusters on either side (distance = surface area
// of the merged box; ties ordered by the pair's indices, which makes the order
// on pairs strict, so the closest pair is always mutual and every pass merges
// at least one pair); mutual neighbours merge into a new node at the lower
// position, and a block scan compacts the cluster array.  Internal nodes are
// numbered downward from n - 2 in creation order, so the last merge, the
// root, is node 0.  The height and internal-node count of each cluster are
// carried along; the root's height is the tree depth.  A final top-down
// pass (passes in reverse, each node placing its children) renumbers the
// nodes in depth-first order, left child first, so that every subtree is a
// contiguous range of nodes, as in the linear BVH: the rays of a wave walking
// nearby subtrees then share cache lines.
constexpr int kPlocThreads = 1024, kPlocR = 16, kPlocTile = kPlocThreads + 2 * kPlocR;
constexpr int kPlocLds = 2 * kPlocThreads;  // clusters kept in LDS for the last passes
constexpr int kPlocLdsNodes = 2 * kPlocLds;  // trees relabelled in LDS (4 ints per node in lb)
constexpr int64_t kPlocMax = kBvhPlocMax;  // pair keys hold two 16-bit cluster indices
static_assert(kPlocMax <= 65536, "PLOC pair keys hold 16-bit cluster indices");

struct PlocArgs {
  const float* lo;  // primitive boxes [n][3]
  const float* hi;
  const uint32_t* order;  // Morton order of the primitives
  int n;
  float* box[2];    // cluster boxes, SoA: component c of cluster i at c * n + i
  int32_t* id[2];   // node index, or ~leaf
  int32_t* ht[2];   // subtree height in internal nodes
  int32_t* sz[2];   // internal nodes in the subtree
  int32_t* nn;      // nearest neighbour
  float4* tmp;      // nodes in creation order [n - 1][4]
  int32_t* nsz;     // internal nodes below and including each created node
  int32_t* dfs;     // depth-first number of each created node
  int32_t* pass_next;  // first free node index at the start of each pass [n + 1]
  float4* nodes;
  float* root_box;
  uint32_t* depth;
};

__device__ inline float merged_area(const float a[6], const float b[6]) {
  const float ex = fmaxf(a[3], b[3]) - fminf(a[0], b[0]);
  const float ey = fmaxf(a[4], b[4]) - fminf(a[1], b[1]);
  const float ez = fmaxf(a[5], b[5]) - fminf(a[2], b[2]);
  return ex * ey + ey * ez + ez * ex;
}

__global__ __launch_bounds__(kPlocThreads) void k_ploc(const PlocArgs A) {
  __shared__ float sb[6][kPlocTile];
  __shared__ uint32_t wsum[kPlocThreads / 64];
  // the passes with at most kPlocLds clusters keep them in LDS
  // lb rows 0-5 hold the cluster boxes; the eight rows are reused by the
  // relabelling of trees up to kPlocLdsNodes nodes (children, sizes, numbers)
  __shared__ float lb[8][kPlocLds];
  __shared__ int32_t lid[kPlocLds], lht[kPlocLds], lsz[kPlocLds], lnn[kPlocLds];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int n = A.n;
  for (int i = t; i < n; i += kPlocThreads) {
    const uint32_t p = A.order[i];
    for (int c = 0; c < 3; ++c) {
      A.box[0][c * n + i] = nextafterf(A.lo[3 * p + c], -INFINITY);
      A.box[0][(3 + c) * n + i] = nextafterf(A.hi[3 * p + c], INFINITY);
    }
    A.id[0][i] = ~i;
    A.ht[0][i] = 0;
    A.sz[0][i] = 0;
  }
  __syncthreads();
  int m = n, cur = 0, next = n - 2;
  // every pass merges at least one pair, so n - 1 passes always suffice; the
  // bound only guarantees that the loop ends
  int pass = 0;
  for (; m > kPlocLds && pass < n; ++pass) {
    if (t == 0) A.pass_next[pass] = next;
    const float* B = A.box[cur];
    // ---- nearest neighbours, one tile of kPlocThreads clusters at a time
    for (int base = 0; base < m; base += kPlocThreads) {
      for (int k = t; k < kPlocTile; k += kPlocThreads) {
        const int g = base - kPlocR + k;
        if (g >= 0 && g < m)
          for (int c = 0; c < 6; ++c) sb[c][k] = B[c * n + g];
      }
      __syncthreads();
      const int i = base + t;
      if (i < m) {
        float a[6];
        for (int c = 0; c < 6; ++c) a[c] = sb[c][t + kPlocR];
        uint64_t best = ~0ull;
        const int j0 = max(0, i - kPlocR), j1 = min(m - 1, i + kPlocR);
        for (int j = j0; j <= j1; ++j) {
          if (j == i) continue;
          float b[6];
          for (int c = 0; c < 6; ++c) b[c] = sb[c][j - base + kPlocR];
          const uint32_t lo = (uint32_t)min(i, j), hi = (uint32_t)max(i, j);
          const uint64_t key = ((uint64_t)__float_as_uint(merged_area(a, b)) << 32) | (lo << 16) | hi;
          best = key < best ? key : best;
        }
        const uint32_t lo = (uint32_t)(best >> 16) & 0xffffu, hi = (uint32_t)best & 0xffffu;
        A.nn[i] = min((int)(lo == (uint32_t)i ? hi : lo), m - 1);
      }
      __syncthreads();
    }
    // ---- merge mutual pairs into the other buffer, compacted
    float* Bo = A.box[cur ^ 1];
    int32_t* Io = A.id[cur ^ 1];
    int32_t* Ho = A.ht[cur ^ 1];
    int32_t* So = A.sz[cur ^ 1];
    int kept = 0, merged = 0;
    for (int base = 0; base < m; base += kPlocThreads) {
      const int i = base + t;
      int j = -1;
      bool keep = false, merge = false;
      if (i < m) {
        j = A.nn[i];
        const bool mutual = A.nn[j] == i;
        merge = mutual && i < j;
        keep = !mutual || i < j;
      }
      // keep counts in the low half, merge counts in the high half (<= kPlocThreads each)
      const uint32_t x = wave_inclusive_scan((keep ? 1u : 0u) | (merge ? 0x10000u : 0u), lane);
      if (lane == 63) wsum[wv] = x;
      __syncthreads();
      uint32_t before = 0, total = 0;
      for (int w = 0; w < kPlocThreads / 64; ++w) {
        const uint32_t sw = wsum[w];
        before += w < wv ? sw : 0u;
        total += sw;
      }
      const uint32_t excl = before + x - ((keep ? 1u : 0u) | (merge ? 0x10000u : 0u));
      if (keep) {
        const int pos = kept + (int)(excl & 0xffffu);
        float a[6];
        for (int c = 0; c < 6; ++c) a[c] = B[c * n + i];
        int32_t nid = A.id[cur][i], h = A.ht[cur][i], z = A.sz[cur][i];
        if (merge) {
          const int node = next - merged - (int)(excl >> 16);
          float b[6];
          for (int c = 0; c < 6; ++c) b[c] = B[c * n + j];
          const int32_t jid = A.id[cur][j];
          A.tmp[4 * node] = make_float4(a[0], a[1], a[2], a[3]);
          A.tmp[4 * node + 1] = make_float4(a[4], a[5], b[0], b[1]);
          A.tmp[4 * node + 2] = make_float4(b[2], b[3], b[4], b[5]);
          A.tmp[4 * node + 3] = make_float4(__int_as_float(nid), __int_as_float(jid), 0.0f, 0.0f);
          for (int c = 0; c < 3; ++c) a[c] = fminf(a[c], b[c]), a[3 + c] = fmaxf(a[3 + c], b[3 + c]);
          h = 1 + max(h, A.ht[cur][j]);
          z = 1 + z + A.sz[cur][j];
          A.nsz[node] = z;
          nid = node;
        }
        for (int c = 0; c < 6; ++c) Bo[c * n + pos] = a[c];
        Io[pos] = nid;
        Ho[pos] = h;
        So[pos] = z;
      }
      kept += (int)(total & 0xffffu);
      merged += (int)(total >> 16);
      __syncthreads();  // wsum is rewritten by the next tile
    }
    next -= merged;
    m = kept;
    cur ^= 1;
  }
  // ---- the remaining passes in LDS: each thread owns clusters t and
  // t + kPlocThreads, reads everything it needs, and after a barrier writes
  // the compacted clusters in place
  const bool in_lds = m <= kPlocLds;
  if (in_lds) {
    for (int i = t; i < m; i += kPlocThreads) {
      for (int c = 0; c < 6; ++c) lb[c][i] = A.box[cur][c * n + i];
      lid[i] = A.id[cur][i], lht[i] = A.ht[cur][i], lsz[i] = A.sz[cur][i];
    }
    __syncthreads();
    for (; m > 1 && pass < n; ++pass) {
      if (t == 0) A.pass_next[pass] = next;
      for (int i = t; i < m; i += kPlocThreads) {
        float a[6];
        for (int c = 0; c < 6; ++c) a[c] = lb[c][i];
        uint64_t best = ~0ull;
        const int j0 = max(0, i - kPlocR), j1 = min(m - 1, i + kPlocR);
        for (int j = j0; j <= j1; ++j) {
          if (j == i) continue;
          float b[6];
          for (int c = 0; c < 6; ++c) b[c] = lb[c][j];
          const uint32_t lo = (uint32_t)min(i, j), hi = (uint32_t)max(i, j);
          const uint64_t key = ((uint64_t)__float_as_uint(merged_area(a, b)) << 32) | (lo << 16) | hi;
          best = key < best ? key : best;
        }
        const uint32_t lo = (uint32_t)(best >> 16) & 0xffffu, hi = (uint32_t)best & 0xffffu;
        lnn[i] = min((int)(lo == (uint32_t)i ? hi : lo), m - 1);
      }
      __syncthreads();
      int kept = 0, merged = 0;
      bool wkeep[2];
      int wpos[2];
      float wbox[2][6];
      int32_t wid[2], wht[2], wsz[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int i = t + e * kPlocThreads;
        int j = -1;
        bool keep = false, merge = false;
        if (i < m) {
          j = lnn[i];
          const bool mutual = lnn[j] == i;
          merge = mutual && i < j;
          keep = !mutual || i < j;
        }
        const uint32_t x = wave_inclusive_scan((keep ? 1u : 0u) | (merge ? 0x10000u : 0u), lane);
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (int w = 0; w < kPlocThreads / 64; ++w) {
          const uint32_t sw = wsum[w];
          before += w < wv ? sw : 0u;
          total += sw;
        }
        const uint32_t excl = before + x - ((keep ? 1u : 0u) | (merge ? 0x10000u : 0u));
        wkeep[e] = keep;
        wpos[e] = kept + (int)(excl & 0xffffu);
        if (keep) {
          for (int c = 0; c < 6; ++c) wbox[e][c] = lb[c][i];
          wid[e] = lid[i], wht[e] = lht[i], wsz[e] = lsz[i];
          if (merge) {
            const int node = next - merged - (int)(excl >> 16);
            float b[6];
            for (int c = 0; c < 6; ++c) b[c] = lb[c][j];
            const float* a = wbox[e];
            A.tmp[4 * node] = make_float4(a[0], a[1], a[2], a[3]);
            A.tmp[4 * node + 1] = make_float4(a[4], a[5], b[0], b[1]);
            A.tmp[4 * node + 2] = make_float4(b[2], b[3], b[4], b[5]);
            A.tmp[4 * node + 3] = make_float4(__int_as_float(wid[e]), __int_as_float(lid[j]), 0.0f, 0.0f);
            for (int c = 0; c < 3; ++c)
              wbox[e][c] = fminf(wbox[e][c], b[c]), wbox[e][3 + c] = fmaxf(wbox[e][3 + c], b[3 + c]);
            wht[e] = 1 + max(wht[e], lht[j]);
            wsz[e] = 1 + wsz[e] + lsz[j];
            A.nsz[node] = wsz[e];
            wid[e] = node;
          }
        }
        kept += (int)(total & 0xffffu);
        merged += (int)(total >> 16);
        __syncthreads();  // wsum is rewritten next; all reads of this pass are done after the last one
      }
#pragma unroll
      for (int e = 0; e < 2; ++e)
        if (wkeep[e]) {
          const int pos = wpos[e];
          for (int c = 0; c < 6; ++c) lb[c][pos] = wbox[e][c];
          lid[pos] = wid[e], lht[pos] = wht[e], lsz[pos] = wsz[e];
        }
      __syncthreads();
      next -= merged;
      m = kept;
    }
  }
  if (t == 0) {
    if (in_lds) {
      for (int c = 0; c < 6; ++c) A.root_box[c] = lb[c][0];
    }
    *A.depth = in_lds && m == 1 ? (uint32_t)lht[0] : 0xffffffffu;
    A.pass_next[pass] = next;  // = -1 once the root exists
    A.dfs[0] = 0;
  }
  if (!in_lds || m != 1) return;
  __syncthreads();
  // ---- depth-first numbering: a node's parent was created in a later pass,
  // so walking the passes backwards numbers every parent before its children
  if (n - 1 <= kPlocLdsNodes) {
    // in LDS: children, sizes and numbers of every node
    int32_t* rcl = reinterpret_cast<int32_t*>(&lb[0][0]);
    int32_t* rcr = rcl + kPlocLdsNodes;
    int32_t* rsz = rcr + kPlocLdsNodes;
    int32_t* rdf = rsz + kPlocLdsNodes;
    for (int x = t; x < n - 1; x += kPlocThreads) {
      const float4 c = A.tmp[4 * x + 3];
      rcl[x] = __float_as_int(c.x), rcr[x] = __float_as_int(c.y), rsz[x] = A.nsz[x];
    }
    if (t == 0) rdf[0] = 0;
    __syncthreads();
    for (int p = pass - 1; p >= 0; --p) {
      const int first = A.pass_next[p + 1] + 1, last = A.pass_next[p];
      for (int x = first + t; x <= last; x += kPlocThreads) {
        const int d = rdf[x];
        const int32_t cl = rcl[x], cr = rcr[x];
        const int left = cl >= 0 ? rsz[cl] : 0;
        if (cl >= 0) rdf[cl] = d + 1;
        if (cr >= 0) rdf[cr] = d + 1 + left;
      }
      __syncthreads();
    }
    for (int x = t; x < n - 1; x += kPlocThreads) {
      const int d = rdf[x];
      const int32_t cl = rcl[x], cr = rcr[x];
      const float4 c = make_float4(__int_as_float(cl >= 0 ? rdf[cl] : cl), __int_as_float(cr >= 0 ? rdf[cr] : cr),
                                   0.0f, 0.0f);
      A.nodes[4 * d] = A.tmp[4 * x];
      A.nodes[4 * d + 1] = A.tmp[4 * x + 1];
      A.nodes[4 * d + 2] = A.tmp[4 * x + 2];
      A.nodes[4 * d + 3] = c;
    }
    return;
  }
  for (int p = pass - 1; p >= 0; --p) {
    const int first = A.pass_next[p + 1] + 1, last = A.pass_next[p];
    for (int x = first + t; x <= last; x += kPlocThreads) {
      const int d = A.dfs[x];
      const float4 c = A.tmp[4 * x + 3];
      const int32_t cl = __float_as_int(c.x), cr = __float_as_int(c.y);
      const int left = cl >= 0 ? A.nsz[cl] : 0;
      if (cl >= 0) A.dfs[cl] = d + 1;
      if (cr >= 0) A.dfs[cr] = d + 1 + left;
    }
    __syncthreads();
  }
  for (int x = t; x < n - 1; x += kPlocThreads) {
    const int d = A.dfs[x];
    float4 c = A.tmp[4 * x + 3];
    const int32_t cl = __float_as_int(c.x), cr = __float_as_int(c.y);
    c.x = __int_as_float(cl >= 0 ? A.dfs[cl] : cl);
    c.y = __int_as_float(cr >= 0 ? A.dfs[cr] : cr);
    A.nodes[4 * d] = A.tmp[4 * x];
    A.nodes[4 * d + 1] = A.tmp[4 * x + 1];
    A.nodes[4 * d + 2] = A.tmp[4 * x + 2];
    A.nodes[4 * d + 3] = c;
  }
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int build_bvh(const float* box_lo, const float* box_hi, int64_t n, const float scene_lo[3], const float scene_hi[3],
              BvhOut out, hipStream_t s, bool linear) {
  SBR_CHECK(n >= 1 && n < (int64_t(1) << 31), SBR_E_UNSUPPORTED, "BVH over %lld primitives", (long long)n);
  if (n == 1) {
    { ::sbr::TimedLaunch tl_("bvh", s); hipLaunchKernelGGL(k_single_leaf, dim3(1), dim3(1), 0, s, box_lo, box_hi, out.nodes, out.order, out.root_box); }
    SBR_LAUNCH_CHECK();
    if (out.depth_dev) {
      fill_u32(out.depth_dev, 1, 1, s);
      return 0;
    }
    if (out.root_host) {
      SBR_HIP(hipMemcpyAsync(out.root_host, out.root_box, 24, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
    return 1;
  }
  const bool ploc = !linear && n <= kPlocMax;
  if (!ploc && n <= kLbvhSmall) {
    float3 slo = make_float3(0.0f, 0.0f, 0.0f), ie = make_float3(0.0f, 0.0f, 0.0f);
    if (!out.bounds_dev) {
      slo = make_float3(scene_lo[0], scene_lo[1], scene_lo[2]);
      ie.x = scene_hi[0] > scene_lo[0] ? 1.0f / (scene_hi[0] - scene_lo[0]) : 0.0f;
      ie.y = scene_hi[1] > scene_lo[1] ? 1.0f / (scene_hi[1] - scene_lo[1]) : 0.0f;
      ie.z = scene_hi[2] > scene_lo[2] ? 1.0f / (scene_hi[2] - scene_lo[2]) : 0.0f;
    }
    Buf dword;
    uint32_t* dd = out.depth_dev;
    if (!dd) {
      dword.alloc(4, s);
      dd = dword.as<uint32_t>();
    }
    { ::sbr::TimedLaunch tl_("bvh", s); hipLaunchKernelGGL(k_lbvh_small, dim3(1), dim3(kSmallThreads), 0, s, box_lo, box_hi, (int)n, slo, ie,
                       out.bounds_dev, out.nodes, out.order, out.root_box, dd); }
    SBR_LAUNCH_CHECK();
    if (out.depth_dev) return 0;
    uint32_t depth = 0;
    SBR_HIP(hipMemcpyAsync(&depth, dd, 4, hipMemcpyDeviceToHost, s));
    if (out.root_host) SBR_HIP(hipMemcpyAsync(out.root_host, out.root_box, 24, hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
    return (int)depth;
  }
  Buf codes, codes2, idx, parents, flags, temp;
  codes.alloc(n * 8, s);
  codes2.alloc(n * 8, s);
  idx.alloc(n * 4, s);
  // PLOC scratch (4-byte words): boxes 12 n, id / height / size pairs 6 n,
  // nn, nsz, dfs 3 n, pass_next n + 1, then creation-order nodes 16 (n - 1)
  // at the next 16-byte boundary
  const int64_t tmp_off = (22 * n + 1 + 3) & ~int64_t(3);
  parents.alloc((ploc ? tmp_off + 16 * (n - 1) : 2 * n) * 4, s);
  flags.alloc((n + 1) * 4, s);
  temp.alloc(radix_sort_temp_bytes(n), s);
  float3 slo = make_float3(0.0f, 0.0f, 0.0f), ie = make_float3(0.0f, 0.0f, 0.0f);
  if (!out.bounds_dev) {
    slo = make_float3(scene_lo[0], scene_lo[1], scene_lo[2]);
    ie.x = scene_hi[0] > scene_lo[0] ? 1.0f / (scene_hi[0] - scene_lo[0]) : 0.0f;
    ie.y = scene_hi[1] > scene_lo[1] ? 1.0f / (scene_hi[1] - scene_lo[1]) : 0.0f;
    ie.z = scene_hi[2] > scene_lo[2] ? 1.0f / (scene_hi[2] - scene_lo[2]) : 0.0f;
  }
  { ::sbr::TimedLaunch tl_("bvh", s); hipLaunchKernelGGL(k_morton, dim3(blocks(n, 256)), dim3(256), 0, s, box_lo, box_hi, n, slo, ie,
                     out.bounds_dev, codes.as<uint64_t>(), idx.as<uint32_t>()); }
  SBR_LAUNCH_CHECK();
  radix_sort_pairs(codes.as<uint64_t>(), idx.as<uint32_t>(), codes2.as<uint64_t>(), out.order, n, 0, 30,
                   temp.p, s);
  uint32_t* dd = out.depth_dev ? out.depth_dev : flags.as<uint32_t>() + n;
  if (ploc) {
    PlocArgs A{};
    A.lo = box_lo, A.hi = box_hi, A.order = out.order, A.n = (int)n;
    float* f = parents.as<float>();
    A.box[0] = f, A.box[1] = f + 6 * n;
    int32_t* q = parents.as<int32_t>() + 12 * n;
    A.id[0] = q, A.id[1] = q + n, A.ht[0] = q + 2 * n, A.ht[1] = q + 3 * n, A.sz[0] = q + 4 * n;
    A.sz[1] = q + 5 * n, A.nn = q + 6 * n, A.nsz = q + 7 * n, A.dfs = q + 8 * n, A.pass_next = q + 9 * n;
    A.tmp = reinterpret_cast<float4*>(parents.as<int32_t>() + tmp_off);
    A.nodes = out.nodes, A.root_box = out.root_box, A.depth = dd;
    { ::sbr::TimedLaunch tl_("bvh", s); hipLaunchKernelGGL(k_ploc, dim3(1), dim3(kPlocThreads), 0, s, A); }
    SBR_LAUNCH_CHECK();
    if (out.depth_dev) return 0;
    uint32_t depth = 0;
    SBR_HIP(hipMemcpyAsync(&depth, dd, 4, hipMemcpyDeviceToHost, s));
    if (out.root_host) SBR_HIP(hipMemcpyAsync(out.root_host, out.root_box, 24, hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
    SBR_CHECK(depth != 0xffffffffu, SBR_E_DEVICE, "BVH clustering did not reach a single root");
    return (int)depth;
  }
  int32_t* pint = parents.as<int32_t>();
  int32_t* pleaf = pint + n;
  { ::sbr::TimedLaunch tl_("bvh", s); hipLaunchKernelGGL(k_karras, dim3(blocks(n - 1, 256)), dim3(256), 0, s, codes2.as<uint64_t>(), n, out.nodes, pint,
                     pleaf); }
  SBR_LAUNCH_CHECK();
  fill_u32(flags.as<uint32_t>(), 0, n + 1, s);
  { ::sbr::TimedLaunch tl_("bvh", s); hipLaunchKernelGGL(k_refit, dim3(blocks(n, 256)), dim3(256), 0, s, box_lo, box_hi, out.order, n, out.nodes, pint,
                     pleaf, flags.as<uint32_t>(), out.root_box); }
  SBR_LAUNCH_CHECK();
  fill_u32(dd, 0, 1, s);
  { ::sbr::TimedLaunch tl_("bvh", s); hipLaunchKernelGGL(k_depth, dim3(blocks(n, 256)), dim3(256), 0, s, pint, pleaf, n, dd); }
  SBR_LAUNCH_CHECK();
  if (out.depth_dev) return 0;
  uint32_t depth = 0;
  SBR_HIP(hipMemcpyAsync(&depth, dd, 4, hipMemcpyDeviceToHost, s));
  if (out.root_host) SBR_HIP(hipMemcpyAsync(out.root_host, out.root_box, 24, hipMemcpyDeviceToHost, s));
  SBR_HIP(hipStreamSynchronize(s));
  return (int)depth;
}

}  // namespace sbr
