// bvh.hip -- linear BVH built on the GPU (Karras 2012, "Maximizing
// Parallelism in the Construction of BVHs, Octrees, and k-d Trees"):
// 30-bit Morton codes of primitive centroids -> stable radix sort (ties keep
// primitive order, which makes the augmented key (code, index) unique) ->
// one thread per internal node finds its key range and split from the
// longest common prefix -> bottom-up box refit where the second thread to
// reach a node (atomic counter, acquire/release) merges its two children.
//
// Node layout (64 B, four float4): both child boxes inline so one node fetch
// serves the two slab tests of the traversal:
//   [0] Llo.x Llo.y Llo.z Lhi.x  [1] Lhi.y Lhi.z Rlo.x Rlo.y
//   [2] Rlo.z Rhi.x Rhi.y Rhi.z  [3] childL childR (int; leaf = ~sorted index)
// Leaf boxes are widened by one float ulp on each side so that they also
// contain the FP64 geometry the FP32 vertices were rounded from.
#include "sbr_device.hpp"
#include "sbr_internal.hpp"

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

__global__ void k_morton(const float* __restrict__ lo, const float* __restrict__ hi, int64_t n, float3 slo,
                         float3 inv_ext, uint64_t* __restrict__ code, uint32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float cx = 0.5f * (lo[3 * i] + hi[3 * i]);
  const float cy = 0.5f * (lo[3 * i + 1] + hi[3 * i + 1]);
  const float cz = 0.5f * (lo[3 * i + 2] + hi[3 * i + 2]);
  auto q = [](float c, float l, float ie) {
    float u = (c - l) * ie;
    u = fminf(fmaxf(u, 0.0f), 1.0f);
    return (uint32_t)fminf(u * 1024.0f, 1023.0f);
  };
  const uint32_t m = (spread10(q(cx, slo.x, inv_ext.x)) << 2) | (spread10(q(cy, slo.y, inv_ext.y)) << 1) |
                     spread10(q(cz, slo.z, inv_ext.z));
  code[i] = m;
  idx[i] = (uint32_t)i;
}

__device__ inline int delta(const uint64_t* __restrict__ code, int64_t n, int64_t i, int64_t j) {
  if (j < 0 || j >= n) return -1;
  const uint64_t a = code[i], b = code[j];
  if (a == b) return 64 + __clz((uint32_t)(i ^ j));
  return __clzll(a ^ b);
}

__global__ void k_karras(const uint64_t* __restrict__ code, int64_t n, float4* __restrict__ nodes,
                         int32_t* __restrict__ parent_int, int32_t* __restrict__ parent_leaf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
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
  int32_t cl, cr;
  if (lo == gamma) {
    cl = ~(int32_t)gamma;
    parent_leaf[gamma] = (int32_t)i;
  } else {
    cl = (int32_t)gamma;
    parent_int[gamma] = (int32_t)i;
  }
  if (hi == gamma + 1) {
    cr = ~(int32_t)(gamma + 1);
    parent_leaf[gamma + 1] = (int32_t)i;
  } else {
    cr = (int32_t)(gamma + 1);
    parent_int[gamma + 1] = (int32_t)i;
  }
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

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int build_lbvh(const float* box_lo, const float* box_hi, int64_t n, const float scene_lo[3], const float scene_hi[3],
               BvhOut out, hipStream_t s) {
  SBR_CHECK(n >= 1 && n < (int64_t(1) << 31), SBR_E_UNSUPPORTED, "LBVH over %lld primitives", (long long)n);
  if (n == 1) {
    { ::sbr::TimedLaunch tl_("lbvh", s); hipLaunchKernelGGL(k_single_leaf, dim3(1), dim3(1), 0, s, box_lo, box_hi, out.nodes, out.order, out.root_box); }
    SBR_LAUNCH_CHECK();
    if (out.root_host) {
      SBR_HIP(hipMemcpyAsync(out.root_host, out.root_box, 24, hipMemcpyDeviceToHost, s));
      SBR_HIP(hipStreamSynchronize(s));
    }
    return 1;
  }
  Buf codes, codes2, idx, parents, flags, temp;
  codes.alloc(n * 8, s);
  codes2.alloc(n * 8, s);
  idx.alloc(n * 4, s);
  parents.alloc(2 * n * 4, s);
  flags.alloc((n + 1) * 4, s);
  temp.alloc(radix_sort_temp_bytes(n), s);
  float3 slo = make_float3(scene_lo[0], scene_lo[1], scene_lo[2]);
  float3 ie;
  ie.x = scene_hi[0] > scene_lo[0] ? 1.0f / (scene_hi[0] - scene_lo[0]) : 0.0f;
  ie.y = scene_hi[1] > scene_lo[1] ? 1.0f / (scene_hi[1] - scene_lo[1]) : 0.0f;
  ie.z = scene_hi[2] > scene_lo[2] ? 1.0f / (scene_hi[2] - scene_lo[2]) : 0.0f;
  { ::sbr::TimedLaunch tl_("lbvh", s); hipLaunchKernelGGL(k_morton, dim3(blocks(n, 256)), dim3(256), 0, s, box_lo, box_hi, n, slo, ie,
                     codes.as<uint64_t>(), idx.as<uint32_t>()); }
  SBR_LAUNCH_CHECK();
  radix_sort_pairs(codes.as<uint64_t>(), idx.as<uint32_t>(), codes2.as<uint64_t>(), out.order, n, 0, 30,
                   temp.p, s);
  int32_t* pint = parents.as<int32_t>();
  int32_t* pleaf = pint + n;
  { ::sbr::TimedLaunch tl_("lbvh", s); hipLaunchKernelGGL(k_karras, dim3(blocks(n - 1, 256)), dim3(256), 0, s, codes2.as<uint64_t>(), n, out.nodes, pint,
                     pleaf); }
  SBR_LAUNCH_CHECK();
  fill_u32(flags.as<uint32_t>(), 0, n + 1, s);
  { ::sbr::TimedLaunch tl_("lbvh", s); hipLaunchKernelGGL(k_refit, dim3(blocks(n, 256)), dim3(256), 0, s, box_lo, box_hi, out.order, n, out.nodes, pint,
                     pleaf, flags.as<uint32_t>(), out.root_box); }
  SBR_LAUNCH_CHECK();
  uint32_t* dd = flags.as<uint32_t>() + n;
  fill_u32(dd, 0, 1, s);
  { ::sbr::TimedLaunch tl_("lbvh", s); hipLaunchKernelGGL(k_depth, dim3(blocks(n, 256)), dim3(256), 0, s, pint, pleaf, n, dd); }
  SBR_LAUNCH_CHECK();
  uint32_t depth = 0;
  SBR_HIP(hipMemcpyAsync(&depth, dd, 4, hipMemcpyDeviceToHost, s));
  if (out.root_host) SBR_HIP(hipMemcpyAsync(out.root_host, out.root_box, 24, hipMemcpyDeviceToHost, s));
  SBR_HIP(hipStreamSynchronize(s));
  return (int)depth;
}

}  // namespace sbr
