// trace.hip -- ray launching and the breadth-first bounce loop (Sec. II-A-1,
// II-A-2).  All rays of one bounce are traced by one persistent launch
// (the paper's "width first" multi-ray tracing), then the survivors are
// compacted into a dense structure-of-arrays for the next bounce.
//
// Precision split: the ray state that survives between bounces (origin,
// direction, unfolded length) is FP64 and is continued exactly on the plane
// of the selected triangle; only the search for the closest triangle runs
// in FP32 (watertight test, Woop/Benthin/Wald 2013), on coordinates centred
// on the scene box.  The FP32 launch point is nudged a few ulps off the
// reflecting plane (integer-ulp offset after Waechter & Binder 2019), and
// triangles coplanar with the previous hit are skipped.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <type_traits>

#include "sbr_device.hpp"
#include "sbr_internal.hpp"

namespace sbr {

// ---------------------------------------------------------------- icosahedron tables
// Built once on the host: the 12 vertices (0,+-1,+-phi), (+-1,+-phi,0),
// (+-phi,0,+-1) with sign pairs in the order (-,-), (-,+), (+,-), (+,+); the
// edges are the vertex pairs at minimum distance, the faces the triples of
// mutually adjacent vertices, both in ascending order.
const GeoTables& geo_tables() {
  static GeoTables G = [] {
    GeoTables t{};
    const double ph = (1.0 + std::sqrt(5.0)) / 2.0;
    const int sg[4][2] = {{-1, -1}, {-1, 1}, {1, -1}, {1, 1}};
    double v[12][3];
    for (int s = 0; s < 4; ++s) {
      const double a = sg[s][0], b = sg[s][1];
      v[s][0] = 0.0, v[s][1] = a, v[s][2] = b * ph;
      v[4 + s][0] = a, v[4 + s][1] = b * ph, v[4 + s][2] = 0.0;
      v[8 + s][0] = a * ph, v[8 + s][1] = 0.0, v[8 + s][2] = b;
    }
    auto dist2 = [&](int a, int b) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += (v[a][k] - v[b][k]) * (v[a][k] - v[b][k]);
      return s;
    };
    double m = 1e300;
    for (int a = 0; a < 12; ++a)
      for (int b = a + 1; b < 12; ++b) m = std::min(m, dist2(a, b));
    bool adj[12][12] = {};
    int ne = 0, nf = 0;
    for (int a = 0; a < 12; ++a)
      for (int b = a + 1; b < 12; ++b)
        if (dist2(a, b) <= m * (1 + 1e-12)) {
          adj[a][b] = adj[b][a] = true;
          t.e[ne][0] = a, t.e[ne][1] = b, ++ne;
        }
    for (int a = 0; a < 12; ++a)
      for (int b = a + 1; b < 12; ++b)
        for (int c = b + 1; c < 12; ++c)
          if (adj[a][b] && adj[b][c] && adj[a][c]) t.f[nf][0] = a, t.f[nf][1] = b, t.f[nf][2] = c, ++nf;
    const double inv = 1.0 / std::sqrt(1.0 + ph * ph);
    for (int a = 0; a < 12; ++a)
      for (int k = 0; k < 3; ++k) t.v[a][k] = v[a][k] * inv;
    if (ne != 30 || nf != 20) std::abort();
    return t;
  }();
  return G;
}

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ void k_geodesic(GeoTables G, int N, int64_t first, int64_t count, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const d3 d = geo_dir(G, N, first + i);
  out[3 * i] = d.x;
  out[3 * i + 1] = d.y;
  out[3 * i + 2] = d.z;
}

__device__ inline d3 face_point(const GeoTables& G, int f, int N, int i, int j) {
  const d3 a = ld3(G.v[G.f[f][0]]), b = ld3(G.v[G.f[f][1]]), c = ld3(G.v[G.f[f][2]]);
  return normalize(a + (b - a) * ((double)i / N) + (c - a) * ((double)j / N));
}
// great-circle angle between unit vectors from their chord
__device__ inline double chord_angle(d3 u, d3 v) {
  double h = 0.5 * norm(u - v);
  return 2.0 * asin(h > 1.0 ? 1.0 : h);
}

// grid: (ceil((N+1)/256), N+1, 20).  Each grid point (i, j) of face f owns the
// three edges (i,j)-(i+1,j), (i,j)-(i,j+1), (i+1,j)-(i,j+1); edges on the
// icosahedron's edges are shared by two faces and weighted 1/2.
__global__ __launch_bounds__(256) void k_edge_partials(GeoTables G, int N, double* __restrict__ part) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int i = blockIdx.y;
  const int f = blockIdx.z;
  double s = 0.0, lo = 1e300, hi = 0.0;
  if (i + j + 1 <= N) {
    const d3 p = face_point(G, f, N, i, j), q1 = face_point(G, f, N, i + 1, j), q2 = face_point(G, f, N, i, j + 1);
    const double a1 = chord_angle(p, q1), a2 = chord_angle(p, q2), a3 = chord_angle(q1, q2);
    s = a1 * (j == 0 ? 0.5 : 1.0) + a2 * (i == 0 ? 0.5 : 1.0) + a3 * (i + j + 1 == N ? 0.5 : 1.0);
    lo = fmin(a1, fmin(a2, a3));
    hi = fmax(a1, fmax(a2, a3));
  }
  __shared__ double ss[256], sl[256], sh[256];
  ss[threadIdx.x] = s, sl[threadIdx.x] = lo, sh[threadIdx.x] = hi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      ss[threadIdx.x] += ss[threadIdx.x + o];
      sl[threadIdx.x] = fmin(sl[threadIdx.x], sl[threadIdx.x + o]);
      sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t b = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    part[3 * b] = ss[0], part[3 * b + 1] = sl[0], part[3 * b + 2] = sh[0];
  }
}

// fixed-order final reduction (deterministic): thread t sums partials t, t+256, ...
__global__ __launch_bounds__(256) void k_edge_final(const double* __restrict__ part, int64_t nb, int N,
                                                    double* __restrict__ out) {
  double s = 0.0, lo = 1e300, hi = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += 256) {
    s += part[3 * b];
    lo = fmin(lo, part[3 * b + 1]);
    hi = fmax(hi, part[3 * b + 2]);
  }
  __shared__ double ss[256], sl[256], sh[256];
  ss[threadIdx.x] = s, sl[threadIdx.x] = lo, sh[threadIdx.x] = hi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      ss[threadIdx.x] += ss[threadIdx.x + o];
      sl[threadIdx.x] = fmin(sl[threadIdx.x], sl[threadIdx.x + o]);
      sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = ss[0] / (30.0 * (double)N * (double)N);
    out[1] = sl[0];
    out[2] = sh[0];
  }
}

// ---------------------------------------------------------------- bounce kernel
struct RaySoA {
  double *ox, *oy, *oz, *dx, *dy, *dz, *L;
  uint32_t* id;
  int32_t* prev;  // original index of the triangle the ray left, -1 at launch
};
inline RaySoA soa_of(void* base, int64_t cap) {
  double* d = static_cast<double*>(base);
  RaySoA r;
  r.ox = d, r.oy = d + cap, r.oz = d + 2 * cap, r.dx = d + 3 * cap, r.dy = d + 4 * cap, r.dz = d + 5 * cap,
  r.L = d + 6 * cap;
  r.id = reinterpret_cast<uint32_t*>(d + 7 * cap);
  r.prev = reinterpret_cast<int32_t*>(r.id + cap);
  return r;
}

__global__ void k_fill_u32_graph(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Everything the bounce kernel needs about one scene and its launch.
struct SceneDesc {
  const float4* nodes;
  const float4* tri;      // kTriVecs per leaf: 3 axis orders x (v0|orig id, v1|plane id, v2|group id)
  const double4* tplane;  // per original triangle
  const int32_t* tplaneid;
  const double* tx;
  int32_t* seq;           // [(K+1)][NR]
  float root[6];
  int has_bvh, N, K, n_big;
  int big_off, pad;       // oversized triangles: tri entries big_off .. big_off + n_big - 1
  double cx, cy, cz;      // FP32 frame centre
  int64_t R, NR, ray_off; // rays per element, rays of the scene, first position of the scene
  int32_t Nt, emin;       // elements; 1: element-minor ray positions (RayOrder)
};

struct BounceParams {
  SceneDesc one;                // single-scene launches
  const SceneDesc* table;       // batched launches: per-scene descriptors
  const int64_t* offs;          // batched: ray_off of every scene, then the total
  int n_scenes;
  GeoTables G;
  int k;
  int64_t n_first;              // rays of bounce 0 (generated, not read)
  RaySoA in, out;
  // Counter block of this bounce and of the previous one (kCtrWords words
  // each): queue, output count and drained flag of each of the 8 regions,
  // every word on its own 128-byte line.
  uint32_t* ctr;
  const uint32_t* ctr_in;
  int chunk;
  int leaf_share;  // a wave tests its queued leaves once this many 64ths of its tracing lanes hold one
  unsigned long long* work;
  unsigned long long* t_first;  // batched: per-scene first/last wall-clock stamp
  unsigned long long* t_last;
};

__device__ inline float sel(float3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

// integer-ulp offset of a point along n (Waechter & Binder 2019, small scale)
__device__ inline float off1(float p, float n) {
  constexpr float kOrigin = 1.0f / 32.0f, kFloatScale = 1.0f / 1048576.0f, kIntScale = 8.0f;
  const int of = (int)(kIntScale * n);
  const float pi = __int_as_float(__float_as_int(p) + ((p < 0.0f) ^ (of < 0) ? -of : of));
  return fabsf(p) < kOrigin ? p + kFloatScale * n : pi;
}

// p[i] read through the constant address space: for memory that no kernel
// writes while the reader runs, so that a wave-uniform index gives scalar loads
__device__ inline float4 ld_const4(const float4* p, int64_t i) {
  using cfloat = const __attribute__((address_space(4))) float;
  cfloat* q = (cfloat*)p + 4 * i;
  return make_float4(q[0], q[1], q[2], q[3]);
}

// Near and far planes of one axis for two boxes, chosen on the scalar unit
// for the whole wave: neg != 0 (a ballot of the lanes whose direction
// component is negative) takes hi as the near plane.  All operands are
// wave-uniform (scalar registers); the outputs are early-clobber so that no
// output shares a register with an input still to be read.
__device__ inline void pick_planes(uint64_t neg, float lo_l, float hi_l, float lo_r, float hi_r, float& n_l, float& f_l,
                                   float& n_r, float& f_r) {
  asm("s_cmp_lg_u64 %4, 0\n\t"
      "s_cselect_b32 %0, %6, %5\n\t"
      "s_cselect_b32 %1, %5, %6\n\t"
      "s_cselect_b32 %2, %8, %7\n\t"
      "s_cselect_b32 %3, %7, %8"
      : "=&s"(n_l), "=&s"(f_l), "=&s"(n_r), "=&s"(f_r)
      : "s"(neg), "s"(lo_l), "s"(hi_l), "s"(lo_r), "s"(hi_r)
      : "scc");
}

// scene of a global ray id: last s with offs[s] <= id
__device__ inline int scene_of(const int64_t* offs, int n, uint64_t id) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((uint64_t)offs[mid] <= id) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// PACKET: the wave traverses the tree as one (single-scene, non-counting
// launches only); otherwise every lane keeps its own traversal.  The
// wave-uniform traversal waits on one node fetch per step for the whole
// wave, and more resident waves hide that: its registers are capped for 7
// waves per SIMD (72 VGPRs, a few spilled; measured faster than 5, 6 or 8).
// The per-lane traversal gained nothing from more waves and keeps its
// registers.
template <int STACK, bool COUNT, bool MULTI, bool PACKET>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PACKET ? 7 : 1))) void k_bounce(
    const BounceParams P) {
  static_assert(!PACKET || (!COUNT && !MULTI), "packet traversal: one scene, no counting");
  __shared__ int32_t stack_mem[256 / kWave][PACKET ? 1 : STACK][kWave];
  __shared__ int32_t wave_stack[256 / kWave][PACKET ? STACK : 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t* stk = &stack_mem[wv][0][lane];
  const bool first = P.k == 0;
  const uint64_t nf = (uint64_t)P.n_first;
  const uint64_t lt = lanemask_lt();
  uint32_t n_node = 0, n_tri = 0;  // work counters (COUNT builds only)
  // Work distribution: the rays of bounce 0 are cut into 8 contiguous
  // regions, one per XCD, and every region keeps its index range for the
  // whole trace: the survivors of region x are appended to the same range of
  // the other ray buffer (never more than its input), so each region has its
  // own queue and output counters and no counter is shared by the whole chip
  // (atomics on one address serialise).  Workgroups are dispatched
  // round-robin over the 8 XCDs, so a wave drains the region of its own XCD
  // first and then steals from the others; a region found empty is flagged
  // so that later waves skip its queue without an atomic.  A wave pulls
  // `chunk` rays per atomic and traces them 64 at a time.
  const int home = blockIdx.x & 7;
  int tried = 0, reg = 0;
  uint64_t base = 0, lo = 0, hi = 0;
  uint32_t sub = 0;
  while (true) {
    if (sub == 0) {
      reg = (home + tried) & 7;
      lo = nf * (uint64_t)reg / 8;
      hi = first ? nf * (uint64_t)(reg + 1) / 8 : lo + (uint64_t)P.ctr_in[kCtrOut + 32 * reg];
      uint32_t b = 0xffffffffu;
      if (lane == 0) {
        uint32_t* q = P.ctr + kCtrQueue + 32 * reg;
        uint32_t* done = P.ctr + kCtrDone + 32 * reg;
        if (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
          b = atomicAdd(q, (uint32_t)P.chunk);
          if (lo + b >= hi) __hip_atomic_store(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      b = __shfl(b, 0, 64);
      base = lo + b;
      if (b == 0xffffffffu || base >= hi) {
        if (++tried == 8) break;
        continue;
      }
    }
    const uint64_t idx = base + sub + lane;
    sub += kWave;
    if (sub >= (uint32_t)P.chunk || base + sub >= hi) sub = 0;
    const bool active = idx < hi;
    // ------------------------------------------------ load / generate the FP64 ray
    d3 o = mk3(0, 0, 0), d = mk3(0, 0, 1);
    double L = 0.0;
    uint32_t rid = 0;  // ray position (over all scenes of a batch)
    int32_t prev = -1;
    if (active) {
      if (first) {
        rid = (uint32_t)idx;
      } else {
        o = mk3(P.in.ox[idx], P.in.oy[idx], P.in.oz[idx]);
        d = mk3(P.in.dx[idx], P.in.dy[idx], P.in.dz[idx]);
        L = P.in.L[idx];
        rid = P.in.id[idx];
        prev = P.in.prev[idx];
      }
    }
    int sid = 0;
    if (MULTI) sid = active ? scene_of(P.offs, P.n_scenes, rid) : 0;
    const SceneDesc& SD = MULTI ? P.table[sid] : P.one;
    const uint64_t lrid = (uint64_t)rid - (uint64_t)(MULTI ? SD.ray_off : 0);
    if (MULTI && P.t_first && active) {
      // first and last lanes of the wave stamp their scenes
      const bool edge = lane == 0 || lane == 63 || !(idx + 1 < hi);
      if (edge) {
        const unsigned long long t = wall_clock64();
        atomicMin(P.t_first + sid, t);
        atomicMax(P.t_last + sid, t);
      }
    }
    const bool last = P.k == SD.K;
    if (active && first) {
      int p;
      int64_t r;
      ray_of_pos(RayOrder{SD.R, SD.Nt, SD.emin}, (int64_t)lrid, p, r);
      o = ld3(SD.tx + 3 * p);
      d = geo_dir(P.G, SD.N, r);
    }
    // ------------------------------------------------ FP32 closest hit
    int32_t hit = -1;  // leaf (sorted) index
    float thit = INFINITY;
    if (active && (SD.has_bvh || SD.n_big > 0)) {
      const float4* __restrict__ nodes = SD.nodes;
      const float4* __restrict__ tri = SD.tri;
      float3 org = make_float3((float)(o.x - SD.cx), (float)(o.y - SD.cy), (float)(o.z - SD.cz));
      const float3 dir = make_float3((float)d.x, (float)d.y, (float)d.z);
      int32_t skip_plane = -1;
      if (prev >= 0) {
        skip_plane = SD.tplaneid[prev];
        const double4 pl = SD.tplane[prev];
        float sgn = (pl.x * d.x + pl.y * d.y + pl.z * d.z) >= 0.0 ? 1.0f : -1.0f;
        org.x = off1(org.x, sgn * (float)pl.x);
        org.y = off1(org.y, sgn * (float)pl.y);
        org.z = off1(org.z, sgn * (float)pl.z);
      }
      auto safe_inv = [](float v) { return 1.0f / (fabsf(v) > 1e-20f ? v : copysignf(1e-20f, v)); };
      const float3 inv = make_float3(safe_inv(dir.x), safe_inv(dir.y), safe_inv(dir.z));
      const float3 oinv = make_float3(org.x * inv.x, org.y * inv.y, org.z * inv.z);
      // watertight shear constants: kz is the dominant axis of the direction,
      // kx and ky the next two in cyclic order.  The usual swap of kx and ky
      // for a negative dir[kz] only fixes the winding; the test is double
      // sided (U, V, W, det and Tn all change sign together), so the cyclic
      // order serves, and the triangle array holds every triangle in the
      // three cyclic orders: the ray reads layout kz and needs no selects.
      const float ax = fabsf(dir.x), ay = fabsf(dir.y), az = fabsf(dir.z);
      const int kz = ax > ay ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
      const int kx = kz == 2 ? 0 : kz + 1;
      const int ky = kx == 2 ? 0 : kx + 1;
      const float dz = sel(dir, kz);
      const float Sx = sel(dir, kx) / dz, Sy = sel(dir, ky) / dz, Sz = 1.0f / dz;
      const float3 orgs = make_float3(sel(org, kx), sel(org, ky), sel(org, kz));  // origin in layout kz
      const int lay = 3 * kz;

      auto box_hit = [&](float lx, float ly, float lz, float hx, float hy, float hz, float tmax, float& tn) {
        const float t0x = fmaf(lx, inv.x, -oinv.x), t1x = fmaf(hx, inv.x, -oinv.x);
        const float t0y = fmaf(ly, inv.y, -oinv.y), t1y = fmaf(hy, inv.y, -oinv.y);
        const float t0z = fmaf(lz, inv.z, -oinv.z), t1z = fmaf(hz, inv.z, -oinv.z);
        const float tmin = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
        const float tmx = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
        tn = tmin;
        return tmin <= tmx * 1.0000004f;
      };
      // The same test with the near and far planes of every axis already
      // chosen (by the sign of the direction): rounding is monotonic, so with
      // inv > 0 the plane lo gives the smaller t and with inv < 0 the plane hi,
      // so it makes box_hit's decision and returns its entry distance (up to
      // the sign of a zero) with half its min / max.
      auto box_nf = [&](float nx, float ny, float nz, float fx, float fy, float fz, float tmax, float& tn) {
        const float tnx = fmaf(nx, inv.x, -oinv.x), tfx = fmaf(fx, inv.x, -oinv.x);
        const float tny = fmaf(ny, inv.y, -oinv.y), tfy = fmaf(fy, inv.y, -oinv.y);
        const float tnz = fmaf(nz, inv.z, -oinv.z), tfz = fmaf(fz, inv.z, -oinv.z);
        const float tmin = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, 0.0f));
        const float tmx = fminf(fminf(tfx, tfy), fminf(tfz, tmax));
        tn = tmin;
        return tmin <= tmx * 1.0000004f;
      };
      // All 48 bytes of the triangle's layout are loaded before any decision, so a
      // test costs one memory round trip; the rejections are folded into one
      // final predicate instead of early exits.  t = Tn / det is formed with
      // the hardware reciprocal (about 1 ulp): t only ranks candidates, and
      // the selected hit is re-evaluated in FP64 on its plane afterwards.
      auto tri_test = [&](int32_t leaf) {
        if (COUNT) ++n_tri;
        const float4* tv = tri + (int64_t)kTriVecs * leaf + lay;
        const float4 a = tv[0], b = tv[1], c = tv[2];
        const float Akz = a.z - orgs.z, Bkz = b.z - orgs.z, Ckz = c.z - orgs.z;
        const float Ax = (a.x - orgs.x) - Sx * Akz, Ay = (a.y - orgs.y) - Sy * Akz;
        const float Bx = (b.x - orgs.x) - Sx * Bkz, By = (b.y - orgs.y) - Sy * Bkz;
        const float Cx = (c.x - orgs.x) - Sx * Ckz, Cy = (c.y - orgs.y) - Sy * Ckz;
        float U = Cx * By - Cy * Bx, V = Ax * Cy - Ay * Cx, W = Bx * Ay - By * Ax;
        if (U == 0.0f || V == 0.0f || W == 0.0f) {
          U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
          V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
          W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
        }
        const bool outside = (U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f);
        const float det = U + V + W;
        const float Tn = U * (Sz * Akz) + V * (Sz * Bkz) + W * (Sz * Ckz);
        const float t = Tn * __builtin_amdgcn_rcpf(det);
        // an exact tie in t goes to the lower leaf, so the order in which the
        // traversal meets the candidates does not decide between them
        if (!outside && det != 0.0f && __float_as_int(b.w) != skip_plane && t > 0.0f &&
            (t < thit || (t == thit && leaf < hit))) {
          thit = t;
          hit = leaf;
        }
      };
      for (int b = 0; b < SD.n_big; ++b) tri_test(SD.big_off + b);
      float tn;
      if (PACKET) {
        // The wave walks the tree depth first as one: it enters a child when
        // any of its lanes' rays enters the child's box (each lane against its
        // own closest hit so far), tests a leaf child at once for the lanes
        // that enter it, and goes first to the child most of the lanes that
        // enter both find nearer.  Every lane still meets every box its own
        // traversal would enter, and the extra ones can only offer triangles
        // its ray really crosses, so each lane's closest hit (with its tie
        // rule) is the one of the per-lane traversal.  The wave's stack holds
        // one node per level in LDS, written by the wave's first active lane.
        const bool want =
            SD.has_bvh && box_hit(SD.root[0], SD.root[1], SD.root[2], SD.root[3], SD.root[4], SD.root[5], thit, tn);
        const uint64_t wm = __ballot(want);
        if (wm != 0) {
          int32_t* ws = &wave_stack[wv][0];
          const bool lead = lane == __builtin_ctzll(__ballot(1));
          // When the wanting lanes agree on the sign of every direction
          // component (a wave of parallel or nearly parallel rays), the near
          // and far planes of each box are chosen once for the wave, on the
          // scalar unit, and the box test needs no per-lane min / max pairs.
          const uint64_t mx = __ballot(want && inv.x < 0.0f), my = __ballot(want && inv.y < 0.0f),
                         mz = __ballot(want && inv.z < 0.0f);

          const bool same = (mx == 0 || mx == wm) && (my == 0 || my == wm) && (mz == 0 || mz == wm);
          auto walk = [&](auto same_t) {
            constexpr bool SAME = decltype(same_t)::value;
            int sp = 0;
            int32_t node = 0;
            while (true) {
              const float4 n0 = ld_const4(nodes, 4 * node), n1 = ld_const4(nodes, 4 * node + 1),
                           n2 = ld_const4(nodes, 4 * node + 2), n3 = ld_const4(nodes, 4 * node + 3);
              float tl, tr;
              bool hl, hr;
              // every lane computes both tests, and the masks are ballots of
              // the bare comparisons (so they need no conversion) cut to the
              // lanes that want the tree on the scalar unit
              if constexpr (SAME) {
                // left box lo (n0.x n0.y n0.z) hi (n0.w n1.x n1.y); right lo (n1.z n1.w n2.x) hi (n2.y n2.z n2.w)
                float nlx, flx, nrx, frx, nly, fly, nry, fry, nlz, flz, nrz, frz;
                pick_planes(mx, n0.x, n0.w, n1.z, n2.y, nlx, flx, nrx, frx);
                pick_planes(my, n0.y, n1.x, n1.w, n2.z, nly, fly, nry, fry);
                pick_planes(mz, n0.z, n1.y, n2.x, n2.w, nlz, flz, nrz, frz);
                hl = box_nf(nlx, nly, nlz, flx, fly, flz, thit, tl);
                hr = box_nf(nrx, nry, nrz, frx, fry, frz, thit, tr);
              } else {
                hl = box_hit(n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, thit, tl);
                hr = box_hit(n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, thit, tr);
              }
              const uint64_t bl = __ballot(hl) & wm, br = __ballot(hr) & wm, bn = __ballot(tl <= tr);
              const int32_t cl = __builtin_amdgcn_readfirstlane(__float_as_int(n3.x));
              const int32_t cr = __builtin_amdgcn_readfirstlane(__float_as_int(n3.y));
              // leaf children are tested at once by the lanes that enter them
              if (cl < 0 && bl != 0) {
                if (want && hl) tri_test(~cl);
              }
              if (cr < 0 && cr != cl && br != 0) {
                if (want && hr) tri_test(~cr);
              }
              // inner children entered by some lane
              const uint64_t ml = cl < 0 ? 0 : bl, mr = cr < 0 ? 0 : br;
              if (ml != 0 && mr != 0) {
                const int nb = __popcll(ml & mr), nl = __popcll(ml & mr & bn);
                const bool lfirst = 2 * nl >= nb;
                if (lead) ws[sp] = lfirst ? cr : cl;
                ++sp;
                node = lfirst ? cl : cr;
              } else if (ml != 0 || mr != 0) {
                node = ml != 0 ? cl : cr;
              } else {
                if (sp == 0) break;
                --sp;
                node = __builtin_amdgcn_readfirstlane(ws[sp]);
              }
            }
          };
          if (same) walk(std::true_type{});
          else walk(std::false_type{});
        }
      } else if (SD.has_bvh &&
                 box_hit(SD.root[0], SD.root[1], SD.root[2], SD.root[3], SD.root[4], SD.root[5], thit, tn)) {
        // Leaves are not tested where they are found: a step finds a leaf in
        // a few lanes only, and a test site entered for them would idle the
        // rest of the wave.  Each lane keeps the leaf pairs of up to two
        // steps (a0 b0, a1 b1, in the order found) and keeps descending while
        // its second pair slot is empty; the wave tests the queues together
        // once `leaf_share` / 64 of its tracing lanes hold a leaf, or when no
        // lane can take another step.  The closest hit does not change: a
        // queued leaf only lets its lane visit nodes that an earlier test
        // could have culled, and those hold no closer triangle.
        int sp = 0;
        int32_t node = 0;
        bool trav = true;
        int32_t a0 = -1, b0 = -1, a1 = -1, b1 = -1;
        const int share = P.leaf_share;
        while (true) {
          if (trav && a1 < 0) {
            if (COUNT) ++n_node;
            const float4 n0 = nodes[4 * node], n1 = nodes[4 * node + 1], n2 = nodes[4 * node + 2],
                         n3 = nodes[4 * node + 3];
            // the entry a pop would take, read while the node is in flight
            // (slot 0 when the stack is empty: in bounds, and then unused)
            const int32_t top = stk[kWave * (sp > 0 ? sp - 1 : 0)];
            float tl, tr;
            bool hl = box_hit(n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, thit, tl);
            bool hr = box_hit(n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, thit, tr);
            const int32_t cl = __float_as_int(n3.x), cr = __float_as_int(n3.y);
            int32_t la = -1, lb = -1;
            if (hl && cl < 0) {
              la = ~cl;
              hl = false;
            }
            if (hr && cr < 0) {
              if (cr != cl) {
                if (la < 0) la = ~cr;
                else lb = ~cr;
              }
              hr = false;
            }
            // both hit: descend into the nearer, push the other; one hit:
            // descend; none: pop (the decision is written as selects so that
            // the stack read above is not deferred into a pop branch)
            const bool both = hl && hr, none = !hl && !hr;
            const bool lnear = tl <= tr;
            if (both) stk[kWave * sp] = lnear ? cr : cl;
            if (none && sp == 0) trav = false;
            node = both ? (lnear ? cl : cr) : hl ? cl : hr ? cr : top;
            sp += both ? 1 : (none && sp > 0) ? -1 : 0;
            // the step's pair goes to the first empty pair slot; a slot is
            // empty when its first entry is -1, so storing a step that found
            // no leaf (la = -1) leaves the slot empty and needs no branch
            const bool e0 = a0 < 0;
            a1 = e0 ? a1 : la;
            b1 = e0 ? b1 : lb;
            a0 = e0 ? la : a0;
            b0 = e0 ? lb : b0;
          }
          const uint64_t held = __ballot(a0 >= 0);
          const uint64_t going = __ballot(trav && a1 < 0);
          if (going == 0 || __popcll(held) * 64 >= share * __popcll(__ballot(1))) {
#pragma unroll 1
            while (a0 >= 0) {
              tri_test(a0);
              // next in discovery order: b0 if the first pair held two
              // leaves, else a1 (a pair's b is set only with its a)
              const bool two = b0 >= 0;
              a0 = two ? b0 : a1;
              b0 = two ? a1 : b1;
              a1 = two ? b1 : -1;
              b1 = -1;
            }
          }
          if (!trav && a0 < 0) break;
        }
      }
      if (hit >= 0) hit = __float_as_int(tri[(int64_t)kTriVecs * hit].w);  // original triangle id
    }
    // ------------------------------------------------ record, reflect in FP64, compact
    const int32_t orig = hit;
    if (active) SD.seq[(int64_t)P.k * SD.NR + (int64_t)lrid] = orig;
    const bool live = active && orig >= 0 && !last;
    if (live) {
      const double4 pl = SD.tplane[orig];
      const double t = advance_t(pl, o, d);
      o = o + d * t;
      L += t;
      d = reflect(d, pl);
    }
    const uint64_t m = __ballot(live);
    if (m != 0) {
      uint32_t ob = 0;
      if (lane == 0) ob = atomicAdd(P.ctr + kCtrOut + 32 * reg, (uint32_t)__popcll(m));
      ob = __shfl(ob, 0, 64);
      if (live) {
        const uint64_t j = lo + ob + (uint32_t)__popcll(m & lt);
        P.out.ox[j] = o.x, P.out.oy[j] = o.y, P.out.oz[j] = o.z;
        P.out.dx[j] = d.x, P.out.dy[j] = d.y, P.out.dz[j] = d.z;
        P.out.L[j] = L;
        P.out.id[j] = rid;
        P.out.prev[j] = orig;
      }
    }
  }
  if (COUNT) {
    unsigned long long a = n_node, b = n_tri;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_xor(a, o, 64);
      b += __shfl_xor(b, o, 64);
    }
    if (lane == 0) {
      atomicAdd(P.work, a);
      atomicAdd(P.work + 1, b);
    }
  }
}

SceneDesc scene_desc(const sbr_scene_s* sc, const double* tx, int Nt, int emin, int N, int K, int64_t R, int64_t NR,
                     int32_t* seq, int64_t ray_off) {
  SceneDesc D{};
  D.has_bvh = sc->n_bvh > 0;
  D.n_big = sc->n_big;
  D.big_off = (int)sc->n_bvh;
  D.nodes = sc->nodes.as<float4>();
  D.tri = sc->tri32.as<float4>();
  D.tplane = sc->tplane.as<double4>();
  D.tplaneid = sc->tplaneid.as<int32_t>();
  for (int k = 0; k < 6; ++k) D.root[k] = sc->root_host[k];
  D.cx = sc->center[0], D.cy = sc->center[1], D.cz = sc->center[2];
  D.tx = tx;
  D.N = N, D.K = K, D.R = R, D.NR = NR, D.seq = seq, D.ray_off = ray_off;
  D.Nt = Nt, D.emin = emin;
  return D;
}

template <bool COUNT, bool MULTI, bool PACKET = false>
void launch_bounce(int depth, dim3 g, const BounceParams& P, hipStream_t s) {
  if (depth <= 16) hipLaunchKernelGGL((k_bounce<16, COUNT, MULTI, PACKET>), g, dim3(256), 0, s, P);
  else if (depth <= 32) hipLaunchKernelGGL((k_bounce<32, COUNT, MULTI, PACKET>), g, dim3(256), 0, s, P);
  else hipLaunchKernelGGL((k_bounce<64, COUNT, MULTI, PACKET>), g, dim3(256), 0, s, P);
}

}  // namespace

void upload_geodesic_tables(int) {}

void launch_geodesic(int N, int64_t first, int64_t count, double* dirs, hipStream_t s) {
  if (count <= 0) return;
  { ::sbr::TimedLaunch tl_("geodesic", s); hipLaunchKernelGGL(k_geodesic, dim3(nblk(count, 256)), dim3(256), 0, s, geo_tables(), N, first, count, dirs); }
  SBR_LAUNCH_CHECK();
}

void geodesic_edge_stats(int N, double* mean, double* mn, double* mx, hipStream_t s) {
  const dim3 grid(nblk(N + 1, 256), N + 1, 20);
  const int64_t nb = (int64_t)grid.x * grid.y * grid.z;
  Buf part, out;
  part.alloc(nb * 3 * sizeof(double), s);
  out.alloc(3 * sizeof(double), s);
  { ::sbr::TimedLaunch tl_("alpha", s); hipLaunchKernelGGL(k_edge_partials, grid, dim3(256), 0, s, geo_tables(), N, part.as<double>()); }
  { ::sbr::TimedLaunch tl_("alpha", s); hipLaunchKernelGGL(k_edge_final, dim3(1), dim3(256), 0, s, part.as<double>(), nb, N, out.as<double>()); }
  SBR_LAUNCH_CHECK();
  double h[3];
  SBR_HIP(hipMemcpyAsync(h, out.p, sizeof h, hipMemcpyDeviceToHost, s));
  SBR_HIP(hipStreamSynchronize(s));
  if (mean) *mean = h[0];
  if (mn) *mn = h[1];
  if (mx) *mx = h[2];
}

int64_t trace_counter_words(int K) { return (int64_t)kCtrWords * (K + 1); }

size_t trace_ray_bytes(int64_t NR) { return (size_t)NR * (7 * sizeof(double) + 2 * sizeof(uint32_t)); }

TraceGraph::~TraceGraph() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
}

namespace {
template <bool COUNT, bool PACKET>
const void* bounce_fn(int depth) {
  if (depth <= 16) return reinterpret_cast<const void*>(&k_bounce<16, COUNT, false, PACKET>);
  if (depth <= 32) return reinterpret_cast<const void*>(&k_bounce<32, COUNT, false, PACKET>);
  return reinterpret_cast<const void*>(&k_bounce<64, COUNT, false, PACKET>);
}
hipKernelNodeParams knode(const void* fn, dim3 g, dim3 b, void** args) {
  hipKernelNodeParams p{};
  p.func = const_cast<void*>(fn);
  p.gridDim = g;
  p.blockDim = b;
  p.sharedMemBytes = 0;
  p.kernelParams = args;
  p.extra = nullptr;
  return p;
}
}  // namespace

// The bounce loop as a graph: fill(counters) -> bounce 0 -> ... -> bounce K,
// all kernel nodes (no memset nodes).  Built on first use for a
// (K, depth class, counting, traversal) shape, then only the kernel arguments
// are updated.
void launch_trace_graph(const TraceLaunch& T, const BounceParams* P, int nP, hipStream_t s) {
  sbr_context_s* c = T.ctx;
  const int depth = T.scene->bvh_depth;
  const int bucket = depth <= 16 ? 16 : depth <= 32 ? 32 : 64;
  const int count = T.work ? 1 : 0;
  const int packet = !count && T.packet ? 1 : 0;
  TraceGraph* G = nullptr;
  for (auto* g : c->graphs)
    if (g->K == T.K && g->depth_bucket == bucket && g->count == count && g->packet == packet) G = g;
  uint32_t* cnt = T.counters;
  int64_t ncnt = trace_counter_words(T.K);
  uint32_t v0 = 0;
  void* a_cnt[] = {&cnt, &v0, &ncnt};
  std::vector<BounceParams> Pc(P, P + nP);
  std::vector<void*> a_b(nP);
  for (int k = 0; k < nP; ++k) a_b[k] = &Pc[k];
  const void* ffill = reinterpret_cast<const void*>(&k_fill_u32_graph);
  const dim3 gc((unsigned)((ncnt + 255) / 256)), gb(T.grid), b256(256);
  const void* fb = count ? bounce_fn<true, false>(depth) : packet ? bounce_fn<false, true>(depth)
                                                                   : bounce_fn<false, false>(depth);
  if (!G) {
    G = new TraceGraph();
    G->K = T.K, G->depth_bucket = bucket, G->count = count, G->packet = packet;
    SBR_HIP(hipGraphCreate(&G->graph, 0));
    hipGraphNode_t prev = nullptr;
    auto add = [&](const void* fn, dim3 g, void** args) {
      hipKernelNodeParams kp = knode(fn, g, b256, args);
      hipGraphNode_t n;
      SBR_HIP(hipGraphAddKernelNode(&n, G->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
      G->nodes.push_back(n);
      prev = n;
    };
    add(ffill, gc, a_cnt);
    for (int k = 0; k < nP; ++k) add(fb, gb, &a_b[k]);
    SBR_HIP(hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0));
    c->graphs.push_back(G);
  } else {
    hipKernelNodeParams kp = knode(ffill, gc, b256, a_cnt);
    SBR_HIP(hipGraphExecKernelNodeSetParams(G->exec, G->nodes[0], &kp));
    for (int k = 0; k < nP; ++k) {
      kp = knode(fb, gb, b256, &a_b[k]);
      SBR_HIP(hipGraphExecKernelNodeSetParams(G->exec, G->nodes[1 + k], &kp));
    }
  }
  ::sbr::TimedLaunch tl_("bounce", s);
  SBR_HIP(hipGraphLaunch(G->exec, s));
}

void launch_trace(const TraceLaunch& T, void* ray_a, void* ray_b, hipStream_t s) {
  BounceParams P{};
  P.one = scene_desc(T.scene, T.tx, T.Nt, T.emin, T.N, T.K, T.R, T.NR, T.seq, 0);
  P.n_scenes = 1;
  P.G = geo_tables();
  P.n_first = T.NR;
  P.work = T.work;
  P.chunk = T.chunk;
  P.leaf_share = T.leaf_share;
  const int depth = T.scene->bvh_depth;
  RaySoA A = soa_of(ray_a, T.NR), B = soa_of(ray_b, T.NR);
  std::vector<BounceParams> Pk(T.K + 1, P);
  for (int k = 0; k <= T.K; ++k) {
    Pk[k].k = k;
    Pk[k].ctr = T.counters + (int64_t)kCtrWords * k;
    Pk[k].ctr_in = k > 0 ? T.counters + (int64_t)kCtrWords * (k - 1) : nullptr;
    Pk[k].in = (k % 2 == 1) ? A : B;
    Pk[k].out = (k % 2 == 1) ? B : A;
  }
  if (T.ctx && T.ctx->tune.trace_graph) {
    launch_trace_graph(T, Pk.data(), T.K + 1, s);
    return;
  }
  // The hit chain is not initialised: bounce k writes seq[k] (hit or -1) for
  // every ray it traces, and every ray live after bounce k - 1 is traced at k,
  // so each chain is written up to its first -1 (or to K), and no reader looks
  // past that entry.
  fill_u32(T.counters, 0, trace_counter_words(T.K), s);
  for (int k = 0; k <= T.K; ++k) {
    ::sbr::TimedLaunch tl_("bounce", s);
    if (T.work) launch_bounce<true, false>(depth, dim3(T.grid), Pk[k], s);
    else if (T.packet) launch_bounce<false, false, true>(depth, dim3(T.grid), Pk[k], s);
    else launch_bounce<false, false>(depth, dim3(T.grid), Pk[k], s);
    SBR_LAUNCH_CHECK();
  }
}

void launch_trace_batch(const std::vector<sbr_trace_s*>& trs, int grid, int chunk, int leaf_share, void* ray_a,
                        void* ray_b, uint32_t* counters, unsigned long long* t_first, unsigned long long* t_last,
                        hipStream_t s) {
  const int n = (int)trs.size();
  std::vector<SceneDesc> tab(n);
  std::vector<int64_t> offs(n + 1);
  int64_t off = 0;
  int depth = 1, Kmax = 0;
  for (int i = 0; i < n; ++i) {
    sbr_trace_s* t = trs[i];
    tab[i] = scene_desc(t->scene, t->tx.as<double>(), t->Nt, t->emin, t->N, t->K, t->R, t->NR, t->seq.as<int32_t>(),
                        off);
    offs[i] = off;
    off += t->NR;
    depth = std::max(depth, t->scene->bvh_depth);
    Kmax = std::max(Kmax, t->K);
  }
  offs[n] = off;
  Buf dtab, doffs;
  dtab.alloc(sizeof(SceneDesc) * n, s);
  doffs.alloc(sizeof(int64_t) * (n + 1), s);
  SBR_HIP(hipMemcpyAsync(dtab.p, tab.data(), sizeof(SceneDesc) * n, hipMemcpyHostToDevice, s));
  SBR_HIP(hipMemcpyAsync(doffs.p, offs.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
  fill_u32(counters, 0, trace_counter_words(Kmax), s);
  fill_u32(reinterpret_cast<uint32_t*>(t_first), 0xffffffffu, 2 * (int64_t)n, s);
  fill_u32(reinterpret_cast<uint32_t*>(t_last), 0u, 2 * (int64_t)n, s);
  BounceParams P{};
  P.table = dtab.as<SceneDesc>();
  P.offs = doffs.as<int64_t>();
  P.n_scenes = n;
  P.G = geo_tables();
  P.n_first = off;
  P.chunk = chunk;
  P.leaf_share = leaf_share;
  P.t_first = t_first;
  P.t_last = t_last;
  RaySoA A = soa_of(ray_a, off), B = soa_of(ray_b, off);
  for (int k = 0; k <= Kmax; ++k) {
    P.k = k;
    P.ctr = counters + (int64_t)kCtrWords * k;
    P.ctr_in = k > 0 ? counters + (int64_t)kCtrWords * (k - 1) : nullptr;
    P.in = (k % 2 == 1) ? A : B;
    P.out = (k % 2 == 1) ? B : A;
    ::sbr::TimedLaunch tl_("bounce", s);
    launch_bounce<false, true>(depth, dim3(grid), P, s);
    SBR_LAUNCH_CHECK();
  }
  // host copies of the table must outlive the copies: synchronise before they go
  SBR_HIP(hipStreamSynchronize(s));
}

}  // namespace sbr
