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

struct BounceParams {
  const float4* nodes;
  const float4* tri;      // 3 per leaf: v0|orig id, v1|plane id, v2|group id
  const double4* tplane;  // per original triangle
  const int32_t* tplaneid;
  float root[6];
  double cx, cy, cz;      // FP32 frame centre
  GeoTables G;
  int N;
  int64_t R;
  const double* tx;
  int k, K;
  int64_t n_first;        // rays of bounce 0 (generated, not read)
  const uint32_t* n_in_ptr;
  RaySoA in, out;
  uint32_t* n_out_ptr;
  uint32_t* queue;
  int32_t* seq_k;
  int has_bvh;
  int chunk;
  unsigned long long* work;
};

__device__ inline float sel(float3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

// integer-ulp offset of a point along n (Waechter & Binder 2019, small scale)
__device__ inline float off1(float p, float n) {
  constexpr float kOrigin = 1.0f / 32.0f, kFloatScale = 1.0f / 1048576.0f, kIntScale = 8.0f;
  const int of = (int)(kIntScale * n);
  const float pi = __int_as_float(__float_as_int(p) + ((p < 0.0f) ^ (of < 0) ? -of : of));
  return fabsf(p) < kOrigin ? p + kFloatScale * n : pi;
}

template <int STACK, bool COUNT>
__global__ __launch_bounds__(256) void k_bounce(const BounceParams P) {
  __shared__ int32_t stack_mem[256 / kWave][STACK][kWave];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t* stk = &stack_mem[wv][0][lane];
  const bool first = P.k == 0, last = P.k == P.K;
  const uint64_t n_in = first ? (uint64_t)P.n_first : (uint64_t)*P.n_in_ptr;
  const uint64_t lt = lanemask_lt();
  uint32_t n_node = 0, n_tri = 0;  // work counters (COUNT builds only)
  // Work distribution: the rays of the bounce are cut into 8 contiguous
  // slices, one per XCD, each with its own queue counter on its own cache
  // line.  Workgroups are dispatched round-robin over the 8 XCDs, so a wave
  // drains the slice of its own XCD first (atomics stay in that XCD's L2) and
  // then steals from the others.  A wave pulls `chunk` rays per atomic and
  // traces them 64 at a time.
  const int home = blockIdx.x & 7;
  int tried = 0;
  uint64_t base = 0, lo = 0, hi = 0;
  uint32_t sub = 0;
  while (true) {
    if (sub == 0) {
      const int x = (home + tried) & 7;
      lo = n_in * (uint64_t)x / 8;
      hi = n_in * (uint64_t)(x + 1) / 8;
      uint32_t b = 0;
      if (lane == 0) b = atomicAdd(P.queue + 32 * x, (uint32_t)P.chunk);
      base = lo + __shfl(b, 0, 64);
      if (base >= hi) {
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
    uint32_t rid = 0;
    int32_t prev = -1;
    if (active) {
      if (first) {
        rid = (uint32_t)idx;
        const int p = (int)(idx / (uint64_t)P.R);
        o = ld3(P.tx + 3 * p);
        d = geo_dir(P.G, P.N, (int64_t)(idx - (uint64_t)p * P.R));
      } else {
        o = mk3(P.in.ox[idx], P.in.oy[idx], P.in.oz[idx]);
        d = mk3(P.in.dx[idx], P.in.dy[idx], P.in.dz[idx]);
        L = P.in.L[idx];
        rid = P.in.id[idx];
        prev = P.in.prev[idx];
      }
    }
    // ------------------------------------------------ FP32 closest hit
    int32_t hit = -1;  // leaf (sorted) index
    float thit = INFINITY;
    if (active && P.has_bvh) {
      float3 org = make_float3((float)(o.x - P.cx), (float)(o.y - P.cy), (float)(o.z - P.cz));
      const float3 dir = make_float3((float)d.x, (float)d.y, (float)d.z);
      int32_t skip_plane = -1;
      if (prev >= 0) {
        skip_plane = P.tplaneid[prev];
        const double4 pl = P.tplane[prev];
        float sgn = (pl.x * d.x + pl.y * d.y + pl.z * d.z) >= 0.0 ? 1.0f : -1.0f;
        org.x = off1(org.x, sgn * (float)pl.x);
        org.y = off1(org.y, sgn * (float)pl.y);
        org.z = off1(org.z, sgn * (float)pl.z);
      }
      auto safe_inv = [](float v) { return 1.0f / (fabsf(v) > 1e-20f ? v : copysignf(1e-20f, v)); };
      const float3 inv = make_float3(safe_inv(dir.x), safe_inv(dir.y), safe_inv(dir.z));
      const float3 oinv = make_float3(org.x * inv.x, org.y * inv.y, org.z * inv.z);
      // watertight shear constants
      const float ax = fabsf(dir.x), ay = fabsf(dir.y), az = fabsf(dir.z);
      int kz = ax > ay ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
      int kx = kz == 2 ? 0 : kz + 1;
      int ky = kx == 2 ? 0 : kx + 1;
      if (sel(dir, kz) < 0.0f) {
        const int t = kx;
        kx = ky;
        ky = t;
      }
      const float dz = sel(dir, kz);
      const float Sx = sel(dir, kx) / dz, Sy = sel(dir, ky) / dz, Sz = 1.0f / dz;

      auto box_hit = [&](float lx, float ly, float lz, float hx, float hy, float hz, float tmax, float& tn) {
        const float t0x = fmaf(lx, inv.x, -oinv.x), t1x = fmaf(hx, inv.x, -oinv.x);
        const float t0y = fmaf(ly, inv.y, -oinv.y), t1y = fmaf(hy, inv.y, -oinv.y);
        const float t0z = fmaf(lz, inv.z, -oinv.z), t1z = fmaf(hz, inv.z, -oinv.z);
        const float tmin = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
        const float tmx = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
        tn = tmin;
        return tmin <= tmx * 1.0000004f;
      };
      auto tri_test = [&](int32_t leaf) {
        if (COUNT) ++n_tri;
        const float4 a = P.tri[3 * leaf], b = P.tri[3 * leaf + 1], c = P.tri[3 * leaf + 2];
        if (__float_as_int(b.w) == skip_plane) return;
        const float3 A = make_float3(a.x - org.x, a.y - org.y, a.z - org.z);
        const float3 B = make_float3(b.x - org.x, b.y - org.y, b.z - org.z);
        const float3 C = make_float3(c.x - org.x, c.y - org.y, c.z - org.z);
        const float Akz = sel(A, kz), Bkz = sel(B, kz), Ckz = sel(C, kz);
        const float Ax = sel(A, kx) - Sx * Akz, Ay = sel(A, ky) - Sy * Akz;
        const float Bx = sel(B, kx) - Sx * Bkz, By = sel(B, ky) - Sy * Bkz;
        const float Cx = sel(C, kx) - Sx * Ckz, Cy = sel(C, ky) - Sy * Ckz;
        float U = Cx * By - Cy * Bx, V = Ax * Cy - Ay * Cx, W = Bx * Ay - By * Ax;
        if (U == 0.0f || V == 0.0f || W == 0.0f) {
          U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
          V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
          W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
        }
        if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return;
        const float det = U + V + W;
        if (det == 0.0f) return;
        const float Tn = U * (Sz * Akz) + V * (Sz * Bkz) + W * (Sz * Ckz);
        const float t = Tn / det;
        if (t > 0.0f && t < thit) {
          thit = t;
          hit = leaf;
        }
      };
      float tn;
      if (box_hit(P.root[0], P.root[1], P.root[2], P.root[3], P.root[4], P.root[5], INFINITY, tn)) {
        int sp = 0;
        int32_t node = 0;
        while (true) {
          if (COUNT) ++n_node;
          const float4 n0 = P.nodes[4 * node], n1 = P.nodes[4 * node + 1], n2 = P.nodes[4 * node + 2],
                       n3 = P.nodes[4 * node + 3];
          float tl, tr;
          bool hl = box_hit(n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, thit, tl);
          bool hr = box_hit(n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, thit, tr);
          const int32_t cl = __float_as_int(n3.x), cr = __float_as_int(n3.y);
          if (hl && cl < 0) {
            tri_test(~cl);
            hl = false;
          }
          if (hr && cr < 0) {
            tri_test(~cr);
            hr = false;
          }
          if (hl && hr) {
            const bool lnear = tl <= tr;
            stk[kWave * sp] = lnear ? cr : cl;
            ++sp;
            node = lnear ? cl : cr;
          } else if (hl) {
            node = cl;
          } else if (hr) {
            node = cr;
          } else {
            if (sp == 0) break;
            --sp;
            node = stk[kWave * sp];
          }
        }
      }
    }
    // ------------------------------------------------ record, reflect in FP64, compact
    int32_t orig = -1;
    if (hit >= 0) orig = __float_as_int(P.tri[3 * hit].w);
    if (active) P.seq_k[rid] = orig;
    const bool live = active && orig >= 0 && !last;
    if (live) {
      const double4 pl = P.tplane[orig];
      const double t = advance_t(pl, o, d);
      o = o + d * t;
      L += t;
      d = reflect(d, pl);
    }
    const uint64_t m = __ballot(live);
    if (m != 0) {
      uint32_t ob = 0;
      if (lane == 0) ob = atomicAdd(P.n_out_ptr, (uint32_t)__popcll(m));
      ob = __shfl(ob, 0, 64);
      if (live) {
        const uint32_t j = ob + (uint32_t)__popcll(m & lt);
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

int64_t trace_counter_words(int K) { return 32 + 256 * (int64_t)(K + 1); }

size_t trace_ray_bytes(int64_t NR) { return (size_t)NR * (7 * sizeof(double) + 2 * sizeof(uint32_t)); }

void launch_trace(const TraceLaunch& T, void* ray_a, void* ray_b, hipStream_t s) {
  const sbr_scene_s* sc = T.scene;
  BounceParams P{};
  P.has_bvh = sc->T > 0;
  P.nodes = sc->nodes.as<float4>();
  P.tri = sc->tri32.as<float4>();
  P.tplane = sc->tplane.as<double4>();
  P.tplaneid = sc->tplaneid.as<int32_t>();
  for (int k = 0; k < 6; ++k) P.root[k] = sc->root_host[k];
  P.cx = sc->center[0], P.cy = sc->center[1], P.cz = sc->center[2];
  P.G = geo_tables();
  P.N = T.N;
  P.R = T.R;
  P.tx = T.tx;
  P.K = T.K;
  P.n_first = T.NR;
  P.work = T.work;
  P.chunk = T.chunk;
  const int depth = sc->bvh_depth;
  // counters: [0..K] survivors of each bounce; then per bounce 8 queue slots of 128 B
  fill_u32(T.counters, 0, trace_counter_words(T.K), s);
  // every chain entry starts as "miss"; the bounce kernels overwrite the ones they trace
  fill_u32(reinterpret_cast<uint32_t*>(T.seq), 0xffffffffu, (int64_t)(T.K + 1) * T.NR, s);
  RaySoA A = soa_of(ray_a, T.NR), B = soa_of(ray_b, T.NR);
  for (int k = 0; k <= T.K; ++k) {
    P.k = k;
    P.queue = T.counters + 32 + 256 * k;
    P.n_in_ptr = k > 0 ? T.counters + (k - 1) : nullptr;
    P.n_out_ptr = T.counters + k;
    P.in = (k % 2 == 1) ? A : B;
    P.out = (k % 2 == 1) ? B : A;
    P.seq_k = T.seq + (int64_t)k * T.NR;
    const dim3 g(T.grid), b(256);
    ::sbr::TimedLaunch tl_("bounce", s);
    if (T.work) {
      if (depth <= 16) hipLaunchKernelGGL((k_bounce<16, true>), g, b, 0, s, P);
      else if (depth <= 32) hipLaunchKernelGGL((k_bounce<32, true>), g, b, 0, s, P);
      else hipLaunchKernelGGL((k_bounce<64, true>), g, b, 0, s, P);
    } else {
      if (depth <= 16) hipLaunchKernelGGL((k_bounce<16, false>), g, b, 0, s, P);
      else if (depth <= 32) hipLaunchKernelGGL((k_bounce<32, false>), g, b, 0, s, P);
      else hipLaunchKernelGGL((k_bounce<64, false>), g, b, 0, s, P);
    }
    SBR_LAUNCH_CHECK();
  }
}

}  // namespace sbr
