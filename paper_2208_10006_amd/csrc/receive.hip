// receive.hip -- ray reception and effective-path extraction (Sec. II-A-3,
// and the "pick out effective paths" of Sec. II-A-2).
//
//  1. replay:   every ray's FP64 chain is rebuilt from its hit chain (the
//               per-ray record the trace kept) and each segment is tested
//               against the receivers through a BVH over the Rx points:
//               captured when the closest approach lies inside the segment
//               and within coeff * alpha * (unfolded distance) / sqrt(3).
//  2. keys:     capture -> (rx*Nt + tx, 64-bit hash of (k, g_1..g_k));
//               radix sort; duplicates (several rays, or both triangles of a
//               wall, finding one geometric path) collapse to one key by an
//               exact sequence comparison inside equal-hash runs.
//  3. rebuild:  each key is rebuilt by the image method in FP64 (Sec. I) and
//               kept when its reflection points lie on their faces, on the
//               incidence side, and no triangle blocks a leg (any-hit BVH
//               traversal with FP64 triangle tests); the frequency-
//               independent part of the field (polarisation chain, incidence
//               cosines, materials) is stored for the channel kernels.
//  4. order:    valid paths sorted by (rx, tx, delay); CSR per (rx, tx).
#include <algorithm>
#include <optional>
#include <cmath>

#include "sbr_device.hpp"
#include "sbr_internal.hpp"
#include "launch_rules.hpp"
#include "occlusion.hpp"

namespace sbr {
namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }


struct ReplayParams {
  GeoTables G;
  int N, K, Nr;
  int64_t T;
  int64_t R, NR;
  RayOrder ord;
  const double* tx;
  const int32_t* seq;
  const double4* tplane;
  const float4* rnodes;
  const uint32_t* rorder;
  float rroot[6];
  const double* rx;
  double rc[3], rrad;  // Rx bounding sphere (FP64); FP32 Rx frame centred on rc
  // device-prepared receiver sets: rc xyz and rrad (4 doubles) and the root
  // box (6 floats) in device memory, used instead of the fields above
  const double* rdev;
  const float* rroot_dev;
  double rfac;         // coeff * alpha / sqrt(3)
  uint32_t* ev_count;
  uint64_t ev_cap;
  uint32_t* ev_ray;
  uint32_t* ev_qk;     // q << 5 | k
};

// SE: stack entry type (int16_t for trees of up to kLbvhSmall primitives,
// whose node and leaf references fit 16 bits).  DEV: the receiver frame and
// root box come from device memory (P.rdev, P.rroot_dev) instead of the
// parameters; they are uniform and are moved to scalar registers.
__device__ inline double uniform_f64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <int STACK, typename SE, bool DEV>
__global__ __launch_bounds__(1024) void k_replay_capture(const ReplayParams P) {
  // The wave's stack: entry e of a lane at slot(e).  For 4-byte entries slot
  // e is word e * 64 + lane; 2-byte entries are paired per lane (entries 2i
  // and 2i + 1 in the two halves of word i * 64 + lane), so that no two lanes
  // share an LDS word.
  extern __shared__ unsigned char stack_raw[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  SE* const stk_base = reinterpret_cast<SE*>(stack_raw) + (size_t)wv * STACK * kWave;
  auto slot = [&](int e) -> SE& {
    if (sizeof(SE) == 2) return stk_base[((e >> 1) * kWave + lane) * 2 + (e & 1)];
    return stk_base[e * kWave + lane];
  };
  const int64_t rid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // ray position
  if (rid >= P.NR) return;
  int p;
  int64_t r;
  ray_of_pos(P.ord, rid, p, r);
  d3 o = ld3(P.tx + 3 * p);
  d3 d = geo_dir(P.G, P.N, r);
  double L = 0.0;
  d3 rc = mk3(P.rc[0], P.rc[1], P.rc[2]);
  double rrad = P.rrad;
  float rroot[6];
  for (int k = 0; k < 6; ++k) rroot[k] = P.rroot[k];
  if (DEV) {
    rc = mk3(uniform_f64(P.rdev[0]), uniform_f64(P.rdev[1]), uniform_f64(P.rdev[2]));
    rrad = uniform_f64(P.rdev[3]);
    for (int k = 0; k < 6; ++k)
      rroot[k] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(P.rroot_dev[k])));
  }
  for (int k = 0; k <= P.K; ++k) {
    int32_t tri = P.seq[(int64_t)k * P.NR + rid];
    if (tri >= P.T) tri = -1;  // defensive: chain entries are triangle ids or -1
    double4 pl = make_double4(0, 0, 0, 0);
    double tend = INFINITY;
    if (tri >= 0) {
      pl = P.tplane[tri];
      tend = advance_t(pl, o, d);
    }
    // ---------------- capture test of segment (o, d, [0, tend], L)
    // any capture has t* = (q - o).d <= |q - o| <= |o - rc| + rrad
    const double thi = fmin(tend, norm(o - rc) + rrad);
    if (thi >= 0.0) {
      const double rmax = P.rfac * (L + thi);
      const float3 org = make_float3((float)(o.x - rc.x), (float)(o.y - rc.y), (float)(o.z - rc.z));
      const float3 dir = make_float3((float)d.x, (float)d.y, (float)d.z);
      const float infl = (float)(rmax + 1e-5 * (fabs(o.x - rc.x) + fabs(o.y - rc.y) + fabs(o.z - rc.z) + thi) + 1e-6);
      const float tmax = (float)thi * 1.00001f + 1e-6f;
      // hardware reciprocal (about 1 ulp): the boxes are inflated by far more
      // (1e-5 of the distances) than its error moves a slab distance
      auto safe_inv = [](float v) {
        return __builtin_amdgcn_rcpf(fabsf(v) > 1e-20f ? v : copysignf(1e-20f, v));
      };
      const float3 inv = make_float3(safe_inv(dir.x), safe_inv(dir.y), safe_inv(dir.z));
      // slab distances of the inflated box, (lo - infl - org) * inv and
      // (hi + infl - org) * inv, as one FMA each with per-segment constants
      const float3 clo = make_float3(-(org.x + infl) * inv.x, -(org.y + infl) * inv.y, -(org.z + infl) * inv.z);
      const float3 chi = make_float3(-(org.x - infl) * inv.x, -(org.y - infl) * inv.y, -(org.z - infl) * inv.z);
      auto box_hit = [&](float lx, float ly, float lz, float hx, float hy, float hz) {
        const float t0x = fmaf(lx, inv.x, clo.x), t1x = fmaf(hx, inv.x, chi.x);
        const float t0y = fmaf(ly, inv.y, clo.y), t1y = fmaf(hy, inv.y, chi.y);
        const float t0z = fmaf(lz, inv.z, clo.z), t1z = fmaf(hz, inv.z, chi.z);
        const float tmin = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
        const float tmx = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
        return tmin <= tmx * 1.0000004f;
      };
      auto leaf_test = [&](int32_t leaf) {
        const int q = (int)P.rorder[leaf];
        const d3 w = ld3(P.rx + 3 * q) - o;
        const double ts = dot(w, d);
        if (ts < 0.0 || ts > tend) return;
        const double dist = norm(w - d * ts);
        const double rad = P.rfac * (L + ts);
        if (dist <= rad) {
          const uint32_t e = atomicAdd(P.ev_count, 1u);
          if (e < P.ev_cap) {
            P.ev_ray[e] = (uint32_t)rid;
            P.ev_qk[e] = ((uint32_t)q << 5) | (uint32_t)k;
          }
        }
      };
      if (box_hit(rroot[0], rroot[1], rroot[2], rroot[3], rroot[4], rroot[5])) {
        int sp = 0;
        int32_t node = 0;
        while (true) {
          const float4 n0 = P.rnodes[4 * node], n1 = P.rnodes[4 * node + 1], n2 = P.rnodes[4 * node + 2],
                       n3 = P.rnodes[4 * node + 3];
          bool hl = box_hit(n0.x, n0.y, n0.z, n0.w, n1.x, n1.y);
          bool hr = box_hit(n1.z, n1.w, n2.x, n2.y, n2.z, n2.w);
          const int32_t cl = __float_as_int(n3.x), cr = __float_as_int(n3.y);
          if (hl && cl < 0) {
            leaf_test(~cl);
            hl = false;
          }
          // a single-receiver tree repeats leaf 0 with an empty right box
          if (hr && cr < 0 && cr != cl) {
            leaf_test(~cr);
          }
          if (cr < 0) hr = false;
          if (hl && hr) {
            slot(sp) = (SE)cr;
            ++sp;
            node = cl;
          } else if (hl) {
            node = cl;
          } else if (hr) {
            node = cr;
          } else {
            if (sp == 0) break;
            --sp;
            node = (int32_t)slot(sp);
          }
        }
      }
    }
    if (tri < 0 || k == P.K) break;
    o = o + d * tend;
    L += tend;
    d = reflect(d, pl);
  }
}

// ---------------------------------------------------------------- hit barycentrics
// (u, v) of every hit on its triangle, P = (1 - u - v) v0 + u v1 + v v2
// (a diagnostic of the trace): each ray's chain replayed in FP64 as the
// capture replays it (the hit triangle's plane, specular reflection), NaN
// from the first segment without a hit; written by global ray id.
__global__ __launch_bounds__(256) void k_hits_uv(const GeoTables G, int N, int K, int64_t NR, int64_t T, RayOrder ord,
                                                 const double* __restrict__ tx, const int32_t* __restrict__ seq,
                                                 const double4* __restrict__ tplane,
                                                 const double* __restrict__ tri64, float* __restrict__ uv) {
  const int64_t rid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rid >= NR) return;
  int p;
  int64_t r;
  ray_of_pos(ord, rid, p, r);
  const int64_t g = rid_of_pos(ord, rid);
  d3 o = ld3(tx + 3 * p);
  d3 d = geo_dir(G, N, r);
  bool ended = false;
  for (int k = 0; k <= K; ++k) {
    float u = NAN, v = NAN;
    const int32_t tri = ended ? -1 : seq[(int64_t)k * NR + rid];
    if (tri >= 0 && tri < T) {
      const double4 pl = tplane[tri];
      const d3 P = o + d * advance_t(pl, o, d);
      const double* t = tri64 + 9 * (int64_t)tri;
      const d3 v0 = ld3(t), e1 = ld3(t + 3) - v0, e2 = ld3(t + 6) - v0, w = P - v0;
      const double d00 = dot(e1, e1), d01 = dot(e1, e2), d11 = dot(e2, e2), d20 = dot(w, e1), d21 = dot(w, e2);
      const double den = d00 * d11 - d01 * d01;
      u = (float)((d11 * d20 - d01 * d21) / den);
      v = (float)((d00 * d21 - d01 * d20) / den);
      o = P;
      d = reflect(d, pl);
    } else {
      ended = true;
    }
    uv[2 * (g * (K + 1) + k)] = u;
    uv[2 * (g * (K + 1) + k) + 1] = v;
  }
}

// ---------------------------------------------------------------- keys
__device__ inline uint64_t mix64(uint64_t h, uint64_t v) {
  h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
  h ^= h >> 31;
  h *= 0xbf58476d1ce4e5b9ull;
  h ^= h >> 29;
  return h;
}

struct KeyParams {
  const uint32_t* ev_ray;  // ray position of each capture
  const uint32_t* ev_qk;
  const int32_t* seq;
  const int32_t* tgroup;
  int64_t R, NR;
  int Nt;
  int64_t n;
  int hbits;  // hash bits below the segment index in the sort key
  int emin;   // ray positions in element-minor order
};

__device__ inline int ev_tx(const KeyParams& P, uint32_t pos) {
  int p;
  int64_t r;
  ray_of_pos(RayOrder{P.R, P.Nt, P.emin}, (int64_t)pos, p, r);
  return p;
}

__device__ inline int ev_groups(const KeyParams& P, int64_t e, int32_t* g) {
  const uint32_t rid = P.ev_ray[e];
  const int k = (int)(P.ev_qk[e] & 31u);
  for (int i = 0; i < k; ++i) g[i] = P.tgroup[P.seq[(int64_t)i * P.NR + rid]];
  return k;
}

// sort key of a capture: (segment = rx * Nt + tx) << hbits | the top hbits
// bits of a 32-bit hash of the face-group sequence.  Hash collisions only
// lengthen an equal-key run; the dedup below compares the exact sequences
// inside each run.
__global__ void k_event_keys(const KeyParams P, uint64_t* __restrict__ key, uint32_t* __restrict__ vals) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P.n) return;
  int32_t g[SBR_MAX_BOUNCES];
  const int k = ev_groups(P, e, g);
  uint64_t h = mix64(0x5bd1e995ull, (uint64_t)k);
  for (int i = 0; i < k; ++i) h = mix64(h, (uint64_t)(uint32_t)g[i]);
  const int64_t p = ev_tx(P, P.ev_ray[e]);
  const uint64_t q = P.ev_qk[e] >> 5;
  const uint32_t h32 = (uint32_t)(h ^ (h >> 32));
  key[e] = ((q * (uint64_t)P.Nt + (uint64_t)p) << P.hbits) | (uint64_t)(h32 >> (32 - P.hbits));
  vals[e] = (uint32_t)e;
}

// head flag: first occurrence of its exact key within its equal-sort-key run
__global__ void k_unique_heads(const KeyParams P, const uint32_t* __restrict__ perm,
                               const uint64_t* __restrict__ key_sorted, uint32_t* __restrict__ head) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n) return;
  const uint32_t e = perm[i];
  uint32_t is_head = 1;
  int32_t g[SBR_MAX_BOUNCES], g2[SBR_MAX_BOUNCES];
  int k = -1;
  for (int64_t j = i - 1; j >= 0; --j) {
    if (key_sorted[j] != key_sorted[i]) break;
    const uint32_t e2 = perm[j];
    if (k < 0) k = ev_groups(P, e, g);
    const int k2 = ev_groups(P, e2, g2);
    bool same = k2 == k;
    for (int t = 0; same && t < k; ++t) same = g[t] == g2[t];
    if (same) {
      is_head = 0;
      break;
    }
  }
  head[i] = is_head;
}

__global__ void k_compact_heads(const uint32_t* __restrict__ perm, const uint32_t* __restrict__ head,
                                const uint32_t* __restrict__ pos, int64_t n, uint32_t* __restrict__ key_event) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (head[i]) key_event[pos[i]] = perm[i];
}

// ---------------------------------------------------------------- rebuild
struct RebuildParams {
  KeyParams kp;
  const uint32_t* key_event;
  int64_t n_keys;               // capacity of the per-key arrays (an upper bound of the key count)
  const uint32_t* n_keys_dev;   // the key count, on the device
  int K, stride;
  const double* tx;
  const double* rx;
  const double4* gplane;
  const float4* gmat;
  const int32_t* gstart;
  const int32_t* gtri;
  const double* tri64;
  const float4* nodes;
  const float4* tri32;
  float root[6];
  double cx, cy, cz;
  int has_bvh;
  int n_big, big_off;  // oversized triangles outside the BVH (tri32 entries big_off ..)
  // outputs (indexed by key)
  uint32_t* valid;
  double* geo;
  double* info;    // length, delay
  float* ang;      // 4
  int32_t* key;    // 4 + K: tx, rx, k, flags, g...
  uint64_t* seg;
};

// Point-in-triangle for a point on the triangle's plane: the three edge
// functions, normalised by |n|^2, are its barycentric coordinates.  Inclusive
// with a 1e-9 margin so that a reflection point on an edge shared by two
// triangles of one face group is never rejected by both through rounding.
__device__ inline bool in_triangle(const double* t, d3 x) {
  const d3 a = ld3(t), b = ld3(t + 3), c = ld3(t + 6);
  const d3 n = cross(b - a, c - a);
  const double inv = 1.0 / dot(n, n);
  const double w0 = dot(n, cross(b - a, x - a)) * inv;
  const double w1 = dot(n, cross(c - b, x - b)) * inv;
  const double w2 = dot(n, cross(a - c, x - c)) * inv;
  return w0 >= -1e-9 && w1 >= -1e-9 && w2 >= -1e-9;
}

__device__ inline d3 mirror(d3 x, double4 pl) {
  const d3 n = mk3(pl.x, pl.y, pl.z);
  return x - n * (2.0 * (dot(n, x) - pl.w));
}

// kRebuildLanes consecutive lanes of a wave serve one key: every lane
// rebuilds the key's image points (a few FP64 steps), lane j checks the
// bounces and legs j, j + kRebuildLanes, ... (face, side and occlusion
// tests), a ballot over the key's lanes combines their verdicts, and the
// key's first lane writes the outputs.  This keeps one traversal, not k + 1,
// on each lane's dependent chain.
constexpr int kRebuildLanes = 8;

template <int STACK>
__global__ __launch_bounds__(128) void k_rebuild(const RebuildParams P) {
  __shared__ int32_t stack_mem[128 / kWave][STACK][kWave];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t* stk = &stack_mem[wv][0][lane];
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = gt / kRebuildLanes;
  const int sub = (int)(gt % kRebuildLanes);
  const int64_t nk = (int64_t)*P.n_keys_dev;
  const bool have = i < P.n_keys && i < nk;
  if (i < P.n_keys && i >= nk && sub == 0) P.valid[i] = 0u;  // slot beyond the keys: no path
  uint32_t e = 0;
  int32_t g[SBR_MAX_BOUNCES];
  int k = 0, p = 0, q = 0;
  bool ok = have;
  d3 X[SBR_MAX_BOUNCES + 2];
  if (have) {
    e = P.key_event[i];
    k = ev_groups(P.kp, e, g);
    p = ev_tx(P.kp, P.kp.ev_ray[e]);
    q = (int)(P.kp.ev_qk[e] >> 5);
    if (sub == 0) {
      int32_t* kk = P.key + i * (4 + P.K);
      kk[0] = p, kk[1] = q, kk[2] = k, kk[3] = 0;
      for (int t = 0; t < P.K; ++t) kk[4 + t] = t < k ? g[t] : -1;
      P.seg[i] = (uint64_t)q * (uint64_t)P.kp.Nt + (uint64_t)p;
    }
    const d3 T = ld3(P.tx + 3 * p), Rq = ld3(P.rx + 3 * q);
    // images S_1..S_k
    d3 S[SBR_MAX_BOUNCES + 1];
    S[0] = T;
    for (int t = 1; t <= k; ++t) S[t] = mirror(S[t - 1], P.gplane[g[t - 1]]);
    X[0] = T;
    X[k + 1] = Rq;
    for (int t = k; t >= 1 && ok; --t) {
      const double4 pl = P.gplane[g[t - 1]];
      const d3 n = mk3(pl.x, pl.y, pl.z);
      const d3 D = X[t + 1] - S[t];
      const double den = dot(n, D);
      if (den == 0.0) {
        ok = false;
        break;
      }
      X[t] = S[t] + D * ((pl.w - dot(n, S[t])) / den);
    }
    for (int t = 1 + sub; t <= k && ok; t += kRebuildLanes) {
      const int gi = g[t - 1];
      bool inside = false;
      for (int j = P.gstart[gi]; j < P.gstart[gi + 1] && !inside; ++j)
        inside = in_triangle(P.tri64 + 9 * (int64_t)P.gtri[j], X[t]);
      const double4 pl = P.gplane[gi];
      const d3 n = mk3(pl.x, pl.y, pl.z);
      const double sa = dot(n, X[t - 1]) - pl.w, sb = dot(n, X[t + 1]) - pl.w;
      ok = inside && (sa * sb > 0.0);
    }
    for (int t = 1 + sub; t <= k + 1 && ok; t += kRebuildLanes) {
      const int ga = t >= 2 ? g[t - 2] : -1;
      const int gb = t <= k ? g[t - 1] : -1;
      ok = !leg_blocked<STACK>(P, stk, X[t - 1], X[t], ga, gb);
    }
  }
  // a key is valid when none of its lanes failed
  const uint64_t failed = __ballot(have && !ok);
  const uint64_t mine = ((1ull << kRebuildLanes) - 1) << (lane & ~(kRebuildLanes - 1));
  ok = have && (failed & mine) == 0;
  if (!have || sub != 0) return;
  P.valid[i] = ok ? 1u : 0u;
  if (!ok) return;
  double len = 0.0;
  for (int t = 1; t <= k + 1; ++t) len += norm(X[t] - X[t - 1]);
  P.info[2 * i] = len;
  P.info[2 * i + 1] = len / kC0;
  const d3 kdep = normalize(X[1] - X[0]);
  const d3 toward = normalize(X[k] - X[k + 1]);
  P.ang[4 * i] = (float)(atan2(kdep.y, kdep.x) * (180.0 / kPi));
  P.ang[4 * i + 1] = (float)(asin(fmax(-1.0, fmin(1.0, kdep.z))) * (180.0 / kPi));
  P.ang[4 * i + 2] = (float)(atan2(toward.y, toward.x) * (180.0 / kPi));
  P.ang[4 * i + 3] = (float)(asin(fmax(-1.0, fmin(1.0, toward.z))) * (180.0 / kPi));
  // ---------------- frequency-independent polarisation chain
  double* G = P.geo + i * (int64_t)P.stride;
  for (int t = 0; t < P.stride; ++t) G[t] = 0.0;
  G[0] = len;
  G[1] = k;
  d3 th0, ph0;
  sph_hats(kdep, &th0, &ph0);
  if (k == 0) {
    // e_rx . e_tx with both ends seeing the same direction
    G[10] = dot(th0, th0), G[11] = dot(th0, ph0), G[12] = dot(ph0, th0), G[13] = dot(ph0, ph0);
    return;
  }
  d3 kin = kdep, s_prev{}, pout_prev{};
  for (int b = 1; b <= k; ++b) {
    const double4 pl = P.gplane[g[b - 1]];
    d3 n = mk3(pl.x, pl.y, pl.z);
    if (dot(kin, n) > 0.0) n = n * -1.0;
    const double cs = -dot(kin, n);
    d3 s = cross(kin, n);
    const double sn = norm(s);
    if (sn < 1e-15) {
      const d3 ref = fabs(kin.z) < 0.9 ? mk3(0, 0, 1) : mk3(1, 0, 0);
      s = normalize(cross(kin, ref));
    } else {
      s = s * (1.0 / sn);
    }
    const d3 pin = cross(s, kin);
    const d3 kout = kin - n * (2.0 * dot(kin, n));
    const d3 pout = cross(s, kout);
    const float4 m = P.gmat[g[b - 1]];
    double* B = G + kGeoHead + kGeoPerBounce * (b - 1);
    B[0] = cs, B[1] = m.x, B[2] = m.y, B[3] = m.z;
    if (b == 1) {
      G[2] = dot(th0, s), G[3] = dot(th0, pin), G[4] = dot(ph0, s), G[5] = dot(ph0, pin);
    } else {
      double* Bp = G + kGeoHead + kGeoPerBounce * (b - 2);
      Bp[4] = dot(s_prev, s), Bp[5] = dot(pout_prev, s), Bp[6] = dot(s_prev, pin), Bp[7] = dot(pout_prev, pin);
    }
    s_prev = s, pout_prev = pout;
    kin = kout;
  }
  d3 thr, phr;
  sph_hats(kin, &thr, &phr);
  G[6] = dot(thr, s_prev), G[7] = dot(thr, pout_prev), G[8] = dot(phr, s_prev), G[9] = dot(phr, pout_prev);
}

// ---------------------------------------------------------------- ordering
// order key of a valid path: segment << 32 | FP32 bits of its delay (positive
// floats order like their bit patterns); equal keys are resolved afterwards by
// the exact FP64 delay
__global__ void k_valid_keys(const uint32_t* __restrict__ valid, const uint32_t* __restrict__ pos,
                             const uint64_t* __restrict__ seg, const double* __restrict__ info, int64_t n,
                             uint64_t* __restrict__ okey, uint32_t* __restrict__ oidx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !valid[i]) return;
  const uint32_t j = pos[i];
  okey[j] = (seg[i] << 32) | (uint32_t)__float_as_uint((float)info[2 * i + 1]);
  oidx[j] = (uint32_t)i;
}

// Paths whose FP32 delays tie (equal sort keys) are put in exact FP64 delay
// order, ties broken by key index: the run starting at i is insertion-sorted
// by the thread that owns its first element.
__global__ void k_fix_delay_ties(const uint64_t* __restrict__ key, const double* __restrict__ info, int64_t n,
                                 uint32_t* __restrict__ order) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || (i > 0 && key[i - 1] == key[i])) return;
  int64_t e = i + 1;
  while (e < n && key[e] == key[i]) ++e;
  for (int64_t a = i + 1; a < e; ++a) {
    const uint32_t v = order[a];
    const double dv = info[2 * (int64_t)v + 1];
    int64_t b = a - 1;
    while (b >= i) {
      const uint32_t u = order[b];
      const double du = info[2 * (int64_t)u + 1];
      if (du < dv || (du == dv && u < v)) break;
      order[b + 1] = u;
      --b;
    }
    order[b + 1] = v;
  }
}

__global__ void k_gather_paths(const uint32_t* __restrict__ order, int64_t n, int stride, int K,
                               const double* __restrict__ geo_in, const double* __restrict__ info_in,
                               const float* __restrict__ ang_in, const int32_t* __restrict__ key_in,
                               double* __restrict__ geo, double* __restrict__ info, float* __restrict__ ang,
                               int32_t* __restrict__ key, uint64_t* __restrict__ seg_in, uint64_t* __restrict__ seg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = order[i];
  for (int t = 0; t < stride; ++t) geo[i * stride + t] = geo_in[(int64_t)s * stride + t];
  info[2 * i] = info_in[2 * s], info[2 * i + 1] = info_in[2 * s + 1];
  for (int t = 0; t < 4; ++t) ang[4 * i + t] = ang_in[4 * s + t];
  for (int t = 0; t < 4 + K; ++t) key[i * (4 + K) + t] = key_in[(int64_t)s * (4 + K) + t];
  seg[i] = seg_in[s];
}

__global__ void k_seg_start(const uint64_t* __restrict__ seg, int64_t n, int64_t nseg, int32_t* __restrict__ start) {
  const int64_t sidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sidx > nseg) return;
  int64_t lo = 0, hi = n;  // first i with seg[i] >= sidx
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (seg[mid] < (uint64_t)sidx) lo = mid + 1;
    else hi = mid;
  }
  start[sidx] = (int32_t)lo;
}

int bits_for(uint64_t v) {
  int b = 0;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

// Receiver frame of a set of up to kLbvhSmall points, on the device (one
// workgroup): FP64 box, centre rc = 0.5 (lo + hi), radius max |x - rc| (times
// 1 + 1e-12, plus 1e-12), FP32 point boxes nextafter((float)(x - rc)) outward
// and their bounds -- the host's operations for larger sets -- and the input
// checks of a receive: bad[0] = lowest receiver with a non-finite coordinate,
// bad[1] = lowest q Nt + p with receiver q on transmitter p (both preset to
// all ones by the host).  Outputs: frame = rc xyz, rrad; bounds = lo xyz, hi xyz.
constexpr int kRxPrepThreads = 1024;
// replay stack of trees from the one-workgroup builder: at most 41 entries
// (one per internal node on a path); 44 two-byte entries keep a 256-thread
// block at 22.5 KB of LDS, so that 7 blocks fit a CU
constexpr int kRxSmallStack = 44;
__global__ __launch_bounds__(kRxPrepThreads) void k_rx_prep(const double* __restrict__ rx, int Nr,
                                                            const double* __restrict__ tx, int Nt,
                                                            float* __restrict__ blo, float* __restrict__ bhi,
                                                            float* __restrict__ bounds, double* __restrict__ frame,
                                                            uint32_t* __restrict__ bad) {
  constexpr int W = kRxPrepThreads / kWave;
  __shared__ double dred[6][W];
  __shared__ float fred[6][W];
  __shared__ double lohi[6];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  auto lesser = [](double a, double b) { return b < a ? b : a; };
  auto greater = [](double a, double b) { return a < b ? b : a; };
  // box
  double b[6] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
  for (int q = t; q < Nr; q += kRxPrepThreads)
    for (int c = 0; c < 3; ++c) {
      const double x = rx[3 * q + c];
      if (!isfinite(x)) atomicMin(bad, (uint32_t)q);
      b[c] = lesser(b[c], x), b[3 + c] = greater(b[3 + c], x);
    }
  for (int o = 32; o > 0; o >>= 1)
    for (int k = 0; k < 6; ++k) {
      const double y = __shfl_xor(b[k], o, 64);
      b[k] = k < 3 ? lesser(b[k], y) : greater(b[k], y);
    }
  if (lane == 0)
    for (int k = 0; k < 6; ++k) dred[k][wv] = b[k];
  __syncthreads();
  if (t < 6) {
    double r = dred[t][0];
    for (int w = 1; w < W; ++w) r = t < 3 ? lesser(r, dred[t][w]) : greater(r, dred[t][w]);
    lohi[t] = r;
  }
  __syncthreads();
  const double rcx = 0.5 * (lohi[0] + lohi[3]), rcy = 0.5 * (lohi[1] + lohi[4]), rcz = 0.5 * (lohi[2] + lohi[5]);
  // radius and FP32 boxes
  double rad = 0.0;
  float fb[6] = {1e30f, 1e30f, 1e30f, -1e30f, -1e30f, -1e30f};
  for (int q = t; q < Nr; q += kRxPrepThreads) {
    const double v[3] = {rx[3 * q] - rcx, rx[3 * q + 1] - rcy, rx[3 * q + 2] - rcz};
    double d2 = 0.0;
    for (int c = 0; c < 3; ++c) d2 += v[c] * v[c];
    rad = greater(rad, sqrt(d2));
    for (int c = 0; c < 3; ++c) {
      const float l = nextafterf((float)v[c], -INFINITY), h = nextafterf((float)v[c], INFINITY);
      blo[3 * q + c] = l, bhi[3 * q + c] = h;
      fb[c] = fminf(fb[c], l), fb[3 + c] = fmaxf(fb[3 + c], h);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    rad = greater(rad, __shfl_xor(rad, o, 64));
    for (int k = 0; k < 6; ++k) {
      const float y = __shfl_xor(fb[k], o, 64);
      fb[k] = k < 3 ? fminf(fb[k], y) : fmaxf(fb[k], y);
    }
  }
  __syncthreads();  // the box reduction's LDS is reused
  if (lane == 0) {
    dred[0][wv] = rad;
    for (int k = 0; k < 6; ++k) fred[k][wv] = fb[k];
  }
  __syncthreads();
  if (t == 0) {
    double r = dred[0][0];
    for (int w = 1; w < W; ++w) r = greater(r, dred[0][w]);
    frame[0] = rcx, frame[1] = rcy, frame[2] = rcz, frame[3] = r * (1.0 + 1e-12) + 1e-12;
  }
  if (t < 6) {
    float r = fred[t][0];
    for (int w = 1; w < W; ++w) r = t < 3 ? fminf(r, fred[t][w]) : fmaxf(r, fred[t][w]);
    bounds[t] = r;
  }
  // a receiver on a transmitter
  for (int64_t i = t; i < (int64_t)Nr * Nt; i += kRxPrepThreads) {
    const int q = (int)(i / Nt), p = (int)(i - (int64_t)q * Nt);
    if (rx[3 * q] == tx[3 * p] && rx[3 * q + 1] == tx[3 * p + 1] && rx[3 * q + 2] == tx[3 * p + 2])
      atomicMin(bad + 1, (uint32_t)i);
  }
}

}  // namespace

void run_receive(sbr_paths_s* ps, const double* hrx, hipStream_t s) {
  sbr_trace_s* tr = ps->trace;
  sbr_scene_s* sc = tr->scene;
  const int Nr = ps->Nr, Nt = tr->Nt, K = tr->K;
  // ---------------- Rx BVH (FP32 boxes in a frame centred on the Rx bounding sphere).
  // Receiver points are clustered with the Morton-ordered LBVH: it builds
  // faster than PLOC for point sets and the capture queries ran faster on it.
  HostPhase hp_all("host:receive");
  std::optional<HostPhase> hp_rx, hp_step;
  hp_rx.emplace("host:rx_tree");
  // Sets of up to kLbvhSmall receivers: frame, boxes, input checks and tree
  // on the device with no synchronisation (the replay reads the frame and the
  // root box from device memory and needs no depth: such a tree has at most
  // 41 internal nodes on a path, within its kRxSmallStack-entry stack).
  // Larger sets: the same steps on the host, then the tree.
  const bool dev_prep = Nr <= kLbvhSmall;
  Buf dlo, dhi, rnodes, rorder, rroot, rframe, bad;
  dlo.alloc((size_t)Nr * 12, s);
  dhi.alloc((size_t)Nr * 12, s);
  rnodes.alloc((size_t)std::max(Nr - 1, 1) * 64, s);
  rorder.alloc((size_t)Nr * 4, s);
  rroot.alloc(32, s);  // 6 floats of root box, then the depth word
  float hroot[8] = {};
  int rdepth = 0;
  double rc[3] = {0.0, 0.0, 0.0}, rrad = 0.0;
  if (dev_prep) {
    rframe.alloc(64, s);  // rc xyz, rrad (doubles); then the FP32 bounds at byte 32
    bad.alloc(8, s);
    fill_u32(bad.as<uint32_t>(), 0xffffffffu, 2, s);
    float* dbounds = reinterpret_cast<float*>(rframe.as<char>() + 32);
    { ::sbr::TimedLaunch tl_("bvh", s); hipLaunchKernelGGL(k_rx_prep, dim3(1), dim3(kRxPrepThreads), 0, s, ps->rx.as<double>(), Nr,
                       tr->tx.as<double>(), Nt, dlo.as<float>(), dhi.as<float>(), dbounds, rframe.as<double>(),
                       bad.as<uint32_t>()); }
    SBR_LAUNCH_CHECK();
    BvhOut bo{rnodes.as<float4>(), rorder.as<uint32_t>(), rroot.as<float>(), nullptr,
              reinterpret_cast<uint32_t*>(rroot.as<float>() + 6)};
    bo.bounds_dev = dbounds;
    build_bvh(dlo.as<float>(), dhi.as<float>(), Nr, nullptr, nullptr, bo, s, /*linear=*/true);
  } else {
    hp_step.emplace("host:rx_boxes");
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int q = 0; q < Nr; ++q)
      for (int c = 0; c < 3; ++c) lo[c] = std::min(lo[c], hrx[3 * q + c]), hi[c] = std::max(hi[c], hrx[3 * q + c]);
    for (int c = 0; c < 3; ++c) rc[c] = 0.5 * (lo[c] + hi[c]);
    for (int q = 0; q < Nr; ++q) {
      double d2 = 0;
      for (int c = 0; c < 3; ++c) d2 += (hrx[3 * q + c] - rc[c]) * (hrx[3 * q + c] - rc[c]);
      rrad = std::max(rrad, std::sqrt(d2));
    }
    rrad = rrad * (1.0 + 1e-12) + 1e-12;
    std::vector<float> blo(3 * (size_t)Nr), bhi(3 * (size_t)Nr);
    float flo[3] = {1e30f, 1e30f, 1e30f}, fhi[3] = {-1e30f, -1e30f, -1e30f};
    for (int q = 0; q < Nr; ++q)
      for (int c = 0; c < 3; ++c) {
        const double v = hrx[3 * q + c] - rc[c];
        blo[3 * q + c] = std::nextafter((float)v, -INFINITY);
        bhi[3 * q + c] = std::nextafter((float)v, INFINITY);
        flo[c] = std::min(flo[c], blo[3 * q + c]);
        fhi[c] = std::max(fhi[c], bhi[3 * q + c]);
      }
    SBR_HIP(hipMemcpyAsync(dlo.p, blo.data(), blo.size() * 4, hipMemcpyHostToDevice, s));
    SBR_HIP(hipMemcpyAsync(dhi.p, bhi.data(), bhi.size() * 4, hipMemcpyHostToDevice, s));
    hp_step.emplace("host:rx_lbvh");
    rdepth = build_bvh(dlo.as<float>(), dhi.as<float>(), Nr, flo, fhi,
                       BvhOut{rnodes.as<float4>(), rorder.as<uint32_t>(), rroot.as<float>(), hroot}, s,
                       /*linear=*/true);
    SBR_CHECK(rdepth <= 64, SBR_E_UNSUPPORTED, "receiver tree depth %d", rdepth);
  }
  hp_step.reset();
  hp_rx.reset();

  // ---------------- replay + capture (grow the event buffer and retry on overflow)
  ReplayParams P{};
  P.G = geo_tables();
  P.N = tr->N, P.K = K, P.Nr = Nr, P.R = tr->R, P.NR = tr->NR;
  P.ord = RayOrder{tr->R, (int32_t)tr->Nt, (int32_t)tr->emin};
  P.T = sc->T;
  P.tx = tr->tx.as<double>();
  P.seq = tr->seq.as<int32_t>();
  P.tplane = sc->tplane.as<double4>();
  P.rnodes = rnodes.as<float4>();
  P.rorder = rorder.as<uint32_t>();
  for (int k = 0; k < 6; ++k) P.rroot[k] = hroot[k];
  P.rx = ps->rx.as<double>();
  for (int c = 0; c < 3; ++c) P.rc[c] = rc[c];
  P.rrad = rrad;
  if (dev_prep) P.rdev = rframe.as<double>(), P.rroot_dev = rroot.as<float>();
  P.rfac = ps->coeff * ps->alpha / std::sqrt(3.0);
  Buf cnt;
  cnt.alloc(16, s);
  const int cap0 = ps->ctx->tune.receive_event_capacity;
  uint64_t cap = cap0 > 0 ? (uint64_t)cap0 : std::max<uint64_t>(1u << 20, (uint64_t)tr->NR / 8);
  Buf& ev_ray = ps->ev_ray;
  Buf& ev_qk = ps->ev_qk;
  uint32_t n_ev = 0, hbad[2] = {0xffffffffu, 0xffffffffu};
  for (int attempt = 0; attempt < 3; ++attempt) {
    ev_ray.alloc(cap * 4, s);
    ev_qk.alloc(cap * 4, s);
    fill_u32(cnt.as<uint32_t>(), 0, 1, s);
    P.ev_count = cnt.as<uint32_t>();
    P.ev_cap = cap;
    P.ev_ray = ev_ray.as<uint32_t>();
    P.ev_qk = ev_qk.as<uint32_t>();
    // the block's traversal stacks live in LDS: a deep receiver tree caps
    // the block size so that they fit the 64 KiB a workgroup may allocate
    const size_t stack_bytes = dev_prep ? sizeof(int16_t) * kRxSmallStack
                                        : sizeof(int32_t) * (rdepth <= 16 ? 16 : rdepth <= 32 ? 32 : 64);
    const int rb = replay_block_for(ps->ctx->tune.replay_block, stack_bytes);
    const unsigned g = nblk(tr->NR, rb);
    const size_t lds = (size_t)rb * stack_bytes;
    ::sbr::TimedLaunch tl_("replay_capture", s);
    if (dev_prep)
      hipLaunchKernelGGL((k_replay_capture<kRxSmallStack, int16_t, true>), dim3(g), dim3(rb), lds, s, P);
    else if (rdepth <= 16)
      hipLaunchKernelGGL((k_replay_capture<16, int32_t, false>), dim3(g), dim3(rb), lds, s, P);
    else if (rdepth <= 32)
      hipLaunchKernelGGL((k_replay_capture<32, int32_t, false>), dim3(g), dim3(rb), lds, s, P);
    else
      hipLaunchKernelGGL((k_replay_capture<64, int32_t, false>), dim3(g), dim3(rb), lds, s, P);
    SBR_LAUNCH_CHECK();
    SBR_HIP(hipMemcpyAsync(&n_ev, cnt.p, 4, hipMemcpyDeviceToHost, s));
    if (dev_prep) SBR_HIP(hipMemcpyAsync(hbad, bad.p, 8, hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
    SBR_CHECK(hbad[0] == 0xffffffffu, SBR_E_INVALID_ARG, "rx coordinates must be finite (rx %u)", hbad[0]);
    SBR_CHECK(hbad[1] == 0xffffffffu, SBR_E_INVALID_ARG, "rx %u coincides with tx %u", hbad[1] / (uint32_t)Nt,
              hbad[1] % (uint32_t)Nt);
    if (n_ev <= cap) break;
    cap = (uint64_t)n_ev + n_ev / 8 + 1024;
  }
  SBR_CHECK(n_ev <= cap, SBR_E_CAPACITY, "capture events overflow (%u)", n_ev);
  SBR_CHECK(n_ev < 0x7fffffffu, SBR_E_UNSUPPORTED, "too many capture events (%u)", n_ev);
  ps->n_events = n_ev;
  const int64_t E = n_ev;
  const int stride = geo_stride(K);
  ps->n_keys = 0;
  ps->n_paths = 0;
  const int64_t nseg = (int64_t)Nr * Nt;
  ps->seg_start.alloc((size_t)(nseg + 1) * 4, s);
  if (E == 0) {
    fill_u32(ps->seg_start.as<uint32_t>(), 0, nseg + 1, s);
    return;
  }
  // ---------------- keys, one sort by (segment, hash), exact dedup
  const int sbits = std::max(1, bits_for((uint64_t)nseg));
  // Sort key: segment index, then a hash of the face-group sequence.  The
  // hash only groups equal keys (k_unique_heads compares the sequences
  // themselves within a run of equal sort keys), so it is cut to fill 32 bits
  // when the segment index leaves at least 16: four 8-bit passes instead of
  // six for up to 65,536 (rx, tx) pairs.
  const int hbits = std::max(16, 32 - sbits);
  KeyParams kp{ev_ray.as<uint32_t>(), ev_qk.as<uint32_t>(), tr->seq.as<int32_t>(), sc->tgroup.as<int32_t>(),
               tr->R, tr->NR, Nt, E, hbits, tr->emin};
  Buf k1, k2, v1, v2, temp;
  k1.alloc(E * 8, s), k2.alloc(E * 8, s), v1.alloc(E * 4, s), v2.alloc(E * 4, s);
  temp.alloc(std::max(radix_sort_temp_bytes(E), scan_temp_bytes(E)), s);
  { ::sbr::TimedLaunch tl_("keys", s); hipLaunchKernelGGL(k_event_keys, dim3(nblk(E, 256)), dim3(256), 0, s, kp, k1.as<uint64_t>(), v1.as<uint32_t>()); }
  SBR_LAUNCH_CHECK();
  radix_sort_pairs(k1.as<uint64_t>(), v1.as<uint32_t>(), k2.as<uint64_t>(), v2.as<uint32_t>(), E, 0, hbits + sbits,
                   temp.p, s);
  // now: v2 = event permutation, k2 = sorted keys
  Buf head, pos, tot;
  head.alloc(E * 4, s), pos.alloc(E * 4, s), tot.alloc(8, s);
  { ::sbr::TimedLaunch tl_("keys", s); hipLaunchKernelGGL(k_unique_heads, dim3(nblk(E, 256)), dim3(256), 0, s, kp, v2.as<uint32_t>(), k2.as<uint64_t>(),
                     head.as<uint32_t>()); }
  SBR_LAUNCH_CHECK();
  exclusive_scan_u32(head.as<uint32_t>(), pos.as<uint32_t>(), E, tot.as<uint32_t>(), temp.p, s);
  // the key count stays on the device: per-key arrays are sized by the event
  // count (an upper bound) and the rebuild reads the count itself
  Buf key_event;
  key_event.alloc((size_t)E * 4, s);
  { ::sbr::TimedLaunch tl_("keys", s); hipLaunchKernelGGL(k_compact_heads, dim3(nblk(E, 256)), dim3(256), 0, s, v2.as<uint32_t>(), head.as<uint32_t>(),
                     pos.as<uint32_t>(), E, key_event.as<uint32_t>()); }
  SBR_LAUNCH_CHECK();
  // ---------------- exact rebuild + validation
  const int64_t nk = E;
  Buf valid, geo, info, ang, key, seg;
  valid.alloc(nk * 4, s), geo.alloc(nk * stride * 8, s), info.alloc(nk * 16, s), ang.alloc(nk * 16, s);
  key.alloc(nk * (4 + K) * 4, s), seg.alloc(nk * 8, s);
  RebuildParams RP{};
  RP.kp = kp;
  RP.key_event = key_event.as<uint32_t>();
  RP.n_keys = nk;
  RP.n_keys_dev = tot.as<uint32_t>();
  RP.K = K;
  RP.stride = stride;
  RP.tx = tr->tx.as<double>();
  RP.rx = ps->rx.as<double>();
  RP.gplane = sc->gplane.as<double4>();
  RP.gmat = sc->gmat.as<float4>();
  RP.gstart = sc->gstart.as<int32_t>();
  RP.gtri = sc->gtri.as<int32_t>();
  RP.tri64 = sc->tri64.as<double>();
  RP.nodes = sc->nodes.as<float4>();
  RP.tri32 = sc->tri32.as<float4>();
  for (int k = 0; k < 6; ++k) RP.root[k] = sc->root_host[k];
  RP.cx = sc->center[0], RP.cy = sc->center[1], RP.cz = sc->center[2];
  RP.has_bvh = sc->n_bvh > 0;
  RP.n_big = sc->n_big;
  RP.big_off = (int)sc->n_bvh;
  RP.valid = valid.as<uint32_t>();
  RP.geo = geo.as<double>();
  RP.info = info.as<double>();
  RP.ang = ang.as<float>();
  RP.key = key.as<int32_t>();
  RP.seg = seg.as<uint64_t>();
  {
    const unsigned g = nblk(nk * kRebuildLanes, 128);
    const int depth = sc->bvh_depth;
    if (depth <= 16)
      { ::sbr::TimedLaunch tl_("rebuild", s); hipLaunchKernelGGL(k_rebuild<16>, dim3(g), dim3(128), 0, s, RP); }
    else if (depth <= 32)
      { ::sbr::TimedLaunch tl_("rebuild", s); hipLaunchKernelGGL(k_rebuild<32>, dim3(g), dim3(128), 0, s, RP); }
    else
      { ::sbr::TimedLaunch tl_("rebuild", s); hipLaunchKernelGGL(k_rebuild<64>, dim3(g), dim3(128), 0, s, RP); }
    SBR_LAUNCH_CHECK();
  }
  Buf tot2;
  tot2.alloc(8, s);
  exclusive_scan_u32(valid.as<uint32_t>(), pos.as<uint32_t>(), nk, tot2.as<uint32_t>(), temp.p, s);
  uint32_t counts[2] = {0, 0};  // keys, paths
  SBR_HIP(hipMemcpyAsync(&counts[0], tot.p, 4, hipMemcpyDeviceToHost, s));
  SBR_HIP(hipMemcpyAsync(&counts[1], tot2.p, 4, hipMemcpyDeviceToHost, s));
  SBR_HIP(hipStreamSynchronize(s));
  ps->n_keys = counts[0];
  const uint32_t n_paths = counts[1];
  ps->n_paths = n_paths;
  const int64_t np = n_paths;
  ps->geo.alloc(std::max<int64_t>(np, 1) * stride * 8, s);
  ps->info.alloc(std::max<int64_t>(np, 1) * 16, s);
  ps->ang.alloc(std::max<int64_t>(np, 1) * 16, s);
  ps->key.alloc(std::max<int64_t>(np, 1) * (4 + K) * 4, s);
  ps->power.alloc(std::max<int64_t>(np, 1) * 8, s);
  if (np == 0) {
    fill_u32(ps->seg_start.as<uint32_t>(), 0, nseg + 1, s);
    return;
  }
  // ---------------- order by (segment, delay)
  Buf ok1, ok2, oi1, oi2, fseg;
  ok1.alloc(np * 8, s), ok2.alloc(np * 8, s), oi1.alloc(np * 4, s), oi2.alloc(np * 4, s), fseg.alloc(np * 8, s);
  { ::sbr::TimedLaunch tl_("order", s); hipLaunchKernelGGL(k_valid_keys, dim3(nblk(nk, 256)), dim3(256), 0, s, valid.as<uint32_t>(), pos.as<uint32_t>(),
                     seg.as<uint64_t>(), info.as<double>(), nk, ok1.as<uint64_t>(), oi1.as<uint32_t>()); }
  SBR_LAUNCH_CHECK();
  Buf ptemp;
  ptemp.alloc(radix_sort_temp_bytes(np), s);
  radix_sort_pairs(ok1.as<uint64_t>(), oi1.as<uint32_t>(), ok2.as<uint64_t>(), oi2.as<uint32_t>(), np, 0, 32 + sbits,
                   ptemp.p, s);
  uint32_t* order_idx = oi2.as<uint32_t>();
  { ::sbr::TimedLaunch tl_("order", s); hipLaunchKernelGGL(k_fix_delay_ties, dim3(nblk(np, 256)), dim3(256), 0, s, ok2.as<uint64_t>(), info.as<double>(), np, order_idx); }
  SBR_LAUNCH_CHECK();
  // order_idx = key index of each final path
  { ::sbr::TimedLaunch tl_("order", s); hipLaunchKernelGGL(k_gather_paths, dim3(nblk(np, 256)), dim3(256), 0, s, order_idx, np, stride, K,
                     geo.as<double>(), info.as<double>(), ang.as<float>(), key.as<int32_t>(), ps->geo.as<double>(),
                     ps->info.as<double>(), ps->ang.as<float>(), ps->key.as<int32_t>(), seg.as<uint64_t>(),
                     fseg.as<uint64_t>()); }
  SBR_LAUNCH_CHECK();
  { ::sbr::TimedLaunch tl_("order", s); hipLaunchKernelGGL(k_seg_start, dim3(nblk(nseg + 1, 256)), dim3(256), 0, s, fseg.as<uint64_t>(), np, nseg,
                     ps->seg_start.as<int32_t>()); }
  SBR_LAUNCH_CHECK();
  // no final synchronisation: the path arrays are written in stream order and
  // the temporaries are released in stream order
}

void run_hits_uv(sbr_trace_s* tr, float* uv, hipStream_t s) {
  const int64_t NR = tr->NR;
  if (NR == 0) return;
  ::sbr::TimedLaunch tl_("misc", s);
  hipLaunchKernelGGL(k_hits_uv, dim3(nblk(NR, 256)), dim3(256), 0, s, geo_tables(), tr->N, tr->K, NR, tr->scene->T,
                     RayOrder{tr->R, (int32_t)tr->Nt, (int32_t)tr->emin}, tr->tx.as<double>(), tr->seq.as<int32_t>(),
                     tr->scene->tplane.as<double4>(), tr->scene->tri64.as<double>(), uv);
  SBR_LAUNCH_CHECK();
}

}  // namespace sbr
