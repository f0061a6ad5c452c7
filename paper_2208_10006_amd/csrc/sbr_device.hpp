// sbr_device.hpp -- device-side helpers shared by the libsbr kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sbr {

// ----------------------------------------------------------------- FP64 vectors
struct d3 {
  double x, y, z;
};
__host__ __device__ inline d3 mk3(double x, double y, double z) { return d3{x, y, z}; }
__host__ __device__ inline d3 operator+(d3 a, d3 b) { return d3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__host__ __device__ inline d3 operator-(d3 a, d3 b) { return d3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__host__ __device__ inline d3 operator*(d3 a, double s) { return d3{a.x * s, a.y * s, a.z * s}; }
__host__ __device__ inline double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__host__ __device__ inline d3 cross(d3 a, d3 b) {
  return d3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__host__ __device__ inline double norm(d3 a) { return sqrt(dot(a, a)); }
__host__ __device__ inline d3 normalize(d3 a) { return a * (1.0 / norm(a)); }
__host__ __device__ inline d3 ld3(const double* p) { return d3{p[0], p[1], p[2]}; }

// ----------------------------------------------------------------- FP64 complex
struct cd {
  double re, im;
};
__device__ inline cd cmk(double r, double i) { return cd{r, i}; }
__device__ inline cd cadd(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ inline cd csub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ inline cd cmul(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cd cscale(cd a, double s) { return cd{a.re * s, a.im * s}; }
// The per-(path, subcarrier) field kernels spend much of their time in a
// complex square root, a reciprocal and a square root per subcarrier.  Their
// arguments stay in ranges where the scaling and special-case handling of
// the general-purpose routines is not needed (the Fresnel terms are of
// moderate size: |eps_c| below about 1e8 even for metals at 1 GHz, so no
// square of them overflows or underflows), so these take the hardware
// estimates and refine them, to within about one unit in the last place:
//   * rcp64: the reciprocal estimate (relative error about 2^-23) and two
//     Newton steps;
//   * sqrt_hrsq: sqrt(x) and 1 / (2 sqrt(x)) together, from Goldschmidt's
//     iteration on the reciprocal square root estimate (twice) and one
//     Newton correction of the square root;
//   * csqrt_mod: the principal square root through t = (|z| + |Re z|) / 2,
//     sqrt(t) and Im z / (2 sqrt(t)) from one sqrt_hrsq (no division).
__device__ inline double rcp64(double x) {  // finite x != 0, 1 / x normal
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ inline void sqrt_hrsq(double x, double& s, double& h) {  // normal x > 0 (0 gives NaN)
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, hh = 0.5 * y;
  double r = fma(-g, hh, 0.5);
  g = fma(g, r, g);
  hh = fma(hh, r, hh);
  r = fma(-g, hh, 0.5);
  g = fma(g, r, g);
  hh = fma(hh, r, hh);
  const double d = fma(-g, g, x);
  s = fma(d, hh, g);
  h = hh;
}
__device__ inline double sqrt_nonneg(double x) {  // x >= 0
  double s, h;
  sqrt_hrsq(x, s, h);
  return x > 0.0 ? s : 0.0;
}
// a / b = conj(b) a / |b|^2
__device__ inline cd cdiv_mod(cd a, cd b) {
  const double inv = rcp64(b.re * b.re + b.im * b.im);
  return cd{(a.re * b.re + a.im * b.im) * inv, (a.im * b.re - a.re * b.im) * inv};
}
// principal square root (0 for z = 0); on the negative real axis the sign of
// Im z, -0 included, picks the branch
__device__ inline cd csqrt_mod(cd z) {
  double m, hm;
  sqrt_hrsq(fma(z.re, z.re, z.im * z.im), m, hm);
  const double t = 0.5 * (m + fabs(z.re));
  double s, h;
  sqrt_hrsq(t, s, h);
  if (!(t > 0.0)) s = h = 0.0;
  const double w = z.im * h;  // Im z / (2 sqrt(t))
  return z.re >= 0.0 ? cd{s, w} : cd{fabs(w), copysign(s, z.im)};
}


// ----------------------------------------------------------------- geodesic
// Icosahedron tables passed by value to kernels (built on the host by search).
struct GeoTables {
  double v[12][3];
  int e[30][2];
  int f[20][3];
};
const GeoTables& geo_tables();

// Direction of ray id of the frequency-N class-I geodesic (Sec. II-A-1):
// 12 corners, then 30 edges x (N-1) interior points from the lower vertex,
// then 20 faces x (N-1)(N-2)/2 interior points in row-major (i, j) order.
__device__ inline d3 geo_dir(const GeoTables& G, int N, int64_t id) {
  if (id < 12) return ld3(G.v[id]);
  id -= 12;
  const int64_t ne = 30LL * (N - 1);
  if (id < ne) {
    const int e = (int)(id / (N - 1));
    const int i = (int)(id - (int64_t)e * (N - 1)) + 1;
    const d3 a = ld3(G.v[G.e[e][0]]), b = ld3(G.v[G.e[e][1]]);
    const double w = (double)i / (double)N;
    return normalize(a + (b - a) * w);
  }
  id -= ne;
  const int64_t per = (int64_t)(N - 1) * (N - 2) / 2;
  const int f = (int)(id / per);
  const int64_t l = id - (int64_t)f * per;
  // rows i = 1..N-2 hold N-1-i points; points before row i:
  //   S(i) = (i-1)(N-1) - (i-1) i / 2.  Invert with a real root, then fix up.
  const double M = (double)(N - 1);
  const double disc = (M - 0.5) * (M - 0.5) - 2.0 * (double)l;
  int i = (int)floor((M - 0.5) - sqrt(disc > 0 ? disc : 0.0)) + 1;
  if (i < 1) i = 1;
  if (i > N - 2) i = N - 2;
  auto S = [&](int r) -> int64_t { return (int64_t)(r - 1) * (N - 1) - (int64_t)(r - 1) * r / 2; };
  while (i > 1 && S(i) > l) --i;
  while (i < N - 2 && S(i + 1) <= l) ++i;
  const int j = (int)(l - S(i)) + 1;
  const d3 a = ld3(G.v[G.f[f][0]]), b = ld3(G.v[G.f[f][1]]), c = ld3(G.v[G.f[f][2]]);
  const double wi = (double)i / (double)N, wj = (double)j / (double)N;
  return normalize(a + (b - a) * wi + (c - a) * wj);
}

// ----------------------------------------------------------------- ray positions
// A trace keeps its rays (hit chain, ray buffers, replay threads) in one of
// two orders.  Element-major: position i is direction i % R of element i / R.
// Element-minor, for arrays of several elements: position i is direction
// i / Nt of element i % Nt, so the 64 lanes of a wave follow one launch
// direction from 64 neighbouring elements -- nearly parallel rays a few
// millimetres apart that visit the same tree nodes and mostly hit the same
// triangles.  Outside the library a ray is always named by its global id
// p R + r, whatever the order.
struct RayOrder {
  int64_t R;   // rays per element
  int32_t Nt;  // elements
  int32_t emin;  // 1: element-minor
};
__host__ __device__ inline void ray_of_pos(const RayOrder& o, int64_t pos, int& p, int64_t& r) {
  if (o.emin) {
    const int64_t q = pos / o.Nt;
    p = (int)(pos - q * o.Nt);
    r = q;
  } else {
    p = (int)(pos / o.R);
    r = pos - (int64_t)p * o.R;
  }
}
__host__ __device__ inline int64_t rid_of_pos(const RayOrder& o, int64_t pos) {
  int p;
  int64_t r;
  ray_of_pos(o, pos, p, r);
  return (int64_t)p * o.R + r;
}

// ----------------------------------------------------------------- FP64 ray step
// Exact continuation of a ray whose FP32 traversal selected a triangle with
// plane (n, c): the hit distance is re-evaluated in FP64 on that plane, so the
// ray state never accumulates FP32 rounding between bounces.
__device__ inline double plane_t(const double4 pl, d3 o, d3 d) {
  const d3 n = mk3(pl.x, pl.y, pl.z);
  return (pl.w - dot(n, o)) / dot(n, d);
}
// distance to the selected plane, used by both the trace and the replay so the
// two rebuild the same FP64 chain (a degenerate value collapses to 0)
__device__ inline double advance_t(const double4 pl, d3 o, d3 d) {
  const double t = plane_t(pl, o, d);
  return (t >= 0.0 && t < INFINITY) ? t : 0.0;
}
// specular reflection about the plane normal (Snell's law, Sec. II-A-2)
__device__ inline d3 reflect(d3 d, const double4 pl) {
  const d3 n = mk3(pl.x, pl.y, pl.z);
  return d - n * (2.0 * dot(d, n));
}

// spherical unit vectors of a propagation direction (phi = atan2(y, x), 0 at the poles)
__device__ inline void sph_hats(d3 u, d3* th, d3* ph) {
  const double st = sqrt(u.x * u.x + u.y * u.y);
  double cp = 1.0, sp = 0.0;
  if (st > 0.0) {
    cp = u.x / st;
    sp = u.y / st;
  }
  *th = mk3(u.z * cp, u.z * sp, -st);
  *ph = mk3(-sp, cp, 0.0);
}

// ----------------------------------------------------------------- wave helpers
__device__ inline uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Inclusive scan over the 64 lanes of a wave with DPP moves: shifts by 1, 2,
// 4 and 8 within each row of 16 lanes, then the row_bcast:15 and row_bcast:31
// broadcasts carry row totals into the rows above (GFX9 DPP controls).  Every
// lane of the wave must be active.
__device__ inline uint32_t wave_inclusive_scan(uint32_t x, int lane) {
  const int rl = lane & 15;
  uint32_t t;
  t = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x111, 0xf, 0xf, false);
  if (rl >= 1) x += t;
  t = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x112, 0xf, 0xf, false);
  if (rl >= 2) x += t;
  t = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x114, 0xf, 0xf, false);
  if (rl >= 4) x += t;
  t = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x118, 0xf, 0xf, false);
  if (rl >= 8) x += t;
  t = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x142, 0xf, 0xf, false);
  if ((lane & 31) >= 16) x += t;
  t = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x143, 0xf, 0xf, false);
  if (lane >= 32) x += t;
  return x;
}

}  // namespace sbr
