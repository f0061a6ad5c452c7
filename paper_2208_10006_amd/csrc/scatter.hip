// scatter.hip -- first-order directive diffuse scattering (the paper's
// scattering coefficient S in the field of a path, eq. (2), and its
// "directive scattering model based on ER theory", Sec. II-A-2 and
// Fig. 3(b); the paper gives no formula).
//
// Reading: the single-lobe directive pattern of the effective-roughness
// model, first order (Tx -> surface tile -> Rx), the scattered share tied to
// the paper's roughness model:
//  * tiles: triangle t of area A is cut by its barycentric grid into m^2
//    equal sub-triangles, m = max(1, ceil(sqrt(A / tile_area))); a tile is a
//    sub-triangle, represented by its centroid and area dS = A / m^2; order:
//    by triangle, then the upward sub-triangles by (i, j), then the downward
//    ones by (i, j);
//  * a path Tx -> C -> Rx through tile centroid C exists when Tx and Rx lie
//    strictly on the same side of the triangle's plane and neither leg
//    crosses a triangle outside the tile's face group;
//  * field: the specularly reflected field at C,
//    E_r = Gamma_TE (E.s) s + Gamma_TM (E.p_in) p_out, without its component
//    along the scattering direction k_s, carries the share 1 - rho^2 of the
//    reflected power that the Kirchhoff factor rho (eq. (8)) removes from the
//    specular reflection, spread by the lobe ((1 + cos psi) / 2)^alpha around
//    the specular direction and normalised by its integral F_alpha over the
//    half-space:
//      a = (lambda / 4 pi) / (r_i r_s) sqrt(dS cos theta_i / F_alpha)
//          sqrt(1 - rho^2) ((1 + cos psi) / 2)^(alpha/2) (E_s . e_rx) e^{-jk (r_i + r_s)}.
//
// Pipeline as for the edge diffraction: a tile table built on the host per
// call -> the same-side test per (Rx, Tx, tile) candidate -> ordered
// compaction -> both legs against the BVH -> ordered compaction -> records
// and a CSR per (Rx, Tx) pair; the field kernel adds each pair's paths to H
// in a fixed order.
#include <algorithm>
#include <cmath>
#include <vector>

#include "occlusion.hpp"
#include "sbr_device.hpp"
#include "sbr_internal.hpp"

namespace sbr {

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

struct ScatArgs {
  const TileDev* tl;
  int64_t NT;  // tiles
  int Nt, Nr;
  const double* tx;
  const double* rx;
};

struct ScatScene {
  const float4* nodes;
  const float4* tri32;
  const double* tri64;
  float root[6];
  double cx, cy, cz;
  int has_bvh, n_big, big_off;
};

// candidate c = ((q Nt + p) NT + tile)
__device__ inline void scat_decode(const ScatArgs& A, int64_t c, int& p, int& q, int& ti) {
  ti = (int)(c % A.NT);
  const int64_t pr = c / A.NT;
  q = (int)(pr / A.Nt);
  p = (int)(pr - (int64_t)q * A.Nt);
}

// The legs factor: Tx -> C depends on (tile, Tx) only and C -> Rx on (tile,
// Rx) only, so each is traced once per (point, tile) rather than once per
// (tile, Tx, Rx) candidate.  h[j NT + tile] = (P_j - C) . n for the tile's
// centroid C and its triangle's unit normal n, set to 0 when the leg between
// P_j and C (from P_j when from_point, else from C) crosses a triangle outside
// the tile's face group; clear counts the non-zero entries.
template <int STACK>
__global__ __launch_bounds__(128) void k_scat_side(ScatArgs A, ScatScene S, const double* __restrict__ pts, int Np,
                                                   int from_point, double* __restrict__ h,
                                                   unsigned long long* __restrict__ clear) {
  __shared__ int32_t stack_mem[2][STACK][kWave];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t* stk = &stack_mem[wv][0][lane];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool nz = false;
  if (i < (int64_t)Np * A.NT) {
    const int j = (int)(i / A.NT);
    const int ti = (int)(i - (int64_t)j * A.NT);
    const TileDev t = A.tl[ti];
    const d3 C = ld3(t.c), P = ld3(pts + 3 * j);
    double v = dot(P - C, ld3(t.n));
    if (v != 0.0) {
      const bool b = from_point ? leg_blocked<STACK>(S, stk, P, C, t.group, t.group)
                                : leg_blocked<STACK>(S, stk, C, P, t.group, t.group);
      if (b) v = 0.0;
    }
    h[i] = v;
    nz = v != 0.0;
  }
  const unsigned long long m = __ballot(nz);
  if (lane == 0 && m) atomicAdd(clear, (unsigned long long)__popcll(m));
}

// a path: Tx and Rx strictly on the same side of the tile's plane, both legs clear
__global__ __launch_bounds__(256) void k_scat_candidates(ScatArgs A, int64_t C, const double* __restrict__ ht,
                                                         const double* __restrict__ hr, uint32_t* __restrict__ flag) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  int p, q, ti;
  scat_decode(A, c, p, q, ti);
  flag[c] = ht[(int64_t)p * A.NT + ti] * hr[(int64_t)q * A.NT + ti] > 0.0 ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_scat_compact(const uint32_t* __restrict__ flag,
                                                      const uint32_t* __restrict__ pos, int64_t n,
                                                      int64_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  dst[pos[i]] = i;
}

// ids[i] = (tx, rx, tile), rec[i] = (r_i, r_s); paths per (Rx, Tx) pair counted
__global__ __launch_bounds__(256) void k_scat_records(ScatArgs A, const int64_t* __restrict__ path, int64_t n,
                                                      int32_t* __restrict__ ids, double* __restrict__ rec,
                                                      uint32_t* __restrict__ pair_count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p, q, ti;
  scat_decode(A, path[i], p, q, ti);
  const TileDev t = A.tl[ti];
  const d3 C = ld3(t.c), dt = C - ld3(A.tx + 3 * p), dr = ld3(A.rx + 3 * q) - C;
  ids[3 * i] = p, ids[3 * i + 1] = q, ids[3 * i + 2] = ti;
  rec[2 * i] = sqrt(dot(dt, dt));
  rec[2 * i + 1] = sqrt(dot(dr, dr));
  atomicAdd(&pair_count[(int64_t)q * A.Nt + p], 1u);
}

// ---------------------------------------------------------------- field
// F_alpha(theta_i) = integral over the half-space of ((1 + cos psi) / 2)^alpha,
// psi measured from the specular direction (at theta_i from the normal).
// With ((1 + x) / 2)^alpha = 2^-alpha sum_j C(alpha, j) x^j and
// cos psi = sin t sin ti cos f + cos t cos ti, the azimuth keeps the even
// powers of cos f (int cos^k f df = 2 pi C(k, k/2) / 2^k) and the polar
// integrals are J(k, m) = int_0^{pi/2} sin^{k+1} t cos^m t dt
//   = 1 / (m + 1) prod_{l = 2, 4 .. k} l / (l + m + 1)   (no cancellation),
// so F = sum_{h, m} B[h][m] cos^m ti sin^{2h} ti with
//   B[h][m] = 2^-alpha C(alpha, m + 2h) C(m + 2h, 2h) 2 pi C(2h, h) 4^-h J(2h, m) >= 0,
// a sum of non-negative terms; the host builds B once per exponent.
__device__ inline double lobe_eval(const double* __restrict__ B, int alpha, double ci) {
  const double s2 = fmax(0.0, 1.0 - ci * ci);
  double tot = 0.0, sp = 1.0;
  for (int h = 0; 2 * h <= alpha; ++h) {
    const double* row = B + h * (alpha + 1);
    double acc = 0.0;
    for (int m = alpha - 2 * h; m >= 0; --m) acc = fma(acc, ci, row[m]);
    tot = fma(acc, sp, tot);
    sp *= s2;
  }
  return tot;
}

// theta-hat (pol 0) or phi-hat (pol 1) of direction u
__device__ inline d3 pol_vec_s(d3 u, int pol) {
  if (pol) {
    const double ph = atan2(u.y, u.x);
    double sp, cp;
    sincos(ph, &sp, &cp);
    return mk3(-sp, cp, 0.0);
  }
  const double st = sqrt(u.x * u.x + u.y * u.y);
  double cp = 1.0, sp = 0.0;
  if (st > 0.0) cp = u.x / st, sp = u.y / st;
  return mk3(u.z * cp, u.z * sp, -st);
}

struct ScatField {
  const double* freq;
  const float* atm_db;
  const float* atm_deg;
  int Nf, ptx, prx, alpha;
  const double* lobe;  // B[alpha / 2 + 1][alpha + 1]
  const float4* gmat;
};

// frequency-independent part of one path for one polarisation pair, written
// once per call by k_scat_geo and read by every frequency
struct ScatRec {
  double wa, wb;     // (E . s)(s' . e_rx) and (E . p_in)(p_out' . e_rx), ' = without the k_s component
  double cs, s2;     // cos theta_i, 1 - cos^2 theta_i
  double er, sg;     // eps_r and -sigma / (2 pi eps0): eps = er + j sg / f
  double gc;         // 4 pi h cos theta_i / c (the roughness exponent g = gc f); 0 on smooth faces
  double len, base;  // r_i + r_s; the amplitude without lambda and sqrt(1 - rho^2)
  double len_c;      // (r_i + r_s) / c
};

__device__ inline ScatRec scat_rec(const ScatArgs& A, const ScatField& F, const int32_t* ids, const double* rec) {
  ScatRec g;
  const TileDev t = A.tl[ids[2]];
  const d3 C = ld3(t.c), T = ld3(A.tx + 3 * ids[0]), R = ld3(A.rx + 3 * ids[1]);
  const double ri = rec[0], rs = rec[1];
  const d3 ki = (C - T) * (1.0 / ri), ks = (R - C) * (1.0 / rs);
  d3 n = ld3(t.n);
  if (dot(ki, n) > 0.0) n = n * -1.0;  // the normal facing the incidence
  const double cs = -dot(ki, n);
  const d3 kr = ki - n * (2.0 * dot(ki, n));
  d3 s = cross(ki, n);
  const double sn = sqrt(dot(s, s));
  if (sn < 1e-15) {  // normal incidence: any s normal to k_i
    const d3 tmp = fabs(ki.x) < 0.9 ? mk3(1, 0, 0) : mk3(0, 1, 0);
    s = cross(ki, tmp);
    s = s * (1.0 / sqrt(dot(s, s)));
  } else {
    s = s * (1.0 / sn);
  }
  const d3 pin = cross(s, ki), pout = cross(s, kr);
  const d3 E = pol_vec_s(ki, F.ptx), er = pol_vec_s(ks, F.prx);
  const double ke = dot(ks, er);
  g.wa = dot(E, s) * (dot(s, er) - dot(s, ks) * ke);
  g.wb = dot(E, pin) * (dot(pout, er) - dot(pout, ks) * ke);
  const double cpsi = dot(ks, kr);
  const double lobe = pow(0.5 * (1.0 + cpsi), 0.5 * F.alpha);
  g.base = (1.0 / (4.0 * kPi)) / (ri * rs) * sqrt(t.ds * cs / lobe_eval(F.lobe, F.alpha, cs)) * lobe;
  g.len = ri + rs;
  const float4 m = F.gmat[t.group];
  g.cs = cs;
  g.s2 = 1.0 - cs * cs;
  g.er = (double)m.x;
  g.sg = -(double)m.y * (1.0 / (2.0 * kPi * kEps0));
  g.gc = m.z > 0.0f ? 4.0 * kPi * (double)m.z * cs / kC0 : 0.0;
  g.len_c = g.len / kC0;
  return g;
}

// the scattered field of one path at frequency f (Fresnel coefficients of
// eq. (6)-(7) at the tile, Kirchhoff factor eq. (8), lobe, phase)
__device__ inline cd scat_amplitude(const ScatRec& g, const ScatField& F, int fi, double f, double inv_f) {
  const double cs = g.cs;
  const cd ec{g.er, g.sg * inv_f};
  const cd root = csqrt_mod(cd{ec.re - g.s2, ec.im});
  // te = (cs - root) / (cs + root), tm = (ecc - root) / (ecc + root), one
  // reciprocal for both denominators' squared magnitudes
  const cd ecc = cscale(ec, cs);
  const cd d1{cs + root.re, root.im}, d2 = cadd(ecc, root);
  const double n1 = d1.re * d1.re + d1.im * d1.im, n2 = d2.re * d2.re + d2.im * d2.im;
  const double inv = rcp64(n1 * n2);
  const double i1 = inv * n2, i2 = inv * n1;
  const cd a1{cs - root.re, -root.im}, a2 = csub(ecc, root);
  const cd te{(a1.re * d1.re + a1.im * d1.im) * i1, (a1.im * d1.re - a1.re * d1.im) * i1};
  const cd tm{(a2.re * d2.re + a2.im * d2.im) * i2, (a2.im * d2.re - a2.re * d2.im) * i2};
  const double gg = g.gc * f;
  const double rho2 = exp(-gg * gg);  // rho^2, eq. (8) squared
  const cd pol = cadd(cscale(te, g.wa), cscale(tm, g.wb));
  double amp = g.base * kC0 * inv_f * sqrt_nonneg(1.0 - rho2);
  if (F.atm_db) amp *= exp10(-(double)F.atm_db[fi] * g.len * (1.0 / 20.0));
  const double cyc = f * g.len_c;
  double ph = 2.0 * (cyc - floor(cyc));
  if (F.atm_deg) ph += (double)F.atm_deg[fi] * g.len * (1.0 / 180.0);
  double sn, cn;
  sincospi(ph, &sn, &cn);
  return cmul(pol, cd{amp * cn, -amp * sn});
}

__global__ __launch_bounds__(256) void k_scat_geo(ScatArgs A, ScatField F, const int32_t* __restrict__ ids,
                                                  const double* __restrict__ rec, int64_t n,
                                                  ScatRec* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = scat_rec(A, F, ids + 3 * i, rec + 2 * i);
}

// block = (Rx, Tx) pair x 256 frequencies, lane l holding frequencies
// l, l + 64, l + 128, l + 192 of the tile; its 4 waves take every 4th path of
// the pair (a path's record is wave-uniform), then add in a fixed order.
// Paths on smooth faces (rho = 1) scatter nothing and are skipped.  Each
// path's |a|^2 summed over the tile's frequencies (one wave reduction per
// path and tile) goes to part[n][tile].
constexpr int kScatLaneF = 4, kScatWaves = 4, kScatTile = 64 * kScatLaneF;
__global__ __launch_bounds__(64 * kScatWaves) void k_scat_channel(ScatField F, int Nt, int Nr,
                                                                  const int32_t* __restrict__ seg_start,
                                                                  const ScatRec* __restrict__ recs, int ntiles,
                                                                  float2* __restrict__ H64,
                                                                  double2* __restrict__ H128,
                                                                  double* __restrict__ part) {
  __shared__ double sre[kScatWaves][kScatTile], sim[kScatWaves][kScatTile];
  const int64_t seg = blockIdx.x / ntiles;
  const int tile = (int)(blockIdx.x - seg * ntiles);
  const int n0 = seg_start[seg], n1 = seg_start[seg + 1];
  if (n0 == n1) return;  // the whole block: no path for this pair
  const int q = (int)(seg / Nt), p = (int)(seg - (int64_t)q * Nt);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int fi[kScatLaneF];
  bool on[kScatLaneF];
  double f[kScatLaneF], inv_f[kScatLaneF];
  cd acc[kScatLaneF];
#pragma unroll
  for (int j = 0; j < kScatLaneF; ++j) {
    fi[j] = tile * kScatTile + 64 * j + lane;
    on[j] = fi[j] < F.Nf;
    f[j] = on[j] ? F.freq[fi[j]] : 1.0;
    inv_f[j] = 1.0 / f[j];
    acc[j] = cd{0.0, 0.0};
  }
  for (int n = n0 + wv; n < n1; n += kScatWaves) {
    const ScatRec g = recs[n];
    double ps = 0.0;
    if (g.gc != 0.0) {
#pragma unroll
      for (int j = 0; j < kScatLaneF; ++j) {
        const cd a = scat_amplitude(g, F, on[j] ? fi[j] : 0, f[j], inv_f[j]);
        if (on[j]) {
          acc[j] = cadd(acc[j], a);
          ps += a.re * a.re + a.im * a.im;
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) ps += __shfl_xor(ps, o, 64);
    }
    if (lane == 0) part[(int64_t)n * ntiles + tile] = ps;
  }
#pragma unroll
  for (int j = 0; j < kScatLaneF; ++j) {
    sre[wv][64 * j + lane] = acc[j].re;
    sim[wv][64 * j + lane] = acc[j].im;
  }
  __syncthreads();
  // thread t of the block finishes frequency t of the tile
  const int t = threadIdx.x, ft = tile * kScatTile + t;
  if (ft < F.Nf) {
    double re = sre[0][t], im = sim[0][t];
#pragma unroll
    for (int w = 1; w < kScatWaves; ++w) re += sre[w][t], im += sim[w][t];
    const int64_t o = ((int64_t)ft * Nr + q) * Nt + p;
    if (H128) {
      const double2 h = H128[o];
      H128[o] = make_double2(h.x + re, h.y + im);
    }
    if (H64) {
      const float2 h = H64[o];
      H64[o] = make_float2((float)((double)h.x + re), (float)((double)h.y + im));
    }
  }
}

// per path: delay (r_i + r_s) / c, departure Tx -> C and arrival Rx -> C as
// (azimuth, elevation) in degrees, for the per-link statistics
__global__ __launch_bounds__(256) void k_scat_aux(ScatArgs A, const int32_t* __restrict__ ids,
                                                  const double* __restrict__ rec, int64_t n, double* __restrict__ delay,
                                                  float* __restrict__ ang) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ri = rec[2 * i], rs = rec[2 * i + 1];
  const d3 C = ld3(A.tl[ids[3 * i + 2]].c), T = ld3(A.tx + 3 * ids[3 * i]), R = ld3(A.rx + 3 * ids[3 * i + 1]);
  delay[i] = (ri + rs) / kC0;
  const d3 u = (C - T) * (1.0 / ri), v = (C - R) * (1.0 / rs);
  constexpr double deg = 180.0 / kPi;
  ang[4 * i] = (float)(atan2(u.y, u.x) * deg);
  ang[4 * i + 1] = (float)(asin(fmax(-1.0, fmin(1.0, u.z))) * deg);
  ang[4 * i + 2] = (float)(atan2(v.y, v.x) * deg);
  ang[4 * i + 3] = (float)(asin(fmax(-1.0, fmin(1.0, v.z))) * deg);
}

__global__ __launch_bounds__(256) void k_scat_field(ScatField F, const ScatRec* __restrict__ recs, int64_t n,
                                                    double2* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * F.Nf) return;
  const int64_t i = e / F.Nf;
  const int fi = (int)(e - i * F.Nf);
  const ScatRec g = recs[i];
  const double f = F.freq[fi];
  const cd a = scat_amplitude(g, F, fi, f, 1.0 / f);
  out[e] = make_double2(a.re, a.im);
}

__global__ __launch_bounds__(256) void k_lobe_norm(const double* __restrict__ B, int alpha,
                                                   const double* __restrict__ ci, int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = lobe_eval(B, alpha, ci[i]);
}

ScatArgs scat_args(sbr_scat_s* d) {
  return ScatArgs{d->tiles.as<TileDev>(), d->n_tiles, d->Nt, d->Nr, d->tx.as<double>(), d->rx.as<double>()};
}

}  // namespace

// ---------------------------------------------------------------- host
std::vector<double> lobe_table(int alpha) {
  std::vector<double> C((size_t)(alpha + 1) * (alpha + 1), 0.0);  // binomials C[n][k]
  for (int n = 0; n <= alpha; ++n) {
    C[(size_t)n * (alpha + 1)] = 1.0;
    for (int k = 1; k <= n; ++k)
      C[(size_t)n * (alpha + 1) + k] = C[(size_t)(n - 1) * (alpha + 1) + k - 1] + (k < n ? C[(size_t)(n - 1) * (alpha + 1) + k] : 0.0);
  }
  auto bin = [&](int n, int k) { return C[(size_t)n * (alpha + 1) + k]; };
  std::vector<double> B((size_t)(alpha / 2 + 1) * (alpha + 1), 0.0);
  const double scale = std::ldexp(1.0, -alpha);
  for (int h = 0; 2 * h <= alpha; ++h)
    for (int m = 0; m + 2 * h <= alpha; ++m) {
      double J = 1.0 / (m + 1);
      for (int l = 2; l <= 2 * h; l += 2) J *= (double)l / (l + m + 1);
      const double az = 2.0 * kPi * bin(2 * h, h) * std::ldexp(1.0, -2 * h);
      B[(size_t)h * (alpha + 1) + m] = scale * bin(alpha, m + 2 * h) * bin(m + 2 * h, 2 * h) * az * J;
    }
  return B;
}

void build_tiles(sbr_scat_s* d, hipStream_t s) {
  sbr_scene_s* sc = d->scene;
  const int64_t T = sc->T;
  std::vector<double> tri(9 * (size_t)T);
  if (T > 0) {
    SBR_HIP(hipMemcpyAsync(tri.data(), sc->tri64.p, (size_t)T * 72, hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
  }
  // grid size m of every triangle, and the limits checked before any tile is made
  std::vector<int64_t> grid((size_t)T);
  double total = 0.0;
  for (int64_t t = 0; t < T; ++t) {
    const double* v = tri.data() + 9 * t;
    const double e1x = v[3] - v[0], e1y = v[4] - v[1], e1z = v[5] - v[2];
    const double e2x = v[6] - v[0], e2y = v[7] - v[1], e2z = v[8] - v[2];
    const double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
    const double md = std::ceil(std::sqrt(0.5 * std::sqrt(nx * nx + ny * ny + nz * nz) / d->tile_area));
    SBR_CHECK(md < 65536.0, SBR_E_UNSUPPORTED, "triangle %lld needs %g x %g tiles of %g m^2", (long long)t, md, md,
              d->tile_area);
    grid[(size_t)t] = std::max<int64_t>(1, (int64_t)md);
    total += (double)grid[(size_t)t] * (double)grid[(size_t)t];
  }
  SBR_CHECK(total < 2147483648.0 && total * d->Nt * d->Nr < 4294967296.0, SBR_E_UNSUPPORTED,
            "%.0f tiles x %d Tx x %d Rx: at most 2^31 tiles and 2^32 (tile, Tx, Rx) candidates in one call", total,
            d->Nt, d->Nr);
  std::vector<TileDev> out;
  out.reserve((size_t)total);
  for (int64_t t = 0; t < T; ++t) {
    const double* v = tri.data() + 9 * t;
    const double e1x = v[3] - v[0], e1y = v[4] - v[1], e1z = v[5] - v[2];
    const double e2x = v[6] - v[0], e2y = v[7] - v[1], e2z = v[8] - v[2];
    const double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
    const double nn = std::sqrt(nx * nx + ny * ny + nz * nz);
    const double A = 0.5 * nn;
    const int64_t m = grid[(size_t)t];
    const double ax = e1x / m, ay = e1y / m, az = e1z / m, bx = e2x / m, by = e2y / m, bz = e2z / m;
    auto P = [&](int64_t i, int64_t j, int c) {
      const double a = c == 0 ? ax : c == 1 ? ay : az, b = c == 0 ? bx : c == 1 ? by : bz;
      return v[c] + i * a + j * b;
    };
    const double dS = A / (double)(m * m);
    auto push = [&](int64_t i0, int64_t j0, int64_t i1, int64_t j1, int64_t i2, int64_t j2) {
      TileDev td{};
      for (int c = 0; c < 3; ++c) td.c[c] = (P(i0, j0, c) + P(i1, j1, c) + P(i2, j2, c)) / 3.0;
      td.n[0] = nx / nn, td.n[1] = ny / nn, td.n[2] = nz / nn;
      td.ds = dS;
      td.tri = (int32_t)t;
      td.group = sc->h_group[t];
      out.push_back(td);
    };
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < m - i; ++j) push(i, j, i + 1, j, i, j + 1);
    for (int64_t i = 0; i + 1 < m; ++i)
      for (int64_t j = 0; j < m - 1 - i; ++j) push(i + 1, j, i, j + 1, i + 1, j + 1);
  }
  d->n_tiles = (int64_t)out.size();
  d->tiles.alloc(std::max<size_t>(out.size(), 1) * sizeof(TileDev), s);
  if (!out.empty())
    SBR_HIP(hipMemcpyAsync(d->tiles.p, out.data(), out.size() * sizeof(TileDev), hipMemcpyHostToDevice, s));
  SBR_HIP(hipStreamSynchronize(s));
}

void run_scatter(sbr_scat_s* d, hipStream_t s) {
  sbr_scene_s* sc = d->scene;
  const std::vector<double> B = lobe_table(d->alpha);
  d->lobe.alloc(B.size() * 8, s);
  SBR_HIP(hipMemcpyAsync(d->lobe.p, B.data(), B.size() * 8, hipMemcpyHostToDevice, s));
  build_tiles(d, s);
  const int64_t npair = (int64_t)d->Nr * d->Nt;
  const int64_t C = d->n_tiles * npair;
  SBR_CHECK(C < (int64_t(1) << 32), SBR_E_UNSUPPORTED,
            "%lld (tile, Tx, Rx) candidates; at most 2^32 in one call", (long long)C);
  d->n_candidates = C;
  d->seg_start.alloc((size_t)(npair + 1) * 4, s);
  d->ids.alloc(4, s), d->rec.alloc(8, s);
  d->n_clear = d->n_paths = 0;
  if (C == 0) {
    fill_u32(d->seg_start.as<uint32_t>(), 0, npair + 1, s);
    return;
  }
  const ScatArgs A = scat_args(d);
  ScatScene S{sc->nodes.as<float4>(), sc->tri32.as<float4>(), sc->tri64.as<double>(), {}, sc->center[0],
              sc->center[1], sc->center[2], sc->n_bvh > 0, sc->n_big, (int)sc->n_bvh};
  for (int k = 0; k < 6; ++k) S.root[k] = sc->root_host[k];
  Buf ht, hr, clear;
  ht.alloc((size_t)d->Nt * d->n_tiles * 8, s), hr.alloc((size_t)d->Nr * d->n_tiles * 8, s);
  clear.alloc(8, s);
  fill_u32(clear.as<uint32_t>(), 0, 2, s);
  {
    ::sbr::TimedLaunch tl_("scattering", s);
    const int depth = sc->bvh_depth;
    for (int side = 0; side < 2; ++side) {
      const int Np = side ? d->Nr : d->Nt;
      const double* pts = side ? d->rx.as<double>() : d->tx.as<double>();
      double* h = side ? hr.as<double>() : ht.as<double>();
      const unsigned g = nblk((int64_t)Np * d->n_tiles, 128);
      auto* cl = clear.as<unsigned long long>();
      if (depth <= 16)
        hipLaunchKernelGGL(k_scat_side<16>, dim3(g), dim3(128), 0, s, A, S, pts, Np, 1 - side, h, cl);
      else if (depth <= 32)
        hipLaunchKernelGGL(k_scat_side<32>, dim3(g), dim3(128), 0, s, A, S, pts, Np, 1 - side, h, cl);
      else
        hipLaunchKernelGGL(k_scat_side<64>, dim3(g), dim3(128), 0, s, A, S, pts, Np, 1 - side, h, cl);
      SBR_LAUNCH_CHECK();
    }
  }
  Buf flag, pos, tot, temp;
  flag.alloc(C * 4, s), pos.alloc(C * 4, s), tot.alloc(8, s);
  temp.alloc(scan_temp_bytes(C), s);
  { ::sbr::TimedLaunch tl_("scattering", s); hipLaunchKernelGGL(k_scat_candidates, dim3(nblk(C, 256)), dim3(256), 0, s, A, C, ht.as<double>(), hr.as<double>(), flag.as<uint32_t>()); }
  SBR_LAUNCH_CHECK();
  exclusive_scan_u32(flag.as<uint32_t>(), pos.as<uint32_t>(), C, tot.as<uint32_t>(), temp.p, s);
  uint32_t n2 = 0;
  unsigned long long ncl = 0;
  SBR_HIP(hipMemcpyAsync(&n2, tot.p, 4, hipMemcpyDeviceToHost, s));
  SBR_HIP(hipMemcpyAsync(&ncl, clear.p, 8, hipMemcpyDeviceToHost, s));
  SBR_HIP(hipStreamSynchronize(s));
  d->n_clear = (int64_t)ncl;
  SBR_CHECK(n2 < (1u << 31) - 64u, SBR_E_UNSUPPORTED, "%u paths; fewer than 2^31 - 64 in one call", n2);
  d->n_paths = n2;
  if (n2 == 0) {
    fill_u32(d->seg_start.as<uint32_t>(), 0, npair + 1, s);
    return;
  }
  Buf paths, cnt;
  paths.alloc((size_t)n2 * 8, s);
  { ::sbr::TimedLaunch tl_("scattering", s); hipLaunchKernelGGL(k_scat_compact, dim3(nblk(C, 256)), dim3(256), 0, s, flag.as<uint32_t>(), pos.as<uint32_t>(), C,
                     paths.as<int64_t>()); }
  SBR_LAUNCH_CHECK();
  d->ids.alloc((size_t)n2 * 12, s);
  d->rec.alloc((size_t)n2 * 16, s);
  cnt.alloc((size_t)npair * 4, s);
  fill_u32(cnt.as<uint32_t>(), 0, npair, s);
  { ::sbr::TimedLaunch tl_("scattering", s); hipLaunchKernelGGL(k_scat_records, dim3(nblk(n2, 256)), dim3(256), 0, s, A, paths.as<int64_t>(), (int64_t)n2,
                     d->ids.as<int32_t>(), d->rec.as<double>(), cnt.as<uint32_t>()); }
  SBR_LAUNCH_CHECK();
  Buf temp2;
  temp2.alloc(scan_temp_bytes(npair), s);
  exclusive_scan_u32(cnt.as<uint32_t>(), d->seg_start.as<uint32_t>(), npair, d->seg_start.as<uint32_t>() + npair,
                     temp2.p, s);
  SBR_HIP(hipStreamSynchronize(s));
}

namespace {
// the per-path records of one polarisation pair (n_paths of them)
void scat_records(sbr_scat_s* d, const ScatField& F, Buf& recs, hipStream_t s) {
  const int64_t n = d->n_paths;
  recs.alloc((size_t)n * sizeof(ScatRec), s);
  ::sbr::TimedLaunch tl_("scattering", s);
  hipLaunchKernelGGL(k_scat_geo, dim3(nblk(n, 256)), dim3(256), 0, s, scat_args(d), F, d->ids.as<int32_t>(),
                     d->rec.as<double>(), n, recs.as<ScatRec>());
  SBR_LAUNCH_CHECK();
}
}  // namespace

void run_scat_channel(sbr_scat_s* d, const double* freq, int Nf, const float* atm_db, const float* atm_deg, int ptx,
                      int prx, float2* H64, double2* H128, hipStream_t s) {
  const int64_t npair = (int64_t)d->Nr * d->Nt;
  const int64_t np = d->n_paths;
  d->power.alloc((size_t)std::max<int64_t>(np, 1) * 8, s);
  d->have_power = true;
  if (np == 0 || Nf == 0) return;
  const int ntiles = (Nf + kScatTile - 1) / kScatTile;
  SBR_CHECK(npair * ntiles < (int64_t(1) << 31), SBR_E_UNSUPPORTED, "too many (rx, tx) pairs x frequency tiles");
  const ScatField F{freq, atm_db, atm_deg, Nf, ptx, prx, d->alpha, d->lobe.as<double>(), d->scene->gmat.as<float4>()};
  Buf recs, part;
  scat_records(d, F, recs, s);
  part.alloc((size_t)np * ntiles * 8, s);
  ::sbr::TimedLaunch tl_("scattering", s);
  hipLaunchKernelGGL(k_scat_channel, dim3((unsigned)(npair * ntiles)), dim3(64 * kScatWaves), 0, s, F, d->Nt,
                     d->Nr, d->seg_start.as<int32_t>(), recs.as<ScatRec>(), ntiles, H64, H128, part.as<double>());
  SBR_LAUNCH_CHECK();
  run_power_final(part.as<double>(), np, ntiles, Nf, d->power.as<double>(), s);
}

void run_scat_aux(sbr_scat_s* d, double* delay, float* ang, hipStream_t s) {
  const int64_t n = d->n_paths;
  if (n == 0) return;
  hipLaunchKernelGGL(k_scat_aux, dim3(nblk(n, 256)), dim3(256), 0, s, scat_args(d), d->ids.as<int32_t>(),
                     d->rec.as<double>(), n, delay, ang);
  SBR_LAUNCH_CHECK();
}

void run_scat_field(sbr_scat_s* d, const double* freq, int Nf, const float* atm_db, const float* atm_deg, int ptx,
                    int prx, double2* out, hipStream_t s) {
  const int64_t n = d->n_paths;
  if (n == 0 || Nf == 0) return;
  const ScatField F{freq, atm_db, atm_deg, Nf, ptx, prx, d->alpha, d->lobe.as<double>(), d->scene->gmat.as<float4>()};
  Buf recs;
  scat_records(d, F, recs, s);
  { ::sbr::TimedLaunch tl_("scattering", s); hipLaunchKernelGGL(k_scat_field, dim3(nblk(n * Nf, 256)), dim3(256), 0, s, F, recs.as<ScatRec>(), n, out); }
  SBR_LAUNCH_CHECK();
}

void run_lobe_norm(int alpha, const double* cos_i, int64_t n, double* out, hipStream_t s) {
  if (n == 0) return;
  const std::vector<double> B = lobe_table(alpha);
  Buf b;
  b.alloc(B.size() * 8, s);
  SBR_HIP(hipMemcpyAsync(b.p, B.data(), B.size() * 8, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_lobe_norm, dim3(nblk(n, 256)), dim3(256), 0, s, b.as<double>(), alpha, cos_i, n, out);
  SBR_LAUNCH_CHECK();
  SBR_HIP(hipStreamSynchronize(s));  // b is freed on return
}

}  // namespace sbr
