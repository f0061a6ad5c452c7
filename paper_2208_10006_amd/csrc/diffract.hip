// diffract.hip -- first-order edge diffraction (Sec. II-A-2 and Fig. B(b) name
// it among the propagation mechanisms, Table I's results include it; the
// paper gives no diffraction coefficient).
//
// Reading: the uniform theory of diffraction of Kouyoumjian and Pathak for a
// straight wedge, its two reflection-type terms weighted by the faces'
// Fresnel coefficients and Kirchhoff roughness factors (Luebbers' form for
// lossy wedges).
//  * Wedges: triangle edges shared by exactly two triangles of different face
//    groups whose planes are not parallel.  The solid fills the smaller
//    sector (alpha < pi) between the two faces, the field the exterior sector
//    n pi = 2 pi - alpha.  An edge lying on a triangle of a third face group
//    (both ends within 1e-9 (1 + max |coordinate|) of its plane, the edge's
//    midpoint inside it with the 1e-9 barycentric margin) is where a solid
//    rests on another surface and is not a wedge.  Face 0 is the triangle of
//    lower index; angles run from face 0 through the exterior.  Wedges are
//    numbered by (lower triangle, its local edge i = vertex i -> vertex i + 1).
//  * A path Tx -> Q -> Rx exists when Tx and Rx lie strictly inside the
//    exterior sector, the diffraction point Q -- on Keller's cone: the edge
//    coordinates of Tx and Rx divided in the ratio of their distances from
//    the edge line -- lies strictly inside the edge, and neither leg crosses
//    a triangle outside the wedge's two face groups.
//  * Field: E^d = E^i(Q) D A e^{-jks} with E^i(Q) = (lambda / 4 pi)
//    e^{-jks'} / s' along the Tx polarisation, the dyadic
//    D = -beta0' beta0 D_s - phi' phi D_h in edge-fixed unit vectors and
//    A = sqrt(s' / (s (s + s'))).
//
// Pipeline: a wedge table built on the host once per scene (exact vertex
// matching) -> the sector and edge tests per (wedge, Rx, Tx) candidate ->
// ordered compaction -> both legs against the BVH with exact FP64 triangle
// tests -> ordered compaction -> a stable sort of the paths by (Rx, Tx) pair
// -> records and a CSR per pair.  Candidates are numbered wedge-major so that
// the lanes of a wave test legs from neighbouring Tx elements to nearly the
// same point of one edge, which traverse the BVH together.  The
// field kernel sums each pair's paths per frequency in a fixed order and adds
// them to H.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <vector>

#include "occlusion.hpp"
#include "sbr_device.hpp"
#include "sbr_internal.hpp"

namespace sbr {

namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

struct DiffArgs {
  const WedgeDev* wd;
  int64_t W;
  int Nt, Nr;
  const double* tx;
  const double* rx;
};

// the scene fields leg_blocked reads
struct DiffScene {
  const float4* nodes;
  const float4* tri32;
  const double* tri64;
  float root[6];
  double cx, cy, cz;
  int has_bvh, n_big, big_off;
};

// edge coordinate, distance from the edge line and angle from face 0 through
// the exterior (in [0, 2 pi)) of point P
__device__ inline void edge_coords(const WedgeDev& w, d3 P, double& z, double& rho, double& phi) {
  const d3 e = ld3(w.e);
  const d3 r = P - ld3(w.a);
  z = dot(r, e);
  const d3 v = r - e * z;
  rho = sqrt(dot(v, v));
  phi = atan2(dot(v, ld3(w.n0)), dot(v, ld3(w.t0)));
  if (phi < 0.0) phi += 2.0 * kPi;
}

// candidate c = ((q Nt + p) W + wedge): its indices and, when it passes the
// sector and edge tests, the diffraction point and the two angles
// candidate c = ((wedge Nr + q) Nt + p)
__device__ inline bool diff_geometry(const DiffArgs& A, int64_t c, int& p, int& q, int& wi, d3& Q, double& ft,
                                     double& fr) {
  p = (int)(c % A.Nt);
  const int64_t wq = c / A.Nt;
  q = (int)(wq % A.Nr);
  wi = (int)(wq / A.Nr);
  const WedgeDev w = A.wd[wi];
  const d3 T = ld3(A.tx + 3 * p), R = ld3(A.rx + 3 * q);
  double zt, rt, zr, rr;
  edge_coords(w, T, zt, rt, ft);
  edge_coords(w, R, zr, rr, fr);
  const double lim = w.nw * kPi;
  if (!(rt > 0.0 && rr > 0.0)) return false;
  if (!(ft > 0.0 && ft < lim && fr > 0.0 && fr < lim)) return false;
  const double zq = zt + (zr - zt) * rt / (rt + rr);
  if (!(zq > 0.0 && zq < w.len)) return false;
  Q = ld3(w.a) + ld3(w.e) * zq;
  return true;
}

__global__ __launch_bounds__(256) void k_diff_candidates(DiffArgs A, int64_t C, uint32_t* __restrict__ flag) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  int p, q, wi;
  d3 Q;
  double ft, fr;
  flag[c] = diff_geometry(A, c, p, q, wi, Q, ft, fr) ? 1u : 0u;
}

// dst[pos[i]] = src ? src[i] : i for every flagged i (pos: exclusive scan of flag)
__global__ __launch_bounds__(256) void k_diff_compact(const uint32_t* __restrict__ flag,
                                                      const uint32_t* __restrict__ pos, int64_t n,
                                                      const int64_t* __restrict__ src, int64_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  dst[pos[i]] = src ? src[i] : i;
}

// both legs of each geometric candidate against the scene (two waves per
// block, each lane's traversal stack in LDS)
template <int STACK>
__global__ __launch_bounds__(128) void k_diff_legs(DiffArgs A, DiffScene S, const int64_t* __restrict__ cand,
                                                   int64_t n, uint32_t* __restrict__ flag) {
  __shared__ int32_t stack_mem[2][STACK][kWave];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t* stk = &stack_mem[wv][0][lane];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p, q, wi;
  d3 Q;
  double ft, fr;
  bool ok = diff_geometry(A, cand[i], p, q, wi, Q, ft, fr);
  if (ok) {
    const WedgeDev w = A.wd[wi];
    const d3 T = ld3(A.tx + 3 * p), R = ld3(A.rx + 3 * q);
    ok = !leg_blocked<STACK>(S, stk, T, Q, w.g0, w.gn) && !leg_blocked<STACK>(S, stk, Q, R, w.g0, w.gn);
  }
  flag[i] = ok ? 1u : 0u;
}

// ids[i] = (tx, rx, wedge), rec[i] = (Q xyz, s', s, beta0, phi', phi); paths per (Rx, Tx) pair counted
// the (Rx, Tx) pair of each path, for the sort into pair order
__global__ __launch_bounds__(256) void k_diff_pair_keys(DiffArgs A, const int64_t* __restrict__ path, int64_t n,
                                                        uint64_t* __restrict__ key, uint32_t* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t c = path[i];
  const int64_t wq = c / A.Nt;
  key[i] = (uint64_t)(wq % A.Nr) * (uint64_t)A.Nt + (uint64_t)(c - wq * A.Nt);
  val[i] = (uint32_t)i;
}

// record i is path order[i]
__global__ __launch_bounds__(256) void k_diff_records(DiffArgs A, const int64_t* __restrict__ path,
                                                      const uint32_t* __restrict__ order, int64_t n,
                                                      int32_t* __restrict__ ids, double* __restrict__ rec,
                                                      uint32_t* __restrict__ pair_count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p, q, wi;
  d3 Q;
  double ft, fr;
  diff_geometry(A, path[order[i]], p, q, wi, Q, ft, fr);
  const WedgeDev w = A.wd[wi];
  const d3 T = ld3(A.tx + 3 * p), R = ld3(A.rx + 3 * q);
  const d3 dt = Q - T, dr = R - Q;
  const double sp = sqrt(dot(dt, dt)), s = sqrt(dot(dr, dr));
  const double cb = fmin(1.0, fmax(-1.0, dot(dt, ld3(w.e)) / sp));
  ids[3 * i] = p, ids[3 * i + 1] = q, ids[3 * i + 2] = wi;
  double* r = rec + 8 * i;
  r[0] = Q.x, r[1] = Q.y, r[2] = Q.z, r[3] = sp, r[4] = s, r[5] = acos(cb), r[6] = ft, r[7] = fr;
  atomicAdd(&pair_count[(int64_t)q * A.Nt + p], 1u);
}

// ---------------------------------------------------------------- field
// Kouyoumjian-Pathak transition function F(X) = 2j sqrt(X) e^{jX} int_{sqrt X}^inf e^{-j t^2} dt.
//  X < 5: the tail as (sqrt(pi)/2) e^{-j pi/4} - G(u), u = sqrt(X), with the
//         power series G(u) = sum_k (-j)^k u^{2k+1} / (k! (2k+1));
//  5 <= X < 80: Laplace's continued fraction of the complementary error
//         function, F = u e^{j pi/4} / (w + (1/2) / (w + (2/2) / (w + (3/2) / ...))),
//         w = e^{j pi/4} u, evaluated from the bottom (60, 40 or 20 levels:
//         below 1e-14 relative for X >= 5, 8, 20);
//  X >= 80: the asymptotic series from repeated integration by parts,
//         F ~ sum_n (2n - 1)!! (j / (2X))^n, twelve terms (the first omitted
//         term is below 7e-15 relative at X = 80).
__device__ inline cd utd_transition(double X) {
  if (!(X > 0.0)) return cd{0.0, 0.0};
  if (X >= 80.0) {
    const double y = 0.5 / X, y2 = y * y;
    const double re = 1.0 + y2 * (-3.0 + y2 * (105.0 + y2 * (-10395.0 + y2 * (2027025.0 + y2 * -654729075.0))));
    const double im =
        y * (1.0 + y2 * (-15.0 + y2 * (945.0 + y2 * (-135135.0 + y2 * (34459425.0 + y2 * -13749310575.0)))));
    return cd{re, im};
  }
  const double u = sqrt(X);
  const double r2 = 0.70710678118654752440;  // cos(pi/4)
  if (X < 5.0) {
    cd t{u, 0.0};
    cd G = t;
    for (int k = 1; k < 80; ++k) {
      const double m = X / k;
      t = cd{t.im * m, -t.re * m};  // t *= -j X / k
      const double g = 1.0 / (2 * k + 1);
      G = cd{G.re + t.re * g, G.im + t.im * g};
      if (k > X && fabs(t.re) + fabs(t.im) < 1e-18 * (fabs(G.re) + fabs(G.im))) break;
    }
    const double h = 0.88622692545275801365 * r2;  // (sqrt(pi) / 2) cos(pi/4)
    const cd tail{h - G.re, -h - G.im};
    double sx, cx;
    sincos(X, &sx, &cx);
    const cd v = cmul(cd{cx, sx}, tail);
    return cd{-2.0 * u * v.im, 2.0 * u * v.re};
  }
  const int N = X < 8.0 ? 60 : (X < 20.0 ? 40 : 20);
  const cd w{u * r2, u * r2};
  cd t = w;
  for (int m = N; m >= 1; --m) t = cadd(w, cdiv_mod(cd{0.5 * m, 0.0}, t));
  return cdiv_mod(w, t);
}

// One term of the coefficients, cot((pi + sign beta) / (2n)) F(k L a^{sign}(beta)),
// a^{+-}(beta) = 2 cos^2((2 n pi N - beta) / 2), N the integer nearest
// (beta +- pi) / (2 pi n): the cotangent and X / f = (2 pi / c) L a, which
// depend on the path only.
__device__ inline void utd_term_geo(double beta, double nw, double L, double sign, double& ct, double& xf) {
  const double N = rint((beta + sign * kPi) / (2.0 * kPi * nw));
  const double c = cos((2.0 * nw * kPi * N - beta) * 0.5);
  ct = 1.0 / tan((kPi + sign * beta) / (2.0 * nw));
  xf = (2.0 * kPi / kC0) * L * 2.0 * c * c;
}

// TE and TM reflection coefficients of one face times its roughness factor
// (eq. (6)-(8)), from the face's record: eps = er + j sg / f, cos and sin^2 of
// the incidence angle, roughness exponent g = gc f (0 on smooth faces); one
// reciprocal serves both quotients.
struct FaceRec {
  double er, sg, cs, s2, gc;
};
__device__ inline void face_reflection(const FaceRec& m, double f, double inv_f, cd& te, cd& tm) {
  const double cs = m.cs;
  const cd ec{m.er, m.sg * inv_f};
  const cd root = csqrt_mod(cd{ec.re - m.s2, ec.im});
  const cd ecc = cscale(ec, cs);
  const cd d1{cs + root.re, root.im}, d2 = cadd(ecc, root);
  const double n1 = d1.re * d1.re + d1.im * d1.im, n2 = d2.re * d2.re + d2.im * d2.im;
  const double inv = rcp64(n1 * n2);
  double i1 = inv * n2, i2 = inv * n1;
  if (m.gc != 0.0) {
    const double g = m.gc * f;
    const double rho = exp(-0.5 * g * g);
    i1 *= rho, i2 *= rho;
  }
  const cd a1{cs - root.re, -root.im}, a2 = csub(ecc, root);
  te = cd{(a1.re * d1.re + a1.im * d1.im) * i1, (a1.im * d1.re - a1.re * d1.im) * i1};
  tm = cd{(a2.re * d2.re + a2.im * d2.im) * i2, (a2.im * d2.re - a2.re * d2.im) * i2};
}

// theta-hat (pol 0) or phi-hat (pol 1) of direction u
__device__ inline d3 pol_vec(d3 u, int pol) {
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

struct DiffField {
  const double* freq;
  const float* atm_db;
  const float* atm_deg;
  int Nf, ptx, prx;
  const float4* gmat;
};

// frequency-independent part of one path for one polarisation pair, written
// once per call by k_diff_geo and read by every frequency
struct DiffRec {
  double wb, wp;       // -(E . beta0')(beta0 . e_rx) and -(E . phi')(phi . e_rx)
  FaceRec f0, fn;      // the two faces at their true incidence angles
  double ct[4], xf[4]; // the four terms: cotangent and X / f
  double magc;         // 1 / (2 n sqrt(2 pi k) sin beta0) times sqrt(f)
  double ampc;         // (c / 4 pi) sqrt(s' / (s (s + s'))) / s', times 1 / f
  double len, len_c;   // s' + s and (s' + s) / c
};

__device__ inline FaceRec face_rec(float4 m, double cs) {
  return FaceRec{(double)m.x, -(double)m.y * (1.0 / (2.0 * kPi * kEps0)), cs, 1.0 - cs * cs,
                 m.z > 0.0f ? 4.0 * kPi * (double)m.z * cs / kC0 : 0.0};
}

__device__ inline DiffRec diff_rec(const DiffArgs& A, const DiffField& F, const int32_t* ids, const double* rec) {
  DiffRec g;
  const int p = ids[0], q = ids[1], wi = ids[2];
  const WedgeDev w = A.wd[wi];
  const d3 Q = mk3(rec[0], rec[1], rec[2]);
  const d3 T = ld3(A.tx + 3 * p), R = ld3(A.rx + 3 * q);
  const double sp = rec[3], s = rec[4], b0 = rec[5], phip = rec[6], phi = rec[7], nw = w.nw;
  const d3 e = ld3(w.e);
  const d3 ih = (Q - T) * (1.0 / sp), sh = (R - Q) * (1.0 / s);
  d3 php = cross(e, ih) * -1.0;
  php = php * (1.0 / sqrt(dot(php, php)));
  const d3 bp = cross(php, ih);
  d3 ph = cross(e, sh);
  ph = ph * (1.0 / sqrt(dot(ph, ph)));
  const d3 bh = cross(ph, sh);
  const d3 Ei = pol_vec(ih, F.ptx), Er = pol_vec(sh, F.prx);
  g.wb = -dot(Ei, bp) * dot(bh, Er);
  g.wp = -dot(Ei, php) * dot(ph, Er);
  const double sb = sin(b0);
  g.f0 = face_rec(F.gmat[w.g0], sb * fabs(sin(phip)));
  g.fn = face_rec(F.gmat[w.gn], sb * fabs(sin(nw * kPi - phi)));
  const double L = s * sp * sb * sb / (s + sp);
  const double bm = phi - phip, bs = phi + phip;
  utd_term_geo(bm, nw, L, 1.0, g.ct[0], g.xf[0]);
  utd_term_geo(bm, nw, L, -1.0, g.ct[1], g.xf[1]);
  utd_term_geo(bs, nw, L, -1.0, g.ct[2], g.xf[2]);
  utd_term_geo(bs, nw, L, 1.0, g.ct[3], g.xf[3]);
  g.magc = 1.0 / (2.0 * nw * sqrt(2.0 * kPi * (2.0 * kPi / kC0)) * sb);
  g.ampc = (kC0 / (4.0 * kPi)) / sp * sqrt(sp / (s * (s + sp)));
  g.len = s + sp;
  g.len_c = g.len / kC0;
  return g;
}

// received diffracted field of one path at frequency f (rsf = 1 / sqrt(f))
__device__ inline cd diff_amplitude(const DiffRec& g, const DiffField& F, int fi, double f, double inv_f,
                                    double rsf) {
  cd r0te, r0tm, rnte, rntm;
  face_reflection(g.f0, f, inv_f, r0te, r0tm);
  face_reflection(g.fn, f, inv_f, rnte, rntm);
  const cd t12 = cadd(cscale(utd_transition(f * g.xf[0]), g.ct[0]), cscale(utd_transition(f * g.xf[1]), g.ct[1]));
  const cd t3 = cscale(utd_transition(f * g.xf[2]), g.ct[2]), t4 = cscale(utd_transition(f * g.xf[3]), g.ct[3]);
  const cd ds = cadd(t12, cadd(cmul(r0te, t3), cmul(rnte, t4)));
  const cd dh = cadd(t12, cadd(cmul(r0tm, t3), cmul(rntm, t4)));
  // -e^{-j pi/4} / (2 n sqrt(2 pi k) sin beta0)
  const double r2 = 0.70710678118654752440;
  const double mag = g.magc * rsf;
  const cd pre{-r2 * mag, r2 * mag};
  // E^d . e_rx = -D_s (E^i . beta0') (beta0 . e_rx) - D_h (E^i . phi') (phi . e_rx)
  const cd pol = cmul(pre, cadd(cscale(ds, g.wb), cscale(dh, g.wp)));
  double amp = g.ampc * inv_f;
  if (F.atm_db) amp *= exp10(-(double)F.atm_db[fi] * g.len * (1.0 / 20.0));
  const double cyc = f * g.len_c;
  double ph = 2.0 * (cyc - floor(cyc));  // in units of pi
  if (F.atm_deg) ph += (double)F.atm_deg[fi] * g.len * (1.0 / 180.0);
  double sn, cn;
  sincospi(ph, &sn, &cn);
  return cmul(pol, cd{amp * cn, -amp * sn});
}

__global__ __launch_bounds__(256) void k_diff_geo(DiffArgs A, DiffField F, const int32_t* __restrict__ ids,
                                                  const double* __restrict__ rec, int64_t n,
                                                  DiffRec* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = diff_rec(A, F, ids + 3 * i, rec + 8 * i);
}

// One block per ((Rx, Tx) pair, 256 frequencies), lane l holding frequencies
// l, l + 64, l + 128, l + 192 of the tile; the four waves take every fourth
// path of the pair (a path's record is wave-uniform), each sums its paths in
// order and the wave sums are added in wave order; the result is added to H.
// Each path's |a|^2 summed over the tile's frequencies goes to part[n][tile].
constexpr int kDiffLaneF = 4, kDiffWaves = 4, kDiffTile = 64 * kDiffLaneF;
__global__ __launch_bounds__(64 * kDiffWaves) void k_diff_channel(DiffField F, int Nt, int Nr,
                                                                  const int32_t* __restrict__ seg_start,
                                                                  const DiffRec* __restrict__ recs, int ntiles,
                                                                  float2* __restrict__ H64,
                                                                  double2* __restrict__ H128,
                                                                  double* __restrict__ part) {
  __shared__ double sre[kDiffWaves][kDiffTile], sim[kDiffWaves][kDiffTile];
  const int64_t seg = blockIdx.x / ntiles;
  const int tile = (int)(blockIdx.x - seg * ntiles);
  const int n0 = seg_start[seg], n1 = seg_start[seg + 1];
  if (n0 == n1) return;  // the whole block: no path for this pair
  const int q = (int)(seg / Nt), p = (int)(seg - (int64_t)q * Nt);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int fi[kDiffLaneF];
  bool on[kDiffLaneF];
  double f[kDiffLaneF], inv_f[kDiffLaneF], rsf[kDiffLaneF];
  cd acc[kDiffLaneF];
#pragma unroll
  for (int j = 0; j < kDiffLaneF; ++j) {
    fi[j] = tile * kDiffTile + 64 * j + lane;
    on[j] = fi[j] < F.Nf;
    f[j] = on[j] ? F.freq[fi[j]] : 1.0;
    inv_f[j] = 1.0 / f[j];
    rsf[j] = 1.0 / sqrt(f[j]);
    acc[j] = cd{0.0, 0.0};
  }
  for (int n = n0 + wv; n < n1; n += kDiffWaves) {
    const DiffRec g = recs[n];
    double ps = 0.0;
#pragma unroll
    for (int j = 0; j < kDiffLaneF; ++j) {
      const cd a = diff_amplitude(g, F, on[j] ? fi[j] : 0, f[j], inv_f[j], rsf[j]);
      if (on[j]) {
        acc[j] = cadd(acc[j], a);
        ps += a.re * a.re + a.im * a.im;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ps += __shfl_xor(ps, o, 64);
    if (lane == 0) part[(int64_t)n * ntiles + tile] = ps;
  }
#pragma unroll
  for (int j = 0; j < kDiffLaneF; ++j) {
    sre[wv][64 * j + lane] = acc[j].re;
    sim[wv][64 * j + lane] = acc[j].im;
  }
  __syncthreads();
  // thread t of the block finishes frequency t of the tile
  const int t = threadIdx.x, ft = tile * kDiffTile + t;
  if (ft < F.Nf) {
    double re = sre[0][t], im = sim[0][t];
#pragma unroll
    for (int w = 1; w < kDiffWaves; ++w) re += sre[w][t], im += sim[w][t];
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

// per path: delay (s' + s) / c, departure Tx -> Q and arrival Rx -> Q as
// (azimuth, elevation) in degrees, for the per-link statistics
__global__ __launch_bounds__(256) void k_diff_aux(DiffArgs A, const int32_t* __restrict__ ids,
                                                  const double* __restrict__ rec, int64_t n, double* __restrict__ delay,
                                                  float* __restrict__ ang) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* r = rec + 8 * i;
  const d3 Q = ld3(r), T = ld3(A.tx + 3 * ids[3 * i]), R = ld3(A.rx + 3 * ids[3 * i + 1]);
  delay[i] = (r[3] + r[4]) / kC0;
  const d3 u = (Q - T) * (1.0 / r[3]), v = (Q - R) * (1.0 / r[4]);
  constexpr double deg = 180.0 / kPi;
  ang[4 * i] = (float)(atan2(u.y, u.x) * deg);
  ang[4 * i + 1] = (float)(asin(fmax(-1.0, fmin(1.0, u.z))) * deg);
  ang[4 * i + 2] = (float)(atan2(v.y, v.x) * deg);
  ang[4 * i + 3] = (float)(asin(fmax(-1.0, fmin(1.0, v.z))) * deg);
}

// a[n][f] of every path (diagnostic and parity output)
__global__ __launch_bounds__(256) void k_diff_field(DiffField F, const DiffRec* __restrict__ recs, int64_t n,
                                                    double2* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * F.Nf) return;
  const int64_t i = e / F.Nf;
  const int fi = (int)(e - i * F.Nf);
  const DiffRec g = recs[i];
  const double f = F.freq[fi];
  const cd a = diff_amplitude(g, F, fi, f, 1.0 / f, 1.0 / sqrt(f));
  out[e] = make_double2(a.re, a.im);
}

__global__ __launch_bounds__(256) void k_utd_transition(const double* __restrict__ X, int64_t n,
                                                        double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const cd v = utd_transition(X[i]);
  out[i] = make_double2(v.re, v.im);
}

using V3 = std::array<double, 3>;
inline V3 vsub(const V3& a, const V3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
inline double vdot(const V3& a, const V3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline V3 vcross(const V3& a, const V3& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
inline V3 vscale(const V3& a, double s) { return {a[0] * s, a[1] * s, a[2] * s}; }
inline V3 vunit(const V3& a) { return vscale(a, 1.0 / std::sqrt(vdot(a, a))); }

DiffArgs diff_args(sbr_diff_s* d) {
  sbr_scene_s* sc = d->scene;
  return DiffArgs{sc->wedges.as<WedgeDev>(), sc->n_wedges, d->Nt, d->Nr, d->tx.as<double>(), d->rx.as<double>()};
}

DiffField diff_field_args(sbr_diff_s* d, const double* freq, int Nf, const float* atm_db, const float* atm_deg,
                          int ptx, int prx) {
  return DiffField{freq, atm_db, atm_deg, Nf, ptx, prx, d->scene->gmat.as<float4>()};
}

}  // namespace

// ---------------------------------------------------------------- host
void scene_wedges(sbr_scene_s* sc, hipStream_t s) {
  std::lock_guard<std::mutex> lk(sc->wedge_mu);
  if (sc->have_wedges) return;
  const int64_t T = sc->T;
  std::vector<double> tri(9 * (size_t)T);
  if (T > 0) {
    SBR_HIP(hipMemcpyAsync(tri.data(), sc->tri64.p, (size_t)T * 72, hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
  }
  auto vert = [&](int64_t t, int i) { return V3{tri[9 * t + 3 * i], tri[9 * t + 3 * i + 1], tri[9 * t + 3 * i + 2]}; };
  // the triangles (and their local edge index) on each undirected edge,
  // matched by exact vertex coordinates: (edge, triangle, edge index) sorted
  struct EdgeRef {
    V3 a, b;
    int64_t t;
    int i;
  };
  std::vector<EdgeRef> edges;
  edges.reserve(3 * (size_t)T);
  for (int64_t t = 0; t < T; ++t)
    for (int i = 0; i < 3; ++i) {
      const V3 a = vert(t, i), b = vert(t, (i + 1) % 3);
      edges.push_back(a < b ? EdgeRef{a, b, t, i} : EdgeRef{b, a, t, i});
    }
  std::sort(edges.begin(), edges.end(), [](const EdgeRef& x, const EdgeRef& y) {
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    return x.t != y.t ? x.t < y.t : x.i < y.i;
  });
  // per triangle: unit normal, plane offset and bounding box (the test of an
  // edge lying on another surface)
  std::vector<V3> tn((size_t)T);
  std::vector<double> tc((size_t)T), tlo(3 * (size_t)T), thi(3 * (size_t)T);
  for (int64_t t = 0; t < T; ++t) {
    tn[t] = vunit(vcross(vsub(vert(t, 1), vert(t, 0)), vsub(vert(t, 2), vert(t, 0))));
    tc[t] = vdot(tn[t], vert(t, 0));
    for (int c = 0; c < 3; ++c) {
      tlo[3 * t + c] = std::min({tri[9 * t + c], tri[9 * t + 3 + c], tri[9 * t + 6 + c]});
      thi[3 * t + c] = std::max({tri[9 * t + c], tri[9 * t + 3 + c], tri[9 * t + 6 + c]});
    }
  }
  // A uniform grid over the triangles' boxes, each inflated by the largest
  // tolerance a query can use (1e-9 (1 + the largest coordinate)), so that
  // the cell of an edge's midpoint lists every triangle the test below can
  // accept; the test itself is unchanged.
  double glo[3] = {INFINITY, INFINITY, INFINITY}, ghi[3] = {-INFINITY, -INFINITY, -INFINITY}, amax = 0.0;
  for (int64_t t = 0; t < T; ++t)
    for (int c = 0; c < 3; ++c) {
      glo[c] = std::min(glo[c], tlo[3 * t + c]), ghi[c] = std::max(ghi[c], thi[3 * t + c]);
      amax = std::max({amax, std::fabs(tlo[3 * t + c]), std::fabs(thi[3 * t + c])});
    }
  const double geps = 1e-9 * (1.0 + amax) * 1.0000001;
  const int G = T > 0 ? (int)std::min<int64_t>(64, std::max<int64_t>(1, (int64_t)std::cbrt((double)T) * 2)) : 1;
  double cell[3];
  for (int c = 0; c < 3; ++c) cell[c] = T > 0 && ghi[c] > glo[c] ? (ghi[c] - glo[c]) / G : 1.0;
  auto cell_of = [&](double v, int c) {
    const double f = (v - glo[c]) / cell[c];
    return f <= 0.0 ? 0 : f >= G - 1 ? G - 1 : (int)f;
  };
  std::vector<std::vector<int32_t>> grid_tris((size_t)G * G * G);
  for (int64_t t = 0; t < T; ++t) {
    int lo[3], hi[3];
    for (int c = 0; c < 3; ++c) lo[c] = cell_of(tlo[3 * t + c] - geps, c), hi[c] = cell_of(thi[3 * t + c] + geps, c);
    for (int x = lo[0]; x <= hi[0]; ++x)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int z = lo[2]; z <= hi[2]; ++z) grid_tris[((size_t)x * G + y) * G + z].push_back((int32_t)t);
  }
  auto covered = [&](const V3& a, const V3& b, int ga, int gb) {
    const double eps =
        1e-9 * (1.0 + std::max({std::fabs(a[0]), std::fabs(a[1]), std::fabs(a[2]), std::fabs(b[0]), std::fabs(b[1]),
                                std::fabs(b[2])}));
    const V3 m{0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1]), 0.5 * (a[2] + b[2])};
    for (const int32_t t : grid_tris[((size_t)cell_of(m[0], 0) * G + cell_of(m[1], 1)) * G + cell_of(m[2], 2)]) {
      const int g = sc->h_group[t];
      if (g == ga || g == gb) continue;
      bool box = true;
      for (int c = 0; c < 3; ++c) box = box && m[c] >= tlo[3 * t + c] - eps && m[c] <= thi[3 * t + c] + eps;
      if (!box) continue;
      if (std::fabs(vdot(tn[t], a) - tc[t]) > eps || std::fabs(vdot(tn[t], b) - tc[t]) > eps) continue;
      const V3 v0 = vert(t, 0), v1 = vert(t, 1), v2 = vert(t, 2);
      const double area = vdot(tn[t], vcross(vsub(v1, v0), vsub(v2, v0)));
      const double w0 = vdot(tn[t], vcross(vsub(v1, v0), vsub(m, v0)));
      const double w1 = vdot(tn[t], vcross(vsub(v2, v1), vsub(m, v1)));
      const double w2 = vdot(tn[t], vcross(vsub(v0, v2), vsub(m, v2)));
      if (std::min({w0, w1, w2}) / area >= -1e-9) return true;
    }
    return false;
  };
  std::vector<std::pair<std::pair<int64_t, int>, WedgeDev>> out;
  for (size_t e0 = 0; e0 < edges.size();) {
    size_t e1 = e0 + 1;
    while (e1 < edges.size() && edges[e1].a == edges[e0].a && edges[e1].b == edges[e0].b) ++e1;
    const size_t first = e0, count = e1 - e0;
    e0 = e1;
    if (count != 2) continue;
    const int64_t ta = edges[first].t, tb = edges[first + 1].t;
    const int ia = edges[first].i, ib = edges[first + 1].i;
    if (sc->h_group[ta] == sc->h_group[tb]) continue;
    const V3 na = vunit(vcross(vsub(vert(ta, 1), vert(ta, 0)), vsub(vert(ta, 2), vert(ta, 0))));
    const V3 nb = vunit(vcross(vsub(vert(tb, 1), vert(tb, 0)), vsub(vert(tb, 2), vert(tb, 0))));
    const V3 cr = vcross(na, nb);
    if (std::sqrt(vdot(cr, cr)) < 1e-9) continue;
    const V3 a = edges[first].a, b = edges[first].b;
    const V3 ab = vsub(b, a);
    const double len = std::sqrt(vdot(ab, ab));
    const V3 e = vscale(ab, 1.0 / len);
    const V3 ca = vsub(vert(ta, (ia + 2) % 3), a), cb = vsub(vert(tb, (ib + 2) % 3), a);
    const V3 t0 = vunit(vsub(ca, vscale(e, vdot(ca, e))));
    const V3 t1 = vunit(vsub(cb, vscale(e, vdot(cb, e))));
    V3 n0 = vcross(e, t0);
    if (vdot(n0, t1) > 0.0) n0 = vscale(n0, -1.0);
    const double alpha = std::acos(std::max(-1.0, std::min(1.0, vdot(t0, t1))));
    if (covered(a, b, sc->h_group[ta], sc->h_group[tb])) continue;
    WedgeDev w{};
    for (int c = 0; c < 3; ++c) w.a[c] = a[c], w.e[c] = e[c], w.t0[c] = t0[c], w.n0[c] = n0[c];
    w.len = len;
    w.nw = 2.0 - alpha / kPi;
    w.g0 = sc->h_group[ta];
    w.gn = sc->h_group[tb];
    out.push_back({{ta, ia}, w});
  }
  std::sort(out.begin(), out.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
  std::vector<WedgeDev> host(out.size());
  for (size_t i = 0; i < out.size(); ++i) host[i] = out[i].second;
  sc->n_wedges = (int64_t)host.size();
  sc->wedges.alloc(std::max<size_t>(host.size(), 1) * sizeof(WedgeDev), s);
  if (!host.empty())
    SBR_HIP(hipMemcpyAsync(sc->wedges.p, host.data(), host.size() * sizeof(WedgeDev), hipMemcpyHostToDevice, s));
  SBR_HIP(hipStreamSynchronize(s));
  sc->have_wedges = true;
}

void run_diffract(sbr_diff_s* d, hipStream_t s) {
  sbr_scene_s* sc = d->scene;
  scene_wedges(sc, s);
  const int64_t W = sc->n_wedges;
  const int64_t npair = (int64_t)d->Nr * d->Nt;
  const int64_t C = W * npair;
  SBR_CHECK(C < (int64_t(1) << 32), SBR_E_UNSUPPORTED,
            "%lld (wedge, Tx, Rx) candidates; at most 2^32 in one call", (long long)C);
  d->n_candidates = C;
  d->seg_start.alloc((size_t)(npair + 1) * 4, s);
  d->ids.alloc(4, s), d->rec.alloc(8, s);
  d->n_geometric = d->n_paths = 0;
  if (C == 0) {
    fill_u32(d->seg_start.as<uint32_t>(), 0, npair + 1, s);
    return;
  }
  const DiffArgs A = diff_args(d);
  Buf flag, pos, tot, temp;
  flag.alloc(C * 4, s), pos.alloc(C * 4, s), tot.alloc(8, s);
  temp.alloc(scan_temp_bytes(C), s);
  { ::sbr::TimedLaunch tl_("diffraction", s); hipLaunchKernelGGL(k_diff_candidates, dim3(nblk(C, 256)), dim3(256), 0, s, A, C, flag.as<uint32_t>()); }
  SBR_LAUNCH_CHECK();
  exclusive_scan_u32(flag.as<uint32_t>(), pos.as<uint32_t>(), C, tot.as<uint32_t>(), temp.p, s);
  uint32_t n1 = 0;
  SBR_HIP(hipMemcpyAsync(&n1, tot.p, 4, hipMemcpyDeviceToHost, s));
  SBR_HIP(hipStreamSynchronize(s));
  d->n_geometric = n1;
  if (n1 == 0) {
    fill_u32(d->seg_start.as<uint32_t>(), 0, npair + 1, s);
    return;
  }
  Buf cand;
  cand.alloc((size_t)n1 * 8, s);
  { ::sbr::TimedLaunch tl_("diffraction", s); hipLaunchKernelGGL(k_diff_compact, dim3(nblk(C, 256)), dim3(256), 0, s, flag.as<uint32_t>(), pos.as<uint32_t>(), C,
                     (const int64_t*)nullptr, cand.as<int64_t>()); }
  SBR_LAUNCH_CHECK();
  DiffScene S{sc->nodes.as<float4>(), sc->tri32.as<float4>(), sc->tri64.as<double>(), {}, sc->center[0],
              sc->center[1], sc->center[2], sc->n_bvh > 0, sc->n_big, (int)sc->n_bvh};
  for (int k = 0; k < 6; ++k) S.root[k] = sc->root_host[k];
  Buf flag2, pos2;
  flag2.alloc((size_t)n1 * 4, s), pos2.alloc((size_t)n1 * 4, s);
  {
    ::sbr::TimedLaunch tl_("diffraction", s);
    const unsigned g = nblk(n1, 128);
    const int depth = sc->bvh_depth;
    if (depth <= 16)
      hipLaunchKernelGGL(k_diff_legs<16>, dim3(g), dim3(128), 0, s, A, S, cand.as<int64_t>(), (int64_t)n1, flag2.as<uint32_t>());
    else if (depth <= 32)
      hipLaunchKernelGGL(k_diff_legs<32>, dim3(g), dim3(128), 0, s, A, S, cand.as<int64_t>(), (int64_t)n1, flag2.as<uint32_t>());
    else
      hipLaunchKernelGGL(k_diff_legs<64>, dim3(g), dim3(128), 0, s, A, S, cand.as<int64_t>(), (int64_t)n1, flag2.as<uint32_t>());
    SBR_LAUNCH_CHECK();
  }
  exclusive_scan_u32(flag2.as<uint32_t>(), pos2.as<uint32_t>(), n1, tot.as<uint32_t>(), temp.p, s);
  uint32_t n2 = 0;
  SBR_HIP(hipMemcpyAsync(&n2, tot.p, 4, hipMemcpyDeviceToHost, s));
  SBR_HIP(hipStreamSynchronize(s));
  SBR_CHECK(n2 < (1u << 31) - 64u, SBR_E_UNSUPPORTED, "%u paths; fewer than 2^31 - 64 in one call", n2);
  d->n_paths = n2;
  if (n2 == 0) {
    fill_u32(d->seg_start.as<uint32_t>(), 0, npair + 1, s);
    return;
  }
  Buf paths, cnt;
  paths.alloc((size_t)n2 * 8, s);
  { ::sbr::TimedLaunch tl_("diffraction", s); hipLaunchKernelGGL(k_diff_compact, dim3(nblk(n1, 256)), dim3(256), 0, s, flag2.as<uint32_t>(), pos2.as<uint32_t>(),
                     (int64_t)n1, cand.as<int64_t>(), paths.as<int64_t>()); }
  SBR_LAUNCH_CHECK();
  // the paths in (Rx, Tx) pair order, wedges ascending within a pair (a
  // stable sort of the wedge-major order by pair)
  Buf keys, vals, keys2, order, stemp;
  keys.alloc((size_t)n2 * 8, s), vals.alloc((size_t)n2 * 4, s);
  keys2.alloc((size_t)n2 * 8, s), order.alloc((size_t)n2 * 4, s);
  stemp.alloc(radix_sort_temp_bytes(n2), s);
  { ::sbr::TimedLaunch tl_("diffraction", s); hipLaunchKernelGGL(k_diff_pair_keys, dim3(nblk(n2, 256)), dim3(256), 0, s, A, paths.as<int64_t>(), (int64_t)n2,
                     keys.as<uint64_t>(), vals.as<uint32_t>()); }
  SBR_LAUNCH_CHECK();
  int pair_bits = 0;
  while ((int64_t(1) << pair_bits) < npair) ++pair_bits;
  radix_sort_pairs(keys.as<uint64_t>(), vals.as<uint32_t>(), keys2.as<uint64_t>(), order.as<uint32_t>(), (int64_t)n2, 0,
                   pair_bits, stemp.p, s);
  d->ids.alloc((size_t)n2 * 12, s);
  d->rec.alloc((size_t)n2 * 64, s);
  cnt.alloc((size_t)npair * 4, s);
  fill_u32(cnt.as<uint32_t>(), 0, npair, s);
  { ::sbr::TimedLaunch tl_("diffraction", s); hipLaunchKernelGGL(k_diff_records, dim3(nblk(n2, 256)), dim3(256), 0, s, A, paths.as<int64_t>(), order.as<uint32_t>(),
                     (int64_t)n2, d->ids.as<int32_t>(), d->rec.as<double>(), cnt.as<uint32_t>()); }
  SBR_LAUNCH_CHECK();
  Buf temp2;
  temp2.alloc(scan_temp_bytes(npair), s);
  exclusive_scan_u32(cnt.as<uint32_t>(), d->seg_start.as<uint32_t>(), npair, d->seg_start.as<uint32_t>() + npair,
                     temp2.p, s);
  SBR_HIP(hipStreamSynchronize(s));
}

namespace {
// the per-path records of one polarisation pair (n_paths of them)
void diff_records(sbr_diff_s* d, const DiffField& F, Buf& recs, hipStream_t s) {
  const int64_t n = d->n_paths;
  recs.alloc((size_t)n * sizeof(DiffRec), s);
  ::sbr::TimedLaunch tl_("diffraction", s);
  hipLaunchKernelGGL(k_diff_geo, dim3(nblk(n, 256)), dim3(256), 0, s, diff_args(d), F, d->ids.as<int32_t>(),
                     d->rec.as<double>(), n, recs.as<DiffRec>());
  SBR_LAUNCH_CHECK();
}
}  // namespace

void run_diff_channel(sbr_diff_s* d, const double* freq, int Nf, const float* atm_db, const float* atm_deg, int ptx,
                      int prx, float2* H64, double2* H128, hipStream_t s) {
  const int64_t npair = (int64_t)d->Nr * d->Nt;
  const int64_t np = d->n_paths;
  d->power.alloc((size_t)std::max<int64_t>(np, 1) * 8, s);
  d->have_power = true;
  if (np == 0 || Nf == 0) return;
  const int ntiles = (Nf + kDiffTile - 1) / kDiffTile;
  SBR_CHECK(npair * ntiles < (int64_t(1) << 31), SBR_E_UNSUPPORTED, "too many (rx, tx) pairs x frequency tiles");
  const DiffField F = diff_field_args(d, freq, Nf, atm_db, atm_deg, ptx, prx);
  Buf recs, part;
  diff_records(d, F, recs, s);
  part.alloc((size_t)np * ntiles * 8, s);
  ::sbr::TimedLaunch tl_("diffraction", s);
  hipLaunchKernelGGL(k_diff_channel, dim3((unsigned)(npair * ntiles)), dim3(64 * kDiffWaves), 0, s, F, d->Nt, d->Nr,
                     d->seg_start.as<int32_t>(), recs.as<DiffRec>(), ntiles, H64, H128, part.as<double>());
  SBR_LAUNCH_CHECK();
  run_power_final(part.as<double>(), np, ntiles, Nf, d->power.as<double>(), s);
}

void run_diff_aux(sbr_diff_s* d, double* delay, float* ang, hipStream_t s) {
  const int64_t n = d->n_paths;
  if (n == 0) return;
  hipLaunchKernelGGL(k_diff_aux, dim3(nblk(n, 256)), dim3(256), 0, s, diff_args(d), d->ids.as<int32_t>(),
                     d->rec.as<double>(), n, delay, ang);
  SBR_LAUNCH_CHECK();
}

void run_diff_field(sbr_diff_s* d, const double* freq, int Nf, const float* atm_db, const float* atm_deg, int ptx,
                    int prx, double2* out, hipStream_t s) {
  const int64_t n = d->n_paths;
  if (n == 0 || Nf == 0) return;
  const DiffField F = diff_field_args(d, freq, Nf, atm_db, atm_deg, ptx, prx);
  Buf recs;
  diff_records(d, F, recs, s);
  ::sbr::TimedLaunch tl_("diffraction", s);
  hipLaunchKernelGGL(k_diff_field, dim3(nblk(n * Nf, 256)), dim3(256), 0, s, F, recs.as<DiffRec>(), n, out);
  SBR_LAUNCH_CHECK();
}

void run_utd_transition(const double* X, int64_t n, double2* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_utd_transition, dim3(nblk(n, 256)), dim3(256), 0, s, X, n, out);
  SBR_LAUNCH_CHECK();
}

}  // namespace sbr
