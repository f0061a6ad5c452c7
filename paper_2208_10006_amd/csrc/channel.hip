// channel.hip -- ray calculation (Sec. II-A-4, II-B, II-C).
//
// Field of path n at frequency f (eq. (1) with reflections only):
//   a_n(f) = lambda/(4 pi d) * e_rx . [prod_b rho_b R_b] e_tx
//            * 10^(-gamma(f) d / 20) * exp(-j pi [2 frac(f d / c) + phi(f) d / 180])
// R_b: Fresnel TE/TM of the smooth interface (eps_c = eps_r - j sigma/(2 pi f eps0)),
// rho_b: Kirchhoff roughness factor exp(-g/2), g = (4 pi sigma_h cos_i / lambda)^2
// (eq. (6)-(8)); gamma, phi: attenuation / dispersion tables standing for
// eq. (9)-(10).  Everything is FP64: at THz carriers over hundreds of metres
// f d / c reaches 1e6 cycles, and the coherent sum of eq. (2) must stay
// accurate in deep fades where sum |a_n| >> |sum a_n|.
//
// H (eq. (13)-(14)): one block per (rx, tx) pair and tile of 64 frequencies;
// its waves split the pair's paths, each sums its share in the stored
// (delay) order, and the wave sums are added in wave order -- a segmented
// reduction with a fixed order and no atomics.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "sbr_device.hpp"
#include "sbr_internal.hpp"

namespace sbr {
namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

struct FieldArgs {
  const double* freq;
  const float* atm_db;
  const float* atm_deg;
  int Nf, ptx, prx;
};

// divisions by constants as multiplications (within 1 ulp; at f d / c ~ 1e6
// cycles that is ~1e-10 of a cycle of phase)
constexpr double kInvC0 = 1.0 / kC0;

// f = freq[fi] and inv_f = 1 / f come from the caller (once per lane, not per path)
__device__ inline cd path_amplitude(const double* __restrict__ G, const FieldArgs& A, int fi, double f,
                                    double inv_f) {
  const double d = G[0];
  const int k = (int)G[1];
  cd pol;
  if (k == 0) {
    pol = cd{G[10 + 2 * A.prx + A.ptx], 0.0};
  } else {
    cd v0{G[2 + 2 * A.ptx], 0.0}, v1{G[3 + 2 * A.ptx], 0.0};
    const double eim = -(1.0 / (2.0 * kPi * kEps0)) * inv_f;
    for (int b = 0; b < k; ++b) {
      const double* B = G + kGeoHead + kGeoPerBounce * b;
      const double cs = B[0];
      const cd ec{B[1], B[2] * eim};
      const cd root = csqrt_mod(cd{ec.re - (1.0 - cs * cs), ec.im});
      const cd rte = cdiv_mod(cd{cs - root.re, -root.im}, cd{cs + root.re, root.im});
      const cd ecc = cscale(ec, cs);
      const cd rtm = cdiv_mod(csub(ecc, root), cadd(ecc, root));
      double rho = 1.0;
      if (B[3] > 0.0) {
        const double gg = 4.0 * kPi * B[3] * cs * f * kInvC0;
        rho = exp(-0.5 * gg * gg);
      }
      const cd a0 = cscale(cmul(rte, v0), rho), a1 = cscale(cmul(rtm, v1), rho);
      if (b < k - 1) {
        v0 = cadd(cscale(a0, B[4]), cscale(a1, B[5]));
        v1 = cadd(cscale(a0, B[6]), cscale(a1, B[7]));
      } else {
        pol = cadd(cscale(a0, G[6 + 2 * A.prx]), cscale(a1, G[7 + 2 * A.prx]));
      }
    }
  }
  double amp = (kC0 / (4.0 * kPi)) * inv_f / d;
  if (A.atm_db) amp *= exp10(-(double)A.atm_db[fi] * d * (1.0 / 20.0));
  const double cyc = f * d * kInvC0;
  double ph = 2.0 * (cyc - floor(cyc));  // in units of pi
  if (A.atm_deg) ph += (double)A.atm_deg[fi] * d * (1.0 / 180.0);
  double sn, cn;
  sincospi(ph, &sn, &cn);
  const cd e{amp * cn, -amp * sn};
  return cmul(pol, e);
}

// One block per ((rx, tx) pair, tile of kChanTile frequencies): lane l of
// every wave owns frequency tile * kChanTile + l, and the waves split the
// pair's paths by index (wave w takes paths w, w + kChanWaves, ...).  Each
// wave sums its paths in their stored order; the wave sums are then added in
// wave order, so every entry of H has a fixed summation order.  The band power
// of each path is reduced over the tile's lanes into part[n][tile]; a second
// kernel adds the tiles in order.
constexpr int kChanTile = 64, kChanWaves = 4, kChanThreads = kChanTile * kChanWaves;

__global__ __launch_bounds__(kChanThreads) void k_channel(const double* __restrict__ geo, int stride,
                                                          const int32_t* __restrict__ seg_start, FieldArgs A, int Nr,
                                                          int Nt, int ntiles, float2* __restrict__ H64,
                                                          double2* __restrict__ H128, double* __restrict__ part) {
  __shared__ double sre[kChanWaves][kChanTile], sim[kChanWaves][kChanTile];
  const int64_t seg = blockIdx.x / ntiles;
  const int tile = (int)(blockIdx.x - seg * ntiles);
  const int q = (int)(seg / Nt), p = (int)(seg - (int64_t)q * Nt);
  const int n0 = seg_start[seg], n1 = seg_start[seg + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int fi = tile * kChanTile + lane;
  const bool on = fi < A.Nf;
  const double f = on ? A.freq[fi] : 1.0, inv_f = 1.0 / f;
  cd acc{0.0, 0.0};
  for (int n = n0 + wv; n < n1; n += kChanWaves) {
    double ps = 0.0;
    if (on) {
      const cd a = path_amplitude(geo + (int64_t)n * stride, A, fi, f, inv_f);
      acc = cadd(acc, a);
      ps = a.re * a.re + a.im * a.im;
    }
    if (part) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) ps += __shfl_xor(ps, o, 64);
      if (lane == 0) part[(int64_t)n * ntiles + tile] = ps;
    }
  }
  sre[wv][lane] = acc.re;
  sim[wv][lane] = acc.im;
  __syncthreads();
  if (wv == 0 && on) {
    double re = sre[0][lane], im = sim[0][lane];
#pragma unroll
    for (int w = 1; w < kChanWaves; ++w) re += sre[w][lane], im += sim[w][lane];
    const int64_t o = ((int64_t)fi * Nr + q) * Nt + p;
    if (H128) H128[o] = make_double2(re, im);
    if (H64) H64[o] = make_float2((float)re, (float)im);
  }
}

// power[n] = band mean of |a_n(f)|^2: the tiles' partial sums added in order
__global__ void k_power_final(const double* __restrict__ part, int64_t n, int ntiles, int Nf,
                              double* __restrict__ power) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double t = 0.0;
  for (int k = 0; k < ntiles; ++k) t += part[i * ntiles + k];
  power[i] = t / (double)Nf;
}

__global__ void k_path_field(const double* __restrict__ geo, int stride, int64_t n, FieldArgs A,
                             double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * A.Nf) return;
  const int64_t pth = i / A.Nf;
  const int fi = (int)(i - pth * A.Nf);
  const double f = A.freq[fi];
  const cd a = path_amplitude(geo + pth * stride, A, fi, f, 1.0 / f);
  out[i] = make_double2(a.re, a.im);
}

// per (rx, tx): incoherent path gain, RMS delay spread (eq. (5)), mean angles
// over up to kMaxStatSets sets of paths (reflection, diffraction,
// scattering).  One wave per (rx, tx) pair: lane l takes paths l, l + 64, ...
// of the pair in each set in turn, and the nine sums are combined by an xor
// butterfly (a fixed order).
struct StatSets {
  StatSet s[kMaxStatSets];
  int n;
};
__global__ __launch_bounds__(256) void k_stats(const StatSets S, int64_t nseg, float* __restrict__ pg_db,
                                               float* __restrict__ tau, float* __restrict__ angles) {
  const int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & 63;
  if (s >= nseg) return;  // whole waves leave together
  double P = 0, Pt = 0, Pt2 = 0, cd_ = 0, sd = 0, ed = 0, ca = 0, sa = 0, ea = 0;
#pragma unroll
  for (int k = 0; k < kMaxStatSets; ++k) {
    if (k >= S.n) break;
    const StatSet& T = S.s[k];
    for (int n = T.seg_start[s] + lane; n < T.seg_start[s + 1]; n += kWave) {
      const double w = T.power[n], t = T.delay[(int64_t)n * T.dstride];
      const float* a = T.ang + 4 * (int64_t)n;
      P += w;
      Pt += w * t;
      Pt2 += w * t * t;
      double sn, cn;
      sincospi((double)a[0] / 180.0, &sn, &cn);
      cd_ += w * cn, sd += w * sn, ed += w * a[1];
      sincospi((double)a[2] / 180.0, &sn, &cn);
      ca += w * cn, sa += w * sn, ea += w * a[3];
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    P += __shfl_xor(P, o, 64), Pt += __shfl_xor(Pt, o, 64), Pt2 += __shfl_xor(Pt2, o, 64);
    cd_ += __shfl_xor(cd_, o, 64), sd += __shfl_xor(sd, o, 64), ed += __shfl_xor(ed, o, 64);
    ca += __shfl_xor(ca, o, 64), sa += __shfl_xor(sa, o, 64), ea += __shfl_xor(ea, o, 64);
  }
  if (lane != 0) return;
  if (pg_db) pg_db[s] = P > 0 ? (float)(10.0 * log10(P)) : -INFINITY;
  if (tau) {
    double v = 0.0;
    if (P > 0) {
      const double m1 = Pt / P, m2 = Pt2 / P;
      v = m2 - m1 * m1;
    }
    tau[s] = (float)sqrt(v > 0 ? v : 0.0);
  }
  if (angles) {
    float* a = angles + 4 * s;
    if (P > 0) {
      a[0] = (float)(atan2(sd, cd_) * (180.0 / kPi));
      a[1] = (float)(ed / P);
      a[2] = (float)(atan2(sa, ca) * (180.0 / kPi));
      a[3] = (float)(ea / P);
    } else {
      a[0] = a[1] = a[2] = a[3] = 0.0f;
    }
  }
}

// ---------------------------------------------------------------- capacity
// per-frequency squared Frobenius norm (block per f, fixed reduction order)
__global__ __launch_bounds__(256) void k_cap_frob(const float2* __restrict__ H, int Nr, int Nt,
                                                  double* __restrict__ frob) {
  const int f = blockIdx.x;
  const int64_t m = (int64_t)Nr * Nt;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const float2 h = H[(int64_t)f * m + i];
    s += (double)h.x * h.x + (double)h.y * h.y;
  }
  __shared__ double sm[256];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) frob[f] = sm[0];
}

// scale^2 applied to W: Nt Nr / mean_f ||H_f||^2 (normalize) or 1
__global__ __launch_bounds__(256) void k_cap_scale(const double* __restrict__ frob, int Nf, int Nr, int Nt,
                                                   int normalize, double* __restrict__ scale2) {
  double s = 0.0;
  for (int f = threadIdx.x; f < Nf; f += 256) s += frob[f];
  __shared__ double sm[256];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double q = sm[0] / Nf;
    *scale2 = normalize ? (q > 0 ? (double)Nt * Nr / q : 0.0) : 1.0;
  }
}

__global__ __launch_bounds__(256) void k_cap_mean(const double* __restrict__ cf, int Nf, int Nsnr,
                                                  double* __restrict__ out) {
  __shared__ double sm[256];
  for (int si = 0; si < Nsnr; ++si) {
    double s = 0.0;
    for (int f = threadIdx.x; f < Nf; f += 256) s += cf[(int64_t)si * Nf + f];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[si] = sm[0] / Nf;
    __syncthreads();
  }
}

// Capacity for n = min(Nr, Nt) <= kCapRegN with every matrix in registers
// (block per frequency, 256 threads, no work buffer).  Thread t owns the
// 4 x 4 tile (ti, tj) = (t / 16, t % 16) of the 64 x 64 matrices, the
// problem padded with zero rows (whose pivots are 1 and add log2 1 = 0).
//  1. Gram: W = s^2 X X^H with X = H_f (Nt >= Nr) or H_f^T; X is staged in
//     LDS kCapChunk columns at a time and every thread accumulates its tile
//     in FP64.  For Nt < Nr this forms the conjugate of H^H H, which has the
//     same determinant.
//  2. For every SNR: M = I + (SNR / Nt) W and its LDL^H factorisation by
//     right-looking elimination: at step j the owners of column j publish it
//     to LDS (double-buffered, one barrier per step), every thread updates
//     its entries below and right of the pivot, M_il -= M_ij conj(M_lj) / d_j,
//     and log2 det M = sum_j log2 d_j.
constexpr int kCapRegN = 64;
constexpr int kCapChunk = 32;
constexpr int kCapSnrMax = 64;  // SNR values passed by value
struct CapSnr {
  double db[kCapSnrMax];
};

__global__ __launch_bounds__(256) void k_cap_logdet_reg(const float2* __restrict__ H, int Nr, int Nt,
                                                        const double* __restrict__ scale2,
                                                        const double* __restrict__ snr_dev, const CapSnr snr_val,
                                                        int Nsnr, double* __restrict__ cf) {
  const int f = blockIdx.x, Nf = gridDim.x;
  const int n = Nr <= Nt ? Nr : Nt;
  const int m = Nr <= Nt ? Nt : Nr;
  const bool rows = Nt >= Nr;
  const int t = threadIdx.x, ti = t >> 4, tj = t & 15;
  __shared__ float2 xs[kCapChunk][kCapRegN + 2];  // X chunk by column; +2 keeps 16-byte rows off one bank
  __shared__ double2 colb[2][kCapRegN];
  const float2* Hf = H + (int64_t)f * Nr * Nt;
  double2 w[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) w[i][j] = make_double2(0.0, 0.0);
  for (int c0 = 0; c0 < m; c0 += kCapChunk) {
    const int nc = m - c0 < kCapChunk ? m - c0 : kCapChunk;
    __syncthreads();
    for (int e = t; e < kCapChunk * kCapRegN; e += 256) {
      int r, c;
      if (rows) r = e / kCapChunk, c = e - r * kCapChunk;  // X[r][c0 + c] = H[r][c0 + c]: along c
      else c = e / kCapRegN, r = e - c * kCapRegN;         // X[r][c0 + c] = H[c0 + c][r]: along r
      float2 v = make_float2(0.0f, 0.0f);
      if (r < n && c < nc) v = rows ? Hf[(int64_t)r * Nt + c0 + c] : Hf[(int64_t)(c0 + c) * Nt + r];
      xs[c][r] = v;
    }
    __syncthreads();
    for (int c = 0; c < nc; ++c) {
      double2 a[4], b[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float2 x = xs[c][4 * ti + k], y = xs[c][4 * tj + k];
        a[k] = make_double2(x.x, x.y);
        b[k] = make_double2(y.x, y.y);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {  // w += a_i conj(b_j)
          w[i][j].x += a[i].x * b[j].x + a[i].y * b[j].y;
          w[i][j].y += a[i].y * b[j].x - a[i].x * b[j].y;
        }
    }
  }
  const double s2 = *scale2;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) w[i][j] = make_double2(w[i][j].x * s2, w[i][j].y * s2);
  for (int si = 0; si < Nsnr; ++si) {
    const double g = pow(10.0, (snr_dev ? snr_dev[si] : snr_val.db[si]) / 10.0) / Nt;
    double2 M[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        M[i][j] = make_double2((4 * ti + i == 4 * tj + j ? 1.0 : 0.0) + g * w[i][j].x, g * w[i][j].y);
    double lsum = 0.0;
    for (int jb = 0; jb < kCapRegN / 4; ++jb) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int j = 4 * jb + jj;
        double2* buf = colb[j & 1];
        if (tj == jb) {
#pragma unroll
          for (int i = 0; i < 4; ++i) buf[4 * ti + i] = M[i][jj];
        }
        __syncthreads();
        const double d = buf[j].x;
        if (t == 0) lsum += log2(d);
        const double inv = 1.0 / d;
        double2 ci[4], cl[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) ci[k] = buf[4 * ti + k], cl[k] = buf[4 * tj + k];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int l = 0; l < 4; ++l) {
            if (4 * ti + i > j && 4 * tj + l > j) {  // M_il -= c_i conj(c_l) / d
              const double re = (ci[i].x * cl[l].x + ci[i].y * cl[l].y) * inv;
              const double im = (ci[i].y * cl[l].x - ci[i].x * cl[l].y) * inv;
              M[i][l].x -= re;
              M[i][l].y -= im;
            }
          }
      }
    }
    if (t == 0) cf[(int64_t)si * Nf + f] = lsum;
  }
}

// Capacity for kCapRegN < n <= kCapBigN: the same elimination on 128 x 128
// matrices with 1,024 threads; thread t owns the 4 x 4 tile (ti, tj) =
// (t / 32, t % 32).  W and every trailing matrix of the elimination are
// Hermitian, so only tiles on or below the diagonal (tj <= ti, 528 of them)
// are formed and updated.  W stays in LDS between SNRs (tile stride 17
// entries against bank conflicts; during the Gram the front of that array
// holds the X chunk), the tile being factorised in registers.
constexpr int kCapBigN = 128;
constexpr int kCapBigSide = kCapBigN / 4;                            // 32 tiles per side
constexpr int kCapBigTiles = kCapBigSide * (kCapBigSide + 1) / 2;  // 528
constexpr int kCapTileStride = 17;                                  // double2 per tile in LDS
static_assert(kCapChunk * (kCapBigN + 2) * sizeof(float2) <= kCapBigTiles * kCapTileStride * sizeof(double2),
              "the X chunk fits in the W array");

__global__ __launch_bounds__(1024) void k_cap_logdet_big(const float2* __restrict__ H, int Nr, int Nt,
                                                         const double* __restrict__ scale2,
                                                         const double* __restrict__ snr_dev, const CapSnr snr_val,
                                                         int Nsnr, double* __restrict__ cf) {
  const int f = blockIdx.x, Nf = gridDim.x;
  const int n = Nr <= Nt ? Nr : Nt;
  const int m = Nr <= Nt ? Nt : Nr;
  const bool rows = Nt >= Nr;
  const int t = threadIdx.x, ti = t >> 5, tj = t & 31;
  const bool lower = tj <= ti;
  const int tile = ti * (ti + 1) / 2 + tj;
  __shared__ double2 wsm[kCapBigTiles * kCapTileStride];
  __shared__ double2 colb[2][kCapBigN];
  float2(*xs)[kCapBigN + 2] = reinterpret_cast<float2(*)[kCapBigN + 2]>(wsm);
  const float2* Hf = H + (int64_t)f * Nr * Nt;
  double2 w[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) w[i][j] = make_double2(0.0, 0.0);
  for (int c0 = 0; c0 < m; c0 += kCapChunk) {
    const int nc = m - c0 < kCapChunk ? m - c0 : kCapChunk;
    __syncthreads();
    for (int e = t; e < kCapChunk * kCapBigN; e += 1024) {
      int r, c;
      if (rows) r = e / kCapChunk, c = e - r * kCapChunk;  // X[r][c0 + c] = H[r][c0 + c]: along c
      else c = e / kCapBigN, r = e - c * kCapBigN;         // X[r][c0 + c] = H[c0 + c][r]: along r
      float2 v = make_float2(0.0f, 0.0f);
      if (r < n && c < nc) v = rows ? Hf[(int64_t)r * Nt + c0 + c] : Hf[(int64_t)(c0 + c) * Nt + r];
      xs[c][r] = v;
    }
    __syncthreads();
    if (lower) {
      for (int c = 0; c < nc; ++c) {
        float2 b[4];  // kept in FP32 (exact) to stay within 128 registers
#pragma unroll
        for (int k = 0; k < 4; ++k) b[k] = xs[c][4 * tj + k];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float2 x = xs[c][4 * ti + i];
          const double ax = x.x, ay = x.y;
#pragma unroll
          for (int j = 0; j < 4; ++j) {  // w += a_i conj(b_j)
            const double bx = b[j].x, by = b[j].y;
            w[i][j].x += ax * bx + ay * by;
            w[i][j].y += ay * bx - ax * by;
          }
        }
      }
    }
  }
  const double s2 = *scale2;
  __syncthreads();  // every thread is done with the X chunk
  if (lower) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) wsm[tile * kCapTileStride + 4 * i + j] = make_double2(w[i][j].x * s2, w[i][j].y * s2);
  }
  // the SNR factors before the elimination and the logarithms after it, so
  // that no constant of pow or log2 stays live (in registers) through it
  __shared__ double gs[kCapSnrMax], pm[kCapSnrMax];
  __shared__ int pe[kCapSnrMax];
  if (t < Nsnr) gs[t] = pow(10.0, (snr_dev ? snr_dev[t] : snr_val.db[t]) / 10.0) / Nt;
  __syncthreads();
  for (int si = 0; si < Nsnr; ++si) {
    const double g = gs[si];
    double2 M[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double2 v = lower ? wsm[tile * kCapTileStride + 4 * i + j] : make_double2(0.0, 0.0);
        M[i][j] = make_double2((4 * ti + i == 4 * tj + j ? 1.0 : 0.0) + g * v.x, g * v.y);
      }
    double pmant = 1.0;  // product of the pivots as pmant * 2^pexp (thread 0)
    int pexp = 0;
    for (int jb = 0; jb < kCapBigSide; ++jb) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int j = 4 * jb + jj;
        double2* buf = colb[j & 1];
        // column j below the diagonal lives in the tiles (ti >= jb, jb)
        if (tj == jb && lower) {
#pragma unroll
          for (int i = 0; i < 4; ++i) buf[4 * ti + i] = M[i][jj];
        }
        __syncthreads();
        const double d = buf[j].x;
        if (t == 0) {
          int e;
          pmant = frexp(pmant * d, &e);
          pexp += e;
        }
        if (lower && tj >= jb) {  // the trailing submatrix (ti >= tj >= jb)
          const double inv = 1.0 / d;
          double2 cl[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) cl[k] = buf[4 * tj + k];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double2 ci = buf[4 * ti + i];
#pragma unroll
            for (int l = 0; l < 4; ++l) {
              if (4 * ti + i > j && 4 * tj + l > j) {  // M_il -= c_i conj(c_l) / d
                const double re = (ci.x * cl[l].x + ci.y * cl[l].y) * inv;
                const double im = (ci.y * cl[l].x - ci.x * cl[l].y) * inv;
                M[i][l].x -= re;
                M[i][l].y -= im;
              }
            }
          }
        }
      }
    }
    if (t == 0) pm[si] = pmant, pe[si] = pexp;
  }
  __syncthreads();
  if (t < Nsnr) cf[(int64_t)t * Nf + f] = (double)pe[t] + log2(pm[t]);
}

FieldArgs field_args(const ChannelArgs& a) { return FieldArgs{a.freq, a.atm_db, a.atm_deg, a.Nf, a.pol_tx, a.pol_rx}; }

}  // namespace

void run_channel(sbr_paths_s* ps, const ChannelArgs& a, float2* H64, double2* H128, hipStream_t s) {
  const int Nt = ps->trace->Nt, Nr = ps->Nr;
  const int64_t nseg = (int64_t)Nr * Nt;
  const int ntiles = (int)((a.Nf + kChanTile - 1) / kChanTile);
  SBR_CHECK(nseg * ntiles < (int64_t(1) << 31), SBR_E_UNSUPPORTED, "too many (rx, tx) pairs x frequency tiles");
  const int64_t np = ps->n_paths;
  Buf part;
  part.alloc((size_t)std::max<int64_t>(np, 1) * ntiles * sizeof(double), s);
  { ::sbr::TimedLaunch tl_("channel", s); hipLaunchKernelGGL(k_channel, dim3((unsigned)(nseg * ntiles)), dim3(kChanThreads), 0, s, ps->geo.as<double>(),
                     geo_stride(ps->trace->K), ps->seg_start.as<int32_t>(), field_args(a), Nr, Nt, ntiles, H64, H128,
                     part.as<double>()); }
  SBR_LAUNCH_CHECK();
  if (np > 0) {
    { ::sbr::TimedLaunch tl_("channel", s); hipLaunchKernelGGL(k_power_final, dim3(nblk(np, 256)), dim3(256), 0, s, part.as<double>(), np, ntiles, a.Nf,
                       ps->power.as<double>()); }
    SBR_LAUNCH_CHECK();
  }
  ps->have_power = true;
}

void run_path_field(sbr_paths_s* ps, const ChannelArgs& a, double2* out, hipStream_t s) {
  const int64_t n = ps->n_paths;
  if (n == 0 || a.Nf == 0) return;
  { ::sbr::TimedLaunch tl_("path_field", s); hipLaunchKernelGGL(k_path_field, dim3(nblk(n * a.Nf, 256)), dim3(256), 0, s, ps->geo.as<double>(),
                     geo_stride(ps->trace->K), n, field_args(a), out); }
  SBR_LAUNCH_CHECK();
}

void run_stats_sets(const StatSet* sets, int nsets, int64_t nseg, float* pg_db, float* tau, float* angles,
                    hipStream_t s) {
  SBR_CHECK(nsets >= 1 && nsets <= kMaxStatSets, SBR_E_INVALID_ARG, "%d path sets", nsets);
  StatSets S{};
  for (int k = 0; k < nsets; ++k) S.s[k] = sets[k];
  S.n = nsets;
  { ::sbr::TimedLaunch tl_("stats", s); hipLaunchKernelGGL(k_stats, dim3(nblk(nseg * kWave, 256)), dim3(256), 0, s, S, nseg, pg_db, tau, angles); }
  SBR_LAUNCH_CHECK();
}

StatSet stat_set(sbr_paths_s* ps) {
  return StatSet{ps->seg_start.as<int32_t>(), ps->power.as<double>(), ps->info.as<double>() + 1, 2,
                 ps->ang.as<float>()};
}

void run_stats(sbr_paths_s* ps, float* pg_db, float* tau, float* angles, hipStream_t s) {
  const StatSet one = stat_set(ps);
  run_stats_sets(&one, 1, (int64_t)ps->Nr * ps->trace->Nt, pg_db, tau, angles, s);
}

void run_power_final(const double* part, int64_t n, int ntiles, int Nf, double* power, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_power_final, dim3(nblk(n, 256)), dim3(256), 0, s, part, n, ntiles, Nf, power);
  SBR_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- per-port power
// Received power of every (Rx port q, Tx port p) entry with its paths combined
// with phase (eq. (14): h_qp = sqrt(P_qp) e^{i theta_qp}), averaged over the
// band: P[q][p] = (1/Nf) sum_f |H_f[q][p]|^2 in FP64.  64 entries per block,
// one per lane (64 consecutive entries of one frequency plane per wave load);
// wave w sums the w-th sixteenth of the band in frequency order and the
// sixteen sums are added in wave order.
constexpr int kPortWaves = 16;
__global__ __launch_bounds__(64 * kPortWaves) void k_port_power(const float2* __restrict__ H, int Nf, int64_t nq,
                                                                 double* __restrict__ P) {
  __shared__ double part[kPortWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  const int per = (Nf + kPortWaves - 1) / kPortWaves, f0 = w * per, f1 = min(Nf, f0 + per);
  double acc = 0.0;
  if (e < nq)
    for (int f = f0; f < f1; ++f) {
      const float2 h = H[(int64_t)f * nq + e];
      acc += (double)h.x * (double)h.x + (double)h.y * (double)h.y;
    }
  part[w][lane] = acc;
  __syncthreads();
  if (w == 0 && e < nq) {
    double t = 0.0;
    for (int i = 0; i < kPortWaves; ++i) t += part[i][lane];
    P[e] = t / Nf;
  }
}

void run_port_power(const float2* H, int Nf, int Nr, int Nt, double* P, hipStream_t s) {
  const int64_t nq = (int64_t)Nr * Nt;
  ::sbr::TimedLaunch tl_("port_power", s);
  hipLaunchKernelGGL(k_port_power, dim3((unsigned)((nq + 63) / 64)), dim3(64 * kPortWaves), 0, s, H, Nf, nq, P);
  SBR_LAUNCH_CHECK();
}

void run_capacity(const float2* H, int Nf, int Nr, int Nt, const double* snr_db, int Nsnr, int normalize,
                  double* C_out, hipStream_t s) {
  const int n = std::min(Nr, Nt);
  Buf frob, sc, cf;
  frob.alloc((size_t)Nf * 8, s);
  sc.alloc(8, s);
  cf.alloc((size_t)Nf * Nsnr * 8, s);
  { ::sbr::TimedLaunch tl_("capacity", s); hipLaunchKernelGGL(k_cap_frob, dim3(Nf), dim3(256), 0, s, H, Nr, Nt, frob.as<double>()); }
  { ::sbr::TimedLaunch tl_("capacity", s); hipLaunchKernelGGL(k_cap_scale, dim3(1), dim3(256), 0, s, frob.as<double>(), Nf, Nr, Nt, normalize,
                     sc.as<double>()); }
  {
    ::sbr::TimedLaunch tl_("capacity", s);
    if (n <= kCapRegN)
      hipLaunchKernelGGL(k_cap_logdet_reg, dim3(Nf), dim3(256), 0, s, H, Nr, Nt, sc.as<double>(), snr_db, CapSnr{},
                         Nsnr, cf.as<double>());
    else
      hipLaunchKernelGGL(k_cap_logdet_big, dim3(Nf), dim3(1024), 0, s, H, Nr, Nt, sc.as<double>(), snr_db, CapSnr{},
                         Nsnr, cf.as<double>());
  }
  { ::sbr::TimedLaunch tl_("capacity", s); hipLaunchKernelGGL(k_cap_mean, dim3(1), dim3(256), 0, s, cf.as<double>(), Nf, Nsnr, C_out); }
  SBR_LAUNCH_CHECK();
  SBR_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- allocation-free capacity
// A fixed device array holds the per-frequency norms, the normalisation and
// the per-(SNR, frequency) log-determinants of sbr_capacity_noalloc.  Host
// code never uses its name as an address: each device's address is looked up
// once (hipGetSymbolAddress with that device current) and kept in cap_scratch_ptr.
static __device__ __align__(256) unsigned char cap_scratch[kCapScratchBytes];

namespace {
std::mutex g_cap_scratch_mu;
void* g_cap_scratch_ptr[kMaxDevices] = {};
}  // namespace

void capacity_scratch_setup(int device) {
  SBR_CHECK(device >= 0 && device < kMaxDevices, SBR_E_UNSUPPORTED, "device %d", device);
  std::lock_guard<std::mutex> lk(g_cap_scratch_mu);
  if (g_cap_scratch_ptr[device]) return;
  void* p = nullptr;
  SBR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(cap_scratch)));
  SBR_CHECK(p != nullptr, SBR_E_DEVICE, "no address for the capacity scratch on device %d", device);
  g_cap_scratch_ptr[device] = p;
}

void* capacity_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_cap_scratch_mu);
  return g_cap_scratch_ptr[device];
}

bool capacity_noalloc_fits(int Nf, int Nr, int Nt, int Nsnr) {
  return std::min(Nr, Nt) <= kCapBigN && Nsnr <= kCapSnrMax &&
         ((uint64_t)Nf * (uint64_t)(Nsnr + 1) + 32) * 8 <= (uint64_t)kCapScratchBytes;
}

// Same kernels as run_capacity (n <= 128), their buffers in `scratch`: the
// normalisation at offset 0, the norms from byte 256, the log-determinants
// after them.  Queued on s; nothing is allocated, nothing waits.
void run_capacity_noalloc(const float2* H, int Nf, int Nr, int Nt, const double* snr_db, int Nsnr, int normalize,
                          double* C_out, void* scratch, hipStream_t s) {
  double* sc = static_cast<double*>(scratch);
  double* frob = sc + 32;
  double* cf = frob + Nf;
  CapSnr sv{};
  for (int i = 0; i < Nsnr; ++i) sv.db[i] = snr_db[i];
  hipLaunchKernelGGL(k_cap_frob, dim3(Nf), dim3(256), 0, s, H, Nr, Nt, frob);
  hipLaunchKernelGGL(k_cap_scale, dim3(1), dim3(256), 0, s, frob, Nf, Nr, Nt, normalize, sc);
  if (std::min(Nr, Nt) <= kCapRegN)
    hipLaunchKernelGGL(k_cap_logdet_reg, dim3(Nf), dim3(256), 0, s, H, Nr, Nt, sc, (const double*)nullptr, sv, Nsnr, cf);
  else
    hipLaunchKernelGGL(k_cap_logdet_big, dim3(Nf), dim3(1024), 0, s, H, Nr, Nt, sc, (const double*)nullptr, sv, Nsnr, cf);
  hipLaunchKernelGGL(k_cap_mean, dim3(1), dim3(256), 0, s, cf, Nf, Nsnr, C_out);
  SBR_LAUNCH_CHECK();
}

}  // namespace sbr
