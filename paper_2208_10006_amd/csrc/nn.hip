// nn.hip -- kernels of the learned radio-map surrogate (BF16 MFMA, FP32
// accumulation): GEMM with fused bias/ReLU and strided operands (forward,
// backward-data and backward-weight are the same kernel with transposed
// strides), 3x3 stride-2 convolution as im2col / col2im around that GEMM,
// Fourier features, ReLU backward, masked MSE loss, column sums, Adam with
// FP32 master weights, and the ensemble mean / spread / fallback mask.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>

#include "sbr_device.hpp"
#include "sbr_internal.hpp"

namespace sbr {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ inline __bf16 f2bf(float x) { return (__bf16)x; }  // round to nearest even
__device__ inline float bf2f(__bf16 x) { return (float)x; }

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------- GEMM
// C[i][j] = sum_k A(i,k) B(k,j) (+ bias[j]) (ReLU) with A(i,k) = A[i*a_si + k*a_sk]
// and B(k,j) = B[k*b_sk + j*b_sj] (bf16), FP32 accumulation on
// v_mfma_f32_16x16x32_bf16.  Square block tile T x T (T = 64 or 128), K step
// 64, 4 waves in a 2 x 2 arrangement each owning a (T/2) x (T/2) quarter.
// Both operands are staged in LDS k-contiguous per row (A) / column (B) so
// one 16-byte LDS read feeds one MFMA operand; the next K step's global loads
// are issued into registers before the current step's MFMAs.
//
// Operand load modes (chosen on the host from strides and alignment):
//   kKC  k contiguous (stride 1 along k), 16-byte vector loads of 8 k values;
//   kRC  row (A) / column (B) contiguous, 16-byte vector loads of 8 rows;
//   kGen any strides, element loads, same register layout as kRC.
// Split-K: blockIdx selects (tile, k-slice); with more than one slice each
// block writes its FP32 partial tile and k_gemm_reduce sums the slices in
// order (deterministic) before the epilogue.
constexpr int BK = 64, BKP = BK + 8;  // padded LDS row: 144 B, conflict-free 16-byte reads

enum : uint32_t { kRelu = 1u, kOutBf16 = 2u, kAccum = 4u };
enum LoadMode { kKC = 0, kRC = 1, kGen = 2 };

// One operand tile (ROWS x BK) of X(r, k) = X[r*s_r + k*s_k], r in [r0, rmax), k in [k0, kend).
template <int ROWS, int MODE>
struct TileLoader {
  static constexpr int CHUNKS = ROWS * BK / 8 / 256;  // 16-byte chunks per thread
  bf16x8 v[CHUNKS];

  // one_r: index of a virtual row of ones beyond the rmax stored rows (-1: none)
  __device__ void load(const __bf16* __restrict__ X, int64_t s_r, int64_t s_k, int r0, int rmax, int k0, int kend,
                       int one_r) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int c = 0; c < CHUNKS; ++c) {
      const int q = tid + c * 256;
      if (MODE == kKC) {  // chunk = 8 consecutive k of one row
        const int r = q / (BK / 8), kq = (q % (BK / 8)) * 8;
        const int row = r0 + r, k = k0 + kq;
        if (row < rmax && k + 8 <= kend) {
          v[c] = *reinterpret_cast<const bf16x8*>(X + (int64_t)row * s_r + k);
        } else {
#pragma unroll
          for (int t = 0; t < 8; ++t)
            v[c][t] = k + t >= kend ? f2bf(0.0f)
                      : row < rmax  ? X[(int64_t)row * s_r + k + t]
                                    : f2bf(row == one_r ? 1.0f : 0.0f);
        }
      } else {  // chunk = 8 consecutive rows of one k
        const int kk = q / (ROWS / 8), r8 = (q % (ROWS / 8)) * 8;
        const int row = r0 + r8, k = k0 + kk;
        if (MODE == kRC && k < kend && row + 8 <= rmax) {
          v[c] = *reinterpret_cast<const bf16x8*>(X + row + (int64_t)k * s_k);
        } else {
#pragma unroll
          for (int t = 0; t < 8; ++t)
            v[c][t] = k >= kend        ? f2bf(0.0f)
                      : row + t < rmax ? X[(int64_t)(row + t) * s_r + (int64_t)k * s_k]
                                       : f2bf(row + t == one_r ? 1.0f : 0.0f);
        }
      }
    }
  }

  __device__ void store(__bf16 (*S)[BKP]) const {
    const int tid = threadIdx.x;
#pragma unroll
    for (int c = 0; c < CHUNKS; ++c) {
      const int q = tid + c * 256;
      if (MODE == kKC) {
        const int r = q / (BK / 8), kq = (q % (BK / 8)) * 8;
        *reinterpret_cast<bf16x8*>(&S[r][kq]) = v[c];
      } else {
        const int kk = q / (ROWS / 8), r8 = (q % (ROWS / 8)) * 8;
#pragma unroll
        for (int t = 0; t < 8; ++t) S[r8 + t][kk] = v[c][t];
      }
    }
  }
};

struct GemmArgs {
  int M, N, K, kchunk, tiles_n, ntiles;
  const __bf16* A;
  int64_t a_si, a_sk;
  const __bf16* B;
  int64_t b_sk, b_sj;
  const float* bias;
  void* C;
  int64_t ldc;
  uint32_t flags;
  float* partial;  // [splits][M][N] when split, else nullptr
  int ones_row;    // row of A that is all ones (= rows of A stored; M = ones_row + 1), -1: none
  float* bsum;     // destination of that row: bsum[j] = sum_k B(k,j)
  const __bf16* mask;  // ReLU-backward mask: the product is zeroed where mask[i*ldm + j] <= 0
  int64_t ldm;
};

__device__ inline void epilogue_store(const GemmArgs& g, int i, int j, float v) {
  if (i == g.ones_row) {
    if (g.flags & kAccum) v += g.bsum[j];
    g.bsum[j] = v;
    return;
  }
  if (g.mask && !(bf2f(g.mask[(int64_t)i * g.ldm + j]) > 0.0f)) v = 0.0f;
  if (g.bias) v += g.bias[j];
  const int64_t o = (int64_t)i * g.ldc + j;
  if (g.flags & kAccum) v += (g.flags & kOutBf16) ? bf2f(static_cast<const __bf16*>(g.C)[o]) : static_cast<const float*>(g.C)[o];
  if (g.flags & kRelu) v = fmaxf(v, 0.0f);
  if (g.flags & kOutBf16) static_cast<__bf16*>(g.C)[o] = f2bf(v);
  else static_cast<float*>(g.C)[o] = v;
}

template <int T, int AMODE, int BMODE>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  constexpr int WT = T / 2, FT = WT / 16;  // wave tile, MFMA tiles per wave side
  __shared__ __bf16 As[T][BKP];
  __shared__ __bf16 Bs[T][BKP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // block -> (tile, k-slice); tiles of one XCD (block id mod 8) are contiguous
  // so blocks that share A rows share an L2
  const int b = blockIdx.x;
  const int split = b / g.ntiles, bt = b - split * g.ntiles;
  const int tile = (g.ntiles % 8 == 0) ? (bt % 8) * (g.ntiles / 8) + bt / 8 : bt;
  const int i0 = (tile / g.tiles_n) * T, j0 = (tile % g.tiles_n) * T;
  const int kb = split * g.kchunk, ke = min(g.K, kb + g.kchunk);
  const int wi = (wv >> 1) * WT, wj = (wv & 1) * WT;
  f32x4 acc[FT][FT];
#pragma unroll
  for (int r = 0; r < FT; ++r)
#pragma unroll
    for (int c = 0; c < FT; ++c) acc[r][c] = f32x4{0, 0, 0, 0};
  TileLoader<T, AMODE> la;
  TileLoader<T, BMODE> lb;
  const int ma = g.ones_row >= 0 ? g.ones_row : g.M;  // rows of A in memory
  if (kb < ke) {
    la.load(g.A, g.a_si, g.a_sk, i0, ma, kb, ke, g.ones_row);
    lb.load(g.B, g.b_sj, g.b_sk, j0, g.N, kb, ke, -1);
  }
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  for (int k0 = kb; k0 < ke; k0 += BK) {
    la.store(As);
    lb.store(Bs);
    __syncthreads();
    if (k0 + BK < ke) {  // next step's loads in flight during this step's MFMAs
      la.load(g.A, g.a_si, g.a_sk, i0, ma, k0 + BK, ke, g.ones_row);
      lb.load(g.B, g.b_sj, g.b_sk, j0, g.N, k0 + BK, ke, -1);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      bf16x8 af[FT], bfv[FT];
#pragma unroll
      for (int r = 0; r < FT; ++r) af[r] = *reinterpret_cast<const bf16x8*>(&As[wi + r * 16 + fr][kk + fk]);
#pragma unroll
      for (int c = 0; c < FT; ++c) bfv[c] = *reinterpret_cast<const bf16x8*>(&Bs[wj + c * 16 + fr][kk + fk]);
#pragma unroll
      for (int r = 0; r < FT; ++r)
#pragma unroll
        for (int c = 0; c < FT; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[r], bfv[c], acc[r][c], 0, 0, 0);
    }
    __syncthreads();
  }
  // acc[r][c][q] is C[wi + r*16 + (lane/16)*4 + q][wj + c*16 + lane%16]
#pragma unroll
  for (int r = 0; r < FT; ++r)
#pragma unroll
    for (int c = 0; c < FT; ++c) {
      const int j = j0 + wj + c * 16 + (lane & 15);
      if (j >= g.N) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + wi + r * 16 + (lane >> 4) * 4 + q;
        if (i >= g.M) continue;
        if (g.partial) g.partial[((int64_t)split * g.M + i) * g.N + j] = acc[r][c][q];
        else epilogue_store(g, i, j, acc[r][c][q]);
      }
    }
}

// 64 outputs per block, one per lane; wave w sums the w-th quarter of the
// k-slices in slice order and the quarters are added in wave order, so the
// result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_gemm_reduce(GemmArgs g, int splits) {
  __shared__ float quarter[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t mn = (int64_t)g.M * g.N;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  const int q = (splits + 3) / 4, z0 = w * q, z1 = min(splits, z0 + q);
  float s = 0.0f;
  if (e < mn)
    for (int z = z0; z < z1; ++z) s += g.partial[(int64_t)z * mn + e];
  quarter[w][lane] = s;
  __syncthreads();
  if (w == 0 && e < mn)
    epilogue_store(g, (int)(e / g.N), (int)(e % g.N), ((quarter[0][lane] + quarter[1][lane]) + quarter[2][lane]) + quarter[3][lane]);
}

// ---------------------------------------------------------------- fused MLP inference
// All hidden layers of one ensemble member for a block of kMlpBM points, the
// activations kept in LDS between layers (HBM sees only the inputs and the
// outputs).  Layer l: act <- ReLU(act W_l + b_l) in BF16 with FP32
// accumulation on v_mfma_f32_16x16x32_bf16; wave w owns output columns
// [64w, 64w + 64) for all kMlpBM rows (6 x 4 MFMA tiles, 96 accumulator
// registers); after a barrier the results overwrite the same LDS rows.  The
// weights are read as k-contiguous 16-byte fragments from a transposed copy
// ([out][in], L2-resident: 128 KB per layer).  Input row = [emb(scene) (128) |
// shared features (128)]; output layer 256 -> T by FMA (FP32 accumulation of
// BF16 products), like the unfused path.
constexpr int kMlpW = 256, kMlpBM = 96, kMlpLd = kMlpW + 8;  // padded LDS row (528 B)

__global__ __launch_bounds__(256) void k_mlp_fused(int64_t n, const __bf16* __restrict__ shared,
                                                   const __bf16* __restrict__ emb, const int32_t* __restrict__ scene,
                                                   const __bf16* __restrict__ wt, const float* __restrict__ bias,
                                                   int depth, const __bf16* __restrict__ out_w,
                                                   const float* __restrict__ out_b, int T, float* __restrict__ out) {
  __shared__ __bf16 act[kMlpBM][kMlpLd];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * kMlpBM;
  // ---- input rows: 32 chunks of 8 bf16 per row (16 embedding, 16 shared)
  for (int q = tid; q < kMlpBM * 32; q += 256) {
    const int r = q >> 5, c = q & 31;
    const int64_t row = r0 + r;
    bf16x8 v;
    if (row < n) {
      v = c < 16 ? *reinterpret_cast<const bf16x8*>(emb + (int64_t)scene[row] * 128 + c * 8)
                 : *reinterpret_cast<const bf16x8*>(shared + row * 128 + (c - 16) * 8);
    } else {
      for (int t = 0; t < 8; ++t) v[t] = f2bf(0.0f);
    }
    *reinterpret_cast<bf16x8*>(&act[r][c * 8]) = v;
  }
  __syncthreads();
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  constexpr int RT = kMlpBM / 16;
  for (int l = 0; l < depth; ++l) {
    const __bf16* W = wt + (int64_t)l * kMlpW * kMlpW;
    f32x4 acc[RT][4];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = f32x4{0, 0, 0, 0};
    for (int k0 = 0; k0 < kMlpW; k0 += 32) {
      bf16x8 bfr[4];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        bfr[c] = *reinterpret_cast<const bf16x8*>(W + (int64_t)(wv * 64 + c * 16 + fr) * kMlpW + k0 + fk);
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const bf16x8 afr = *reinterpret_cast<const bf16x8*>(&act[r * 16 + fr][k0 + fk]);
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[c], acc[r][c], 0, 0, 0);
      }
    }
    __syncthreads();  // every wave has read this layer's input
    const float* b = bias + (int64_t)l * kMlpW;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int col = wv * 64 + c * 16 + fr;
        const float bj = b[col];
#pragma unroll
        for (int q = 0; q < 4; ++q) act[r * 16 + (lane >> 4) * 4 + q][col] = f2bf(fmaxf(acc[r][c][q] + bj, 0.0f));
      }
    __syncthreads();
  }
  // ---- output layer: one (row, output) dot product per thread
  for (int q = tid; q < kMlpBM * T; q += 256) {
    const int r = q / T, o = q - r * T;
    const int64_t row = r0 + r;
    if (row >= n) continue;
    float sum = 0.0f;
    for (int k = 0; k < kMlpW; ++k) sum = fmaf(bf2f(act[r][k]), bf2f(out_w[k * T + o]), sum);
    out[row * T + o] = sum + out_b[o];
  }
}

// dst[c][r] = src[r][c] for a [rows][cols] bf16 matrix
__global__ void k_transpose_bf16(const __bf16* __restrict__ src, int rows, int cols, __bf16* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int r = (int)(e / cols), c = (int)(e - (int64_t)r * cols);
  dst[(int64_t)c * rows + r] = src[e];
}

// ---------------------------------------------------------------- conv helpers
// x: [n][H][W][C] bf16 (channels last); col: [n*Ho*Wo][9*C] bf16, column index
// (ky*3 + kx)*C + c; 3x3 window, stride 2, zero padding 1; Ho = H/2.
__global__ void k_im2col(const __bf16* __restrict__ x, int n, int H, int W, int C, __bf16* __restrict__ col) {
  const int Ho = H / 2, Wo = W / 2;
  const int64_t total = (int64_t)n * Ho * Wo * 9 * C;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int c = (int)(e % C);
  const int64_t t = e / C;
  const int tap = (int)(t % 9);
  const int64_t p = t / 9;
  const int ox = (int)(p % Wo), oy = (int)((p / Wo) % Ho), b = (int)(p / ((int64_t)Wo * Ho));
  const int iy = 2 * oy - 1 + tap / 3, ix = 2 * ox - 1 + tap % 3;
  col[e] = (iy >= 0 && iy < H && ix >= 0 && ix < W) ? x[(((int64_t)b * H + iy) * W + ix) * C + c] : f2bf(0.0f);
}

// dx[b][iy][ix][c] = sum over the (at most 4) output positions and taps that read it
// y == nullptr: dx = sum; else dz_bf = bf16(y > 0 ? sum : 0) (ReLU backward of the layer whose output is y)
__global__ void k_col2im(const float* __restrict__ dcol, int n, int H, int W, int C, float* __restrict__ dx,
                         const __bf16* __restrict__ y, __bf16* __restrict__ dz_bf) {
  const int Ho = H / 2, Wo = W / 2;
  const int64_t total = (int64_t)n * H * W * C;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int c = (int)(e % C);
  const int64_t t = e / C;
  const int ix = (int)(t % W), iy = (int)((t / W) % H), b = (int)(t / ((int64_t)W * H));
  float s = 0.0f;
  for (int ky = 0; ky < 3; ++ky) {
    const int yy = iy + 1 - ky;  // = 2 * oy
    if (yy < 0 || (yy & 1) || yy / 2 >= Ho) continue;
    for (int kx = 0; kx < 3; ++kx) {
      const int xx = ix + 1 - kx;
      if (xx < 0 || (xx & 1) || xx / 2 >= Wo) continue;
      const int64_t p = ((int64_t)b * Ho + yy / 2) * Wo + xx / 2;
      s += dcol[p * 9 * C + (ky * 3 + kx) * C + c];
    }
  }
  if (y) dz_bf[e] = f2bf(bf2f(y[e]) > 0.0f ? s : 0.0f);
  else dx[e] = s;
}

// ---------------------------------------------------------------- elementwise
// feature row of point i: [emb(scene(i)) (E), raw x (D), sin(2^l pi x_d), cos(2^l pi x_d) for l < L,
// extra (X)] zero padded to F
__global__ void k_fourier(const float* __restrict__ x, int64_t n, int D, int L, const __bf16* __restrict__ emb, int E,
                          const int32_t* __restrict__ scene, const float* __restrict__ extra, int X, int F,
                          __bf16* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * F) return;
  const int64_t i = e / F;
  const int f = (int)(e - i * F);
  const int fe = E + D + 2 * D * L;
  float v = 0.0f;
  if (f < E) {
    v = bf2f(emb[(int64_t)scene[i] * E + f]);
  } else if (f < E + D) {
    v = x[i * D + (f - E)];
  } else if (f < fe) {
    const int g = f - E - D;
    const int d = g / (2 * L), r = g - d * 2 * L, l = r >> 1;
    const double a = (double)x[i * D + d] * (double)(1 << l);  // sin / cos (2^l pi x) via sinpi / cospi
    v = (r & 1) ? (float)cospi(a) : (float)sinpi(a);
  } else if (f < fe + X) {
    v = extra[i * X + (f - fe)];
  }
  out[e] = f2bf(v);
}

// Link features of point i from its raw row (Tx x, y, z, Rx x, y, z in metres,
// f in Hz) and its scene's height map hmap[s][H][H] (bf16, height / 60 m;
// pixel (r, c) centred at (-half + (c + 0.5) * 2 half / H, -half + (r + 0.5) * 2 half / H)):
//   x[i][0..6]   Tx x / half, y / half, z / 60, Rx the same, log f mapped
//                from [ln 28 GHz, ln 300 GHz] to [-1, 1];
//   extra[i][0]  free-space path gain in the network's target units,
//                (-20 log10(4 pi d f / c) + 120) / 20, d >= 1 m;
//   extra[i][1]  min over the segment of (segment height - terrain height) / 60;
//   extra[i][2]  mean over the segment of max(0, terrain - segment height) / 60,
// the terrain sampled bilinearly (edge-clamped) at samples points (k + 0.5) / samples.
__device__ inline float hmap_bilinear(const __bf16* __restrict__ m, int H, float half, float px, float py) {
  const float pix = 2.0f * half / (float)H;
  const float u = (px + half) / pix - 0.5f, w = (py + half) / pix - 0.5f;
  const int c0 = min(max((int)floorf(u), 0), H - 2), r0 = min(max((int)floorf(w), 0), H - 2);
  const float fu = fminf(fmaxf(u - (float)c0, 0.0f), 1.0f), fw = fminf(fmaxf(w - (float)r0, 0.0f), 1.0f);
  const float h00 = bf2f(m[r0 * H + c0]), h01 = bf2f(m[r0 * H + c0 + 1]);
  const float h10 = bf2f(m[(r0 + 1) * H + c0]), h11 = bf2f(m[(r0 + 1) * H + c0 + 1]);
  return (1.0f - fw) * ((1.0f - fu) * h00 + fu * h01) + fw * ((1.0f - fu) * h10 + fu * h11);
}

__global__ void k_link_features(const float* __restrict__ raw, int64_t n, const int32_t* __restrict__ scene,
                                const __bf16* __restrict__ hmap, int H, float half, int samples, float* __restrict__ x,
                                float* __restrict__ extra) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* p = raw + i * 7;
  const float tx = p[0], ty = p[1], tz = p[2], rx = p[3], ry = p[4], rz = p[5], f = p[6];
  float* xo = x + i * 7;
  xo[0] = tx / half, xo[1] = ty / half, xo[2] = tz / 60.0f;
  xo[3] = rx / half, xo[4] = ry / half, xo[5] = rz / 60.0f;
  const float lo = logf(28e9f), hi = logf(300e9f);
  xo[6] = 2.0f * (logf(f) - lo) / (hi - lo) - 1.0f;
  const float dx = rx - tx, dy = ry - ty, dz = rz - tz;
  const float d = fmaxf(sqrtf(dx * dx + dy * dy + dz * dz), 1.0f);
  const float fspl = 20.0f * log10f(4.0f * 3.14159265358979f * d * f / 299792458.0f);
  const __bf16* m = hmap + (int64_t)scene[i] * H * H;
  float clr = 3.0e38f, sh = 0.0f;
  for (int k = 0; k < samples; ++k) {
    const float t = ((float)k + 0.5f) / (float)samples;
    const float h = 60.0f * hmap_bilinear(m, H, half, tx + t * dx, ty + t * dy);
    const float z = tz + t * dz;
    clr = fminf(clr, z - h);
    sh += fmaxf(h - z, 0.0f);
  }
  float* eo = extra + i * 3;
  eo[0] = (120.0f - fspl) / 20.0f;
  eo[1] = clr / 60.0f;
  eo[2] = sh / (float)samples / 60.0f;
}

// g (fp32, in place allowed) <- g * (y > 0); optional bf16 copy
__global__ void k_relu_bwd(const float* __restrict__ g, const __bf16* __restrict__ y, int64_t n, float* __restrict__ gout,
                           __bf16* __restrict__ gbf) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float v = bf2f(y[e]) > 0.0f ? g[e] : 0.0f;
  if (gout) gout[e] = v;
  if (gbf) gbf[e] = f2bf(v);
}

// The ReLU backward of a [M][N] gradient (N at most 256) fused with the
// column sums of its result (the bias gradient), so the matrix is read once.
// Block b covers rows [b R, (b + 1) R) with R = kReluColPerThread G and
// G = 256 / N row groups: thread t = g N + j takes column j of rows r0 + g,
// r0 + g + G, ... (kReluColPerThread of them, so that even a few thousand
// rows spread over many blocks); the groups' FP64 sums of a column are added
// in group order and go to partial[b][N], and k_colsum_final adds the blocks
// in order.
constexpr int kReluColPerThread = 32;
__global__ __launch_bounds__(256) void k_relu_bwd_colsum(const float* __restrict__ g, const __bf16* __restrict__ y,
                                                         int64_t M, int N, float* __restrict__ gout,
                                                         __bf16* __restrict__ gbf, double* __restrict__ partial) {
  const int t = threadIdx.x;
  const int groups = 256 / N;
  const int gi = t / N, j = t - gi * N;
  const int64_t rows = (int64_t)kReluColPerThread * groups;
  const int64_t r0 = (int64_t)blockIdx.x * rows;
  const int64_t r1 = min<int64_t>(M, r0 + rows);
  double s = 0.0;
  if (gi < groups) {
    for (int64_t r = r0 + gi; r < r1; r += groups) {
      const int64_t e = r * N + j;
      const float v = bf2f(y[e]) > 0.0f ? g[e] : 0.0f;
      if (gout) gout[e] = v;
      if (gbf) gbf[e] = f2bf(v);
      s += v;
    }
  }
  __shared__ double sm[256];
  sm[t] = s;
  __syncthreads();
  if (t < N) {
    double acc = 0.0;
    for (int k = 0; k < groups; ++k) acc += sm[k * N + t];
    partial[(int64_t)blockIdx.x * N + t] = acc;
  }
}

__global__ void k_cast_f32_bf16(const float* __restrict__ a, int64_t n, __bf16* __restrict__ b) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = f2bf(a[e]);
}

// masked MSE over [n][T] predictions: dpred = 2 w (pred - target) / (count), per-block partial losses
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ pred, int64_t ldp, const float* __restrict__ target,
                                             const float* __restrict__ weight, int64_t n, int T, float scale,
                                             float* __restrict__ dpred, int64_t ldd, double* __restrict__ partial) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (e < n * T) {
    const int64_t i = e / T;
    const int t = (int)(e - i * T);
    const float w = weight ? weight[e] : 1.0f;
    const float r = pred[i * ldp + t] - target[e];
    l = (double)w * r * r * scale;
    dpred[i * ldd + t] = 2.0f * w * r * scale;
  }
  __shared__ double sm[256];
  sm[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

// column sums of a [M][N] fp32 matrix (bias gradients), deterministic two-pass:
// block (column group of 64, row chunk) -> partial[chunk][j] in FP64, then
// k_colsum_final adds the chunks in order.
constexpr int kColsumRows = 1024;
__global__ __launch_bounds__(256) void k_colsum_part(const float* __restrict__ g, int64_t M, int N, int64_t ld,
                                                     double* __restrict__ partial) {
  const int jl = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + jl;
  const int64_t r0 = (int64_t)blockIdx.y * kColsumRows, r1 = min<int64_t>(M, r0 + kColsumRows);
  double s = 0.0;
  if (j < N)
    for (int64_t i = r0 + rg; i < r1; i += 4) s += g[i * ld + j];
  __shared__ double sm[4][64];
  sm[rg][jl] = s;
  __syncthreads();
  if (rg == 0 && j < N) partial[(int64_t)blockIdx.y * N + j] = ((sm[0][jl] + sm[1][jl]) + sm[2][jl]) + sm[3][jl];
}

// block per column j: thread t adds chunks t, t + 256, ... and a fixed tree
// adds the threads' sums, so many chunks of a narrow matrix reduce in parallel
__global__ __launch_bounds__(256) void k_colsum_final(const double* __restrict__ partial, int chunks, int N,
                                                      float* __restrict__ out, int accumulate) {
  const int j = blockIdx.x;
  double s = 0.0;
  for (int c = threadIdx.x; c < chunks; c += 256) s += partial[(int64_t)c * N + j];
  __shared__ double sm[256];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = (accumulate ? out[j] : 0.0f) + (float)sm[0];
}

__global__ void k_sum_f64(const double* __restrict__ p, int64_t n, double* __restrict__ out) {
  __shared__ double sm[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += p[i];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

// Adam (Kingma & Ba) on FP32 master weights; refreshes the BF16 working copy
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float wd, float c1, float c2,
                       __bf16* __restrict__ wbf) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e] + wd * w[e];
  const float mm = b1 * m[e] + (1.0f - b1) * gg;
  const float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
  m[e] = mm, v[e] = vv;
  const float upd = (mm / c1) / (sqrtf(vv / c2) + eps);
  const float nw = w[e] - lr * upd;
  w[e] = nw;
  if (wbf) wbf[e] = f2bf(nw);
}

// ensemble over E members of [n][ld] outputs: mean and (population) spread of
// output column t; mask = spread > threshold
__global__ void k_ensemble(const float* __restrict__ out, int E, int64_t member_stride, int64_t n, int64_t ld, int t,
                           float threshold, float* __restrict__ mean, float* __restrict__ spread,
                           uint8_t* __restrict__ mask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0, s2 = 0.0;
  for (int m = 0; m < E; ++m) {
    const double v = out[m * member_stride + i * ld + t];
    s += v;
    s2 += v * v;
  }
  const double mu = s / E;
  const double var = s2 / E - mu * mu;
  const float sd = (float)sqrt(var > 0 ? var : 0.0);
  mean[i] = (float)mu;
  if (spread) spread[i] = sd;
  if (mask) mask[i] = sd > threshold ? 1 : 0;
}

// dst row r = src row idx[r] (rows of row_bytes, a multiple of 4)
__global__ void k_gather_rows(const uint32_t* __restrict__ src, int64_t words, const int64_t* __restrict__ idx,
                              int64_t n, uint32_t* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * words) return;
  const int64_t r = e / words, w = e - r * words;
  dst[e] = src[idx[r] * words + w];
}

// out[i][j] = (idx[i] == j), bf16, [n][width]
__global__ void k_onehot(const int32_t* __restrict__ idx, int64_t n, int width, __bf16* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * width) return;
  const int64_t i = e / width;
  out[e] = f2bf(idx[i] == (int)(e - i * width) ? 1.0f : 0.0f);
}

}  // namespace

void nn_gather_rows(const void* src, int64_t row_bytes, const int64_t* idx, int64_t n, void* dst, hipStream_t s) {
  const int64_t words = row_bytes / 4;
  ::sbr::TimedLaunch tl_("nn_elem", s);
  hipLaunchKernelGGL(k_gather_rows, dim3(nblk(n * words, 256)), dim3(256), 0, s, static_cast<const uint32_t*>(src),
                     words, idx, n, static_cast<uint32_t*>(dst));
  SBR_LAUNCH_CHECK();
}
void nn_onehot(const int32_t* idx, int64_t n, int width, void* out, hipStream_t s) {
  ::sbr::TimedLaunch tl_("nn_elem", s);
  hipLaunchKernelGGL(k_onehot, dim3(nblk(n * width, 256)), dim3(256), 0, s, idx, n, width, static_cast<__bf16*>(out));
  SBR_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- launchers
namespace {
int load_mode(const void* X, int64_t s_r, int64_t s_k) {
  const bool al = (reinterpret_cast<uintptr_t>(X) & 15) == 0;
  if (s_k == 1 && s_r % 8 == 0 && al) return kKC;
  if (s_r == 1 && s_k % 8 == 0 && al) return kRC;
  return kGen;
}

template <int T>
void launch_gemm_t(const GemmArgs& g, int am, int bm, int blocks, hipStream_t s) {
#define SBR_GEMM_CASE(A_, B_) \
  if (am == A_ && bm == B_) { hipLaunchKernelGGL((k_gemm_bf16<T, A_, B_>), dim3(blocks), dim3(256), 0, s, g); return; }
  SBR_GEMM_CASE(kKC, kKC) SBR_GEMM_CASE(kKC, kRC) SBR_GEMM_CASE(kKC, kGen)
  SBR_GEMM_CASE(kRC, kKC) SBR_GEMM_CASE(kRC, kRC) SBR_GEMM_CASE(kRC, kGen)
  SBR_GEMM_CASE(kGen, kKC) SBR_GEMM_CASE(kGen, kRC) SBR_GEMM_CASE(kGen, kGen)
#undef SBR_GEMM_CASE
}
}  // namespace

void nn_gemm(int M, int N, int K, const void* A, int64_t a_si, int64_t a_sk, const void* B, int64_t b_sk,
             int64_t b_sj, const float* bias, void* C, int64_t ldc, uint32_t flags, hipStream_t s,
             const void* mask, int64_t ldm, float* bsum) {
  if (N <= 0 || (M <= 0 && !bsum)) return;
  int num_cus = 256;
  {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&num_cus, hipDeviceAttributeMultiprocessorCount, dev);
  }
  // column sums of B ride along as one more row of A (all ones)
  const int Mr = M + (bsum ? 1 : 0);
  // 128-wide tiles when they alone fill the chip, else 64
  const int64_t t128 = (int64_t)((Mr + 127) / 128) * ((N + 127) / 128);
  const int T = t128 >= 2 * num_cus ? 128 : 64;
  const int tiles_m = (Mr + T - 1) / T, tiles_n = (N + T - 1) / T, ntiles = tiles_m * tiles_n;
  // split K only when the tiles leave CUs idle and K is long; at most 64
  // slices so that the ordered reduction stays short
  const int ksteps = (K + BK - 1) / BK;
  int splits = 1;
  if (ntiles < num_cus && ksteps >= 8)
    splits = std::max(1, std::min(std::min((2 * num_cus + ntiles - 1) / ntiles, ksteps / 4), 64));
  const int kchunk = ((ksteps + splits - 1) / splits) * BK;
  if (K > 0) splits = (K + kchunk - 1) / kchunk;
  GemmArgs g{Mr, N, K, kchunk, tiles_n, ntiles, static_cast<const __bf16*>(A), a_si, a_sk,
             static_cast<const __bf16*>(B), b_sk, b_sj, bias, C, ldc, flags, nullptr,
             bsum ? M : -1, bsum, static_cast<const __bf16*>(mask), ldm};
  Buf part;
  if (splits > 1) {
    part.alloc((size_t)splits * Mr * N * 4, s);
    g.partial = part.as<float>();
  }
  const int am = load_mode(A, a_si, a_sk), bm = load_mode(B, b_sj, b_sk);
  ::sbr::TimedLaunch tl_("nn_gemm", s);
  if (T == 128) launch_gemm_t<128>(g, am, bm, ntiles * splits, s);
  else launch_gemm_t<64>(g, am, bm, ntiles * splits, s);
  if (splits > 1) {
    const int64_t mn = (int64_t)Mr * N;
    hipLaunchKernelGGL(k_gemm_reduce, dim3(nblk(mn, 64)), dim3(256), 0, s, g, splits);
  }
  SBR_LAUNCH_CHECK();
}
void nn_mlp_fused(int64_t n, const void* shared, const void* emb, const int32_t* scene, const void* wt,
                  const float* bias, int depth, const void* out_w, const float* out_b, int T, float* out,
                  hipStream_t s) {
  if (n <= 0) return;
  ::sbr::TimedLaunch tl_("nn_mlp", s);
  hipLaunchKernelGGL(k_mlp_fused, dim3(nblk(n, kMlpBM)), dim3(256), 0, s, n, static_cast<const __bf16*>(shared),
                     static_cast<const __bf16*>(emb), scene, static_cast<const __bf16*>(wt), bias, depth,
                     static_cast<const __bf16*>(out_w), out_b, T, out);
  SBR_LAUNCH_CHECK();
}
void nn_transpose(const void* src, int rows, int cols, void* dst, hipStream_t s) {
  ::sbr::TimedLaunch tl_("nn_elem", s);
  hipLaunchKernelGGL(k_transpose_bf16, dim3(nblk((int64_t)rows * cols, 256)), dim3(256), 0, s,
                     static_cast<const __bf16*>(src), rows, cols, static_cast<__bf16*>(dst));
  SBR_LAUNCH_CHECK();
}
void nn_im2col(const void* x, int n, int H, int W, int C, void* col, hipStream_t s) {
  const int64_t total = (int64_t)n * (H / 2) * (W / 2) * 9 * C;
  ::sbr::TimedLaunch tl_("nn_conv", s);
  hipLaunchKernelGGL(k_im2col, dim3(nblk(total, 256)), dim3(256), 0, s, static_cast<const __bf16*>(x), n, H, W, C,
                     static_cast<__bf16*>(col));
  SBR_LAUNCH_CHECK();
}
void nn_col2im(const float* dcol, int n, int H, int W, int C, float* dx, hipStream_t s, const void* y, void* dz_bf) {
  const int64_t total = (int64_t)n * H * W * C;
  ::sbr::TimedLaunch tl_("nn_conv", s);
  hipLaunchKernelGGL(k_col2im, dim3(nblk(total, 256)), dim3(256), 0, s, dcol, n, H, W, C, dx,
                     static_cast<const __bf16*>(y), static_cast<__bf16*>(dz_bf));
  SBR_LAUNCH_CHECK();
}
void nn_fourier(const float* x, int64_t n, int D, int L, const void* emb, int E, const int32_t* scene,
                const float* extra, int X, int F, void* out, hipStream_t s) {
  ::sbr::TimedLaunch tl_("nn_elem", s);
  hipLaunchKernelGGL(k_fourier, dim3(nblk(n * F, 256)), dim3(256), 0, s, x, n, D, L, static_cast<const __bf16*>(emb),
                     E, scene, extra, X, F, static_cast<__bf16*>(out));
  SBR_LAUNCH_CHECK();
}
void nn_link_features(const float* raw, int64_t n, const int32_t* scene, const void* hmap, int H, float half,
                      int samples, float* x, float* extra, hipStream_t s) {
  ::sbr::TimedLaunch tl_("nn_elem", s);
  hipLaunchKernelGGL(k_link_features, dim3(nblk(n, 256)), dim3(256), 0, s, raw, n, scene,
                     static_cast<const __bf16*>(hmap), H, half, samples, x, extra);
  SBR_LAUNCH_CHECK();
}
void nn_relu_bwd(const float* g, const void* y, int64_t n, float* gout, void* gbf, hipStream_t s) {
  ::sbr::TimedLaunch tl_("nn_elem", s);
  hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(n, 256)), dim3(256), 0, s, g, static_cast<const __bf16*>(y), n, gout,
                     static_cast<__bf16*>(gbf));
  SBR_LAUNCH_CHECK();
}
void nn_cast(const float* a, int64_t n, void* b, hipStream_t s) {
  ::sbr::TimedLaunch tl_("nn_elem", s);
  hipLaunchKernelGGL(k_cast_f32_bf16, dim3(nblk(n, 256)), dim3(256), 0, s, a, n, static_cast<__bf16*>(b));
  SBR_LAUNCH_CHECK();
}
void nn_mse(const float* pred, int64_t ldp, const float* target, const float* weight, int64_t n, int T, float scale,
            float* dpred, int64_t ldd, double* loss, hipStream_t s) {
  const int64_t nb = std::max<int64_t>(1, (n * T + 255) / 256);
  Buf part;
  part.alloc(nb * 8, s);
  ::sbr::TimedLaunch tl_("nn_elem", s);
  hipLaunchKernelGGL(k_mse, dim3((unsigned)nb), dim3(256), 0, s, pred, ldp, target, weight, n, T, scale, dpred, ldd,
                     part.as<double>());
  hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, s, part.as<double>(), nb, loss);
  SBR_LAUNCH_CHECK();
}
void nn_relu_bwd_colsum(const float* g, const void* y, int64_t M, int N, float* gout, void* gbf, float* colsum,
                        hipStream_t s) {
  const int64_t rows = (int64_t)kReluColPerThread * (256 / N);
  const int chunks = (int)std::max<int64_t>(1, (M + rows - 1) / rows);
  Buf part;
  part.alloc((size_t)chunks * N * 8, s);
  ::sbr::TimedLaunch tl_("nn_elem", s);
  hipLaunchKernelGGL(k_relu_bwd_colsum, dim3(chunks), dim3(256), 0, s, g, static_cast<const __bf16*>(y), M, N, gout,
                     static_cast<__bf16*>(gbf), part.as<double>());
  hipLaunchKernelGGL(k_colsum_final, dim3(N), dim3(256), 0, s, part.as<double>(), chunks, N, colsum, 0);
  SBR_LAUNCH_CHECK();
}
void nn_colsum(const float* g, int64_t M, int N, int64_t ld, float* out, int accumulate, hipStream_t s) {
  const int chunks = (int)std::max<int64_t>(1, (M + kColsumRows - 1) / kColsumRows);
  Buf part;
  part.alloc((size_t)chunks * N * 8, s);
  ::sbr::TimedLaunch tl_("nn_elem", s);
  hipLaunchKernelGGL(k_colsum_part, dim3((N + 63) / 64, chunks), dim3(256), 0, s, g, M, N, ld, part.as<double>());
  hipLaunchKernelGGL(k_colsum_final, dim3(N), dim3(256), 0, s, part.as<double>(), chunks, N, out, accumulate);
  SBR_LAUNCH_CHECK();
}
void nn_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
             float wd, int step, void* wbf, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  ::sbr::TimedLaunch tl_("nn_adam", s);
  hipLaunchKernelGGL(k_adam, dim3(nblk(n, 256)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, wd, c1, c2,
                     static_cast<__bf16*>(wbf));
  SBR_LAUNCH_CHECK();
}
void nn_ensemble(const float* out, int E, int64_t member_stride, int64_t n, int64_t ld, int t, float threshold,
                 float* mean, float* spread, uint8_t* mask, hipStream_t s) {
  ::sbr::TimedLaunch tl_("nn_elem", s);
  hipLaunchKernelGGL(k_ensemble, dim3(nblk(n, 256)), dim3(256), 0, s, out, E, member_stride, n, ld, t, threshold,
                     mean, spread, mask);
  SBR_LAUNCH_CHECK();
}

}  // namespace sbr
