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
// v_mfma_f32_16x16x32_bf16.  Block tile 64 x 64, K step 32, 4 waves each
// owning a 32 x 32 quarter (2 x 2 MFMA tiles).  Tiles are staged in LDS
// k-contiguous per row / column so one 16-byte LDS read feeds one operand.
constexpr int TM = 64, TN = 64, TK = 32, TKP = TK + 8;  // padded row (80 B) avoids bank conflicts

enum : uint32_t { kRelu = 1u, kOutBf16 = 2u, kAccum = 4u };

__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const __bf16* __restrict__ A, int64_t a_si,
                                                   int64_t a_sk, const __bf16* __restrict__ B, int64_t b_sk,
                                                   int64_t b_sj, const float* __restrict__ bias, void* __restrict__ C,
                                                   int64_t ldc, uint32_t flags) {
  __shared__ __bf16 As[TM][TKP];
  __shared__ __bf16 Bs[TN][TKP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
  const int wi = (wv >> 1) * 32, wj = (wv & 1) * 32;
  f32x4 acc[2][2];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) acc[r][c] = f32x4{0, 0, 0, 0};
  const bool a_kc = a_sk == 1, b_kc = b_sk == 1;
  for (int k0 = 0; k0 < K; k0 += TK) {
    // ---- stage A (64 x 32) and B (32 x 64): 256 threads x 8 elements each
    {
      if (a_kc) {  // k contiguous: thread loads 8 consecutive k of one row
        const int r = tid >> 2, kk = (tid & 3) * 8;
        const int i = i0 + r;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int k = k0 + kk + t;
          As[r][kk + t] = (i < M && k < K) ? A[(int64_t)i * a_si + k] : f2bf(0.0f);
        }
      } else {  // i contiguous: thread loads 8 consecutive rows of one k
        const int kk = tid >> 3, r = (tid & 7) * 8;
        const int k = k0 + kk;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int i = i0 + r + t;
          As[r + t][kk] = (i < M && k < K) ? A[(int64_t)i * a_si + (int64_t)k * a_sk] : f2bf(0.0f);
        }
      }
      if (b_kc) {  // k contiguous: 8 consecutive k of one column
        const int c = tid >> 2, kk = (tid & 3) * 8;
        const int j = j0 + c;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int k = k0 + kk + t;
          Bs[c][kk + t] = (j < N && k < K) ? B[k + (int64_t)j * b_sj] : f2bf(0.0f);
        }
      } else {  // j contiguous: 8 consecutive columns of one k
        const int kk = tid >> 3, c = (tid & 7) * 8;
        const int k = k0 + kk;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int j = j0 + c + t;
          Bs[c + t][kk] = (j < N && k < K) ? B[(int64_t)k * b_sk + (int64_t)j * b_sj] : f2bf(0.0f);
        }
      }
    }
    __syncthreads();
    // ---- MFMA: lane l holds row/col (l % 16) and k = (l / 16) * 8 .. + 7
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    bf16x8 af[2], bfv[2];
    for (int r = 0; r < 2; ++r) af[r] = *reinterpret_cast<const bf16x8*>(&As[wi + r * 16 + fr][fk]);
    for (int c = 0; c < 2; ++c) bfv[c] = *reinterpret_cast<const bf16x8*>(&Bs[wj + c * 16 + fr][fk]);
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[r], bfv[c], acc[r][c], 0, 0, 0);
    __syncthreads();
  }
  // ---- epilogue: acc[r][c][q] is C[wi + r*16 + (lane/16)*4 + q][wj + c*16 + lane%16]
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      const int j = j0 + wj + c * 16 + (lane & 15);
      if (j >= N) continue;
      const float bj = bias ? bias[j] : 0.0f;
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + wi + r * 16 + (lane >> 4) * 4 + q;
        if (i >= M) continue;
        float v = acc[r][c][q] + bj;
        const int64_t o = (int64_t)i * ldc + j;
        if (flags & kAccum) v += (flags & kOutBf16) ? bf2f(static_cast<__bf16*>(C)[o]) : static_cast<float*>(C)[o];
        if (flags & kRelu) v = fmaxf(v, 0.0f);
        if (flags & kOutBf16) static_cast<__bf16*>(C)[o] = f2bf(v);
        else static_cast<float*>(C)[o] = v;
      }
    }
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
__global__ void k_col2im(const float* __restrict__ dcol, int n, int H, int W, int C, float* __restrict__ dx) {
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
  dx[e] = s;
}

// ---------------------------------------------------------------- elementwise
// feature row of point i: [emb(scene(i)) (E), raw x (D), sin(2^l pi x_d), cos(2^l pi x_d) for l < L] zero padded to F
__global__ void k_fourier(const float* __restrict__ x, int64_t n, int D, int L, const __bf16* __restrict__ emb, int E,
                          const int32_t* __restrict__ scene, int F, __bf16* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * F) return;
  const int64_t i = e / F;
  const int f = (int)(e - i * F);
  float v = 0.0f;
  if (f < E) {
    v = bf2f(emb[(int64_t)scene[i] * E + f]);
  } else if (f < E + D) {
    v = x[i * D + (f - E)];
  } else if (f < E + D + 2 * D * L) {
    const int g = f - E - D;
    const int d = g / (2 * L), r = g - d * 2 * L, l = r >> 1;
    const double a = (double)x[i * D + d] * (double)(1 << l);  // sin / cos (2^l pi x) via sinpi / cospi
    v = (r & 1) ? (float)cospi(a) : (float)sinpi(a);
  }
  out[e] = f2bf(v);
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

// column sums of a [M][N] fp32 matrix (bias gradients), fixed order: block per column tile
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ g, int64_t M, int N, int64_t ld,
                                                float* __restrict__ out, int accumulate) {
  const int j = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < M; i += 256) s += g[i * ld + j];
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
void nn_gemm(int M, int N, int K, const void* A, int64_t a_si, int64_t a_sk, const void* B, int64_t b_sk,
             int64_t b_sj, const float* bias, void* C, int64_t ldc, uint32_t flags, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  const dim3 g(nblk(N, TN), nblk(M, TM));
  ::sbr::TimedLaunch tl_("nn_gemm", s);
  hipLaunchKernelGGL(k_gemm_bf16, g, dim3(256), 0, s, M, N, K, static_cast<const __bf16*>(A), a_si, a_sk,
                     static_cast<const __bf16*>(B), b_sk, b_sj, bias, C, ldc, flags);
  SBR_LAUNCH_CHECK();
}
void nn_im2col(const void* x, int n, int H, int W, int C, void* col, hipStream_t s) {
  const int64_t total = (int64_t)n * (H / 2) * (W / 2) * 9 * C;
  ::sbr::TimedLaunch tl_("nn_conv", s);
  hipLaunchKernelGGL(k_im2col, dim3(nblk(total, 256)), dim3(256), 0, s, static_cast<const __bf16*>(x), n, H, W, C,
                     static_cast<__bf16*>(col));
  SBR_LAUNCH_CHECK();
}
void nn_col2im(const float* dcol, int n, int H, int W, int C, float* dx, hipStream_t s) {
  const int64_t total = (int64_t)n * H * W * C;
  ::sbr::TimedLaunch tl_("nn_conv", s);
  hipLaunchKernelGGL(k_col2im, dim3(nblk(total, 256)), dim3(256), 0, s, dcol, n, H, W, C, dx);
  SBR_LAUNCH_CHECK();
}
void nn_fourier(const float* x, int64_t n, int D, int L, const void* emb, int E, const int32_t* scene, int F,
                void* out, hipStream_t s) {
  ::sbr::TimedLaunch tl_("nn_elem", s);
  hipLaunchKernelGGL(k_fourier, dim3(nblk(n * F, 256)), dim3(256), 0, s, x, n, D, L, static_cast<const __bf16*>(emb),
                     E, scene, F, static_cast<__bf16*>(out));
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
void nn_colsum(const float* g, int64_t M, int N, int64_t ld, float* out, int accumulate, hipStream_t s) {
  ::sbr::TimedLaunch tl_("nn_elem", s);
  hipLaunchKernelGGL(k_colsum, dim3(N), dim3(256), 0, s, g, M, N, ld, out, accumulate);
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
