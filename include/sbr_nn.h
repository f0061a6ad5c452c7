/*
 * sbr_nn.h -- C-ABI of the learned radio-map surrogate kernels in libsbr.
 *
 * The surrogate predicts a link's path gain (dB) and RMS delay spread from a
 * scene height map, the Tx and Rx positions and the frequency, and is
 * trained on the outputs of the SBR path itself (sbr.h); where its ensemble
 * disagrees the caller falls back to the SBR path.  These entry points are
 * its building blocks: every array is a DEVICE pointer on the context's
 * device, every call is asynchronous on the context stream, and every call
 * returns an sbr_status (SBR_E_INVALID_ARG on a bad size or NULL pointer).
 * bf16 = IEEE bfloat16 (round to nearest even); accumulation is FP32.
 */
#ifndef SBR_NN_H_
#define SBR_NN_H_

#include "sbr.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SBR_NN_RELU 0x1u       /* max(0, .) after the bias                       */
#define SBR_NN_OUT_BF16 0x2u   /* C is bf16 (else FP32)                          */
#define SBR_NN_ACCUMULATE 0x4u /* C += result (else C = result)                  */

/* C[i][j] = sum_k A(i,k) B(k,j) + bias[j] (bias may be NULL), i < M, j < N, k < K,
 * with A(i,k) = A[i*a_si + k*a_sk] and B(k,j) = B[k*b_sk + j*b_sj] (bf16, any
 * strides: forward X W, backward-data dY W^T and backward-weight X^T dY are
 * stride choices), C[i*ldc + j].  BF16 matrix cores (v_mfma_f32_16x16x32_bf16),
 * FP32 accumulation.  A and B may be NULL when K == 0 (C = bias). */
sbr_status sbr_nn_gemm_bf16(sbr_context_t ctx, int32_t M, int32_t N, int32_t K, const void* A, int64_t a_si,
                            int64_t a_sk, const void* B, int64_t b_sk, int64_t b_sj, const float* bias, void* C,
                            int64_t ldc, uint32_t flags);
/* sbr_nn_gemm_bf16 with two backward-pass options (both may be NULL):
 * relu_mask (bf16, [M][ld_mask], ld_mask >= N): the product is set to 0 where
 *   relu_mask[i*ld_mask + j] <= 0 before bias, accumulation, ReLU and rounding,
 *   i.e. C = dY * (Y > 0) for a ReLU layer's output Y (ReLU backward fused into
 *   the backward-data product);
 * bsum (FP32, [N]): bsum[j] = sum_k B(k,j) (+= with SBR_NN_ACCUMULATE),
 *   accumulated in FP32 on the same matrix cores as one more row of A that is
 *   all ones (the bias gradient of a layer from its bf16 output gradient,
 *   fused into the backward-weight product).  M may then be 0 (A unused).
 * The K reduction is deterministic: split-K slices are summed in a fixed order. */
sbr_status sbr_nn_gemm_bf16_ex(sbr_context_t ctx, int32_t M, int32_t N, int32_t K, const void* A, int64_t a_si,
                               int64_t a_sk, const void* B, int64_t b_sk, int64_t b_sj, const float* bias, void* C,
                               int64_t ldc, uint32_t flags, const void* relu_mask, int64_t ld_mask, float* bsum);
/* 3x3, stride 2, zero-padding 1 patches of x[n][H][W][C] (bf16, channels
 * last) into col[n*(H/2)*(W/2)][9*C] (bf16, column (ky*3+kx)*C + c); H, W even. */
sbr_status sbr_nn_im2col(sbr_context_t ctx, const void* x, int32_t n, int32_t H, int32_t W, int32_t C, void* col);
/* adjoint of sbr_nn_im2col: dx[n][H][W][C] = sum of the dcol entries that read it (FP32) */
sbr_status sbr_nn_col2im(sbr_context_t ctx, const float* dcol, int32_t n, int32_t H, int32_t W, int32_t C, float* dx);
/* dz[n][H][W][C] (bf16) = that adjoint where y > 0, else 0 (y bf16, same shape):
 * the ReLU backward of the convolution layer whose output is y, fused with col2im */
sbr_status sbr_nn_col2im_relu_backward(sbr_context_t ctx, const float* dcol, int32_t n, int32_t H, int32_t W,
                                       int32_t C, const void* y, void* dz);
/* feature rows out[n][F] (bf16): emb[scene[i]][0..E), x[i][0..D), then
 * sin(2^l pi x_d), cos(2^l pi x_d) for d < D, l < L (d-major), then
 * extra[i][0..X) (extra may be NULL when X == 0), zero padded to F. */
sbr_status sbr_nn_fourier(sbr_context_t ctx, const float* x, int64_t n, int32_t D, int32_t L, const void* emb,
                          int32_t E, const int32_t* scene, const float* extra, int32_t X, int32_t F, void* out);
/* Per-link inputs of the surrogate from raw[n][7] = (Tx x, y, z, Rx x, y, z
 * in metres, f in Hz) and the scene height maps hmap[S][H][H] (bf16, height /
 * 60 m; row = y, column = x; pixel centres at -half + (c + 0.5) 2 half / H):
 * x[n][7] = (Tx x/half, y/half, z/60, Rx x/half, y/half, z/60, log f mapped
 * from [ln 28 GHz, ln 300 GHz] to [-1, 1]); extra[n][3] = (free-space path
 * gain as (120 - 20 log10(4 pi d f / c)) / 20 with d >= 1 m, minimum of
 * (segment height - terrain) / 60 over the Tx-Rx segment, mean of
 * max(0, terrain - segment height) / 60), the terrain sampled bilinearly
 * (edge-clamped) at `samples` points (k + 0.5) / samples along the segment. */
sbr_status sbr_nn_link_features(sbr_context_t ctx, const float* raw, int64_t n, const int32_t* scene,
                                const void* hmap, int32_t H, float half_extent_m, int32_t samples, float* x,
                                float* extra);
/* Fused inference of one member's point MLP for n points, all hidden layers
 * kept on chip: row i of the first layer's input is
 * [emb[scene[i]][0..128) | shared[i][0..128)] (bf16), each hidden layer
 * l < depth computes ReLU(x W_l + bias[l]) with W_l given transposed in
 * wt[l][256 out][256 in] (bf16) and bias[l][256] (FP32), rounded to bf16
 * like sbr_nn_gemm_bf16 with SBR_NN_RELU | SBR_NN_OUT_BF16; then
 * out[i][t] = sum_k x[k] out_w[k][t] + out_b[t] (out_w bf16 [256][T], FP32
 * sums), t < T.  shared, emb and wt must be 16-byte aligned. */
sbr_status sbr_nn_mlp_infer(sbr_context_t ctx, int64_t n, const void* shared, const void* emb,
                            const int32_t* scene, const void* wt, const float* bias, int32_t depth, const void* out_w,
                            const float* out_b, int32_t T, float* out);
/* dst[c][r] = src[r][c] for a bf16 matrix src[rows][cols] (dst != src) */
sbr_status sbr_nn_transpose_bf16(sbr_context_t ctx, const void* src, int32_t rows, int32_t cols, void* dst);
/* gout / gbf (either may be NULL) = g * (y > 0), y bf16 */
sbr_status sbr_nn_relu_backward(sbr_context_t ctx, const float* g, const void* y, int64_t n, float* gout, void* gbf);
sbr_status sbr_nn_cast_bf16(sbr_context_t ctx, const float* a, int64_t n, void* b);
/* loss = scale * sum w (pred - target)^2 over [n][T] (pred row stride ldp,
 * weight may be NULL), dpred = d loss / d pred (row stride ldd), loss FP64 [1] */
sbr_status sbr_nn_mse(sbr_context_t ctx, const float* pred, int64_t ldp, const float* target, const float* weight,
                      int64_t n, int32_t T, float scale, float* dpred, int64_t ldd, double* loss);
/* The ReLU backward of a [M][N] matrix (row stride N, 1 <= N <= 256) and
 * the column sums of its result in one pass:
 * gout / gbf (either may be NULL) = g * (y > 0), colsum[j] = sum_i of
 * that result's column j (FP64 sums in a fixed order, FP32 out): the
 * bias gradient of the layer, computed while the gradient is produced. */
sbr_status sbr_nn_relu_backward_colsum(sbr_context_t ctx, const float* g, const void* y, int64_t M, int32_t N,
                                       float* gout, void* gbf, float* colsum);
/* out[j] (+)= sum_i g[i*ld + j], j < N (bias gradients) */
sbr_status sbr_nn_colsum(sbr_context_t ctx, const float* g, int64_t M, int32_t N, int64_t ld, float* out,
                         int32_t accumulate);
/* Adam step `step` (1-based) on FP32 master weights w with moments m, v;
 * decoupled-free L2 term wd*w added to the gradient; wbf (may be NULL) gets
 * the bf16 copy of the updated weights. */
sbr_status sbr_nn_adam(sbr_context_t ctx, float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float wd, int32_t step, void* wbf);
/* ensemble over E members (member m at out + m*member_stride, rows of length
 * ld): mean and population spread of column t per row; mask[i] = spread > threshold */
sbr_status sbr_nn_ensemble(sbr_context_t ctx, const float* out, int32_t E, int64_t member_stride, int64_t n,
                           int64_t ld, int32_t t, float threshold, float* mean, float* spread, uint8_t* mask);

/* dst row r = src row idx[r] (row_bytes a multiple of 4; idx int64 [n]) */
sbr_status sbr_nn_gather_rows(sbr_context_t ctx, const void* src, int64_t row_bytes, const int64_t* idx, int64_t n,
                              void* dst);
/* out[i][j] = (idx[i] == j) as bf16, [n][width]: selection matrices for
 * per-scene sums done as GEMMs (deterministic) */
sbr_status sbr_nn_onehot_bf16(sbr_context_t ctx, const int32_t* idx, int64_t n, int32_t width, void* out);

#ifdef __cplusplus
}
#endif
#endif /* SBR_NN_H_ */
