// nn_api.hip -- C-ABI wrappers of the surrogate kernels (include/sbr_nn.h).
#include <cmath>
#include <functional>

#include "../../include/sbr_nn.h"
#include "sbr_internal.hpp"

namespace sbr {
sbr_status nn_guard_call(sbr_context_t ctx, const std::function<void(hipStream_t)>& f);
}

using namespace sbr;

#define NN_ENTRY(body)                                                                    \
  return nn_guard_call(ctx, [&](hipStream_t s) { body; })
#define NN_REQUIRE(cond, ...) SBR_CHECK(cond, SBR_E_INVALID_ARG, __VA_ARGS__)

extern "C" {

sbr_status sbr_nn_gemm_bf16(sbr_context_t ctx, int32_t M, int32_t N, int32_t K, const void* A, int64_t a_si,
                            int64_t a_sk, const void* B, int64_t b_sk, int64_t b_sj, const float* bias, void* C,
                            int64_t ldc, uint32_t flags) {
  NN_ENTRY({
    NN_REQUIRE(M >= 0 && N >= 0 && K >= 0 && (M == 0 || N == 0 || (C && (K == 0 || (A && B)))), "gemm arguments");
    NN_REQUIRE((flags & ~7u) == 0, "gemm flags 0x%x", flags);
    nn_gemm(M, N, K, A, a_si, a_sk, B, b_sk, b_sj, bias, C, ldc, flags, s);
  });
}

sbr_status sbr_nn_gemm_bf16_ex(sbr_context_t ctx, int32_t M, int32_t N, int32_t K, const void* A, int64_t a_si,
                               int64_t a_sk, const void* B, int64_t b_sk, int64_t b_sj, const float* bias, void* C,
                               int64_t ldc, uint32_t flags, const void* relu_mask, int64_t ld_mask, float* bsum) {
  NN_ENTRY({
    NN_REQUIRE(M >= 0 && N >= 0 && K >= 0 && (M == 0 || N == 0 || (C && (K == 0 || (A && B)))), "gemm arguments");
    NN_REQUIRE(!bsum || N == 0 || K == 0 || B, "gemm column sums need B");
    NN_REQUIRE(!relu_mask || ld_mask >= N, "gemm mask leading dimension %lld < N %d", (long long)ld_mask, N);
    NN_REQUIRE((flags & ~7u) == 0, "gemm flags 0x%x", flags);
    nn_gemm(M, N, K, A, a_si, a_sk, B, b_sk, b_sj, bias, C, ldc, flags, s, relu_mask, ld_mask, bsum);
  });
}

sbr_status sbr_nn_im2col(sbr_context_t ctx, const void* x, int32_t n, int32_t H, int32_t W, int32_t C, void* col) {
  NN_ENTRY({
    NN_REQUIRE(x && col && n > 0 && H > 0 && W > 0 && C > 0 && H % 2 == 0 && W % 2 == 0, "im2col arguments");
    nn_im2col(x, n, H, W, C, col, s);
  });
}

sbr_status sbr_nn_col2im(sbr_context_t ctx, const float* dcol, int32_t n, int32_t H, int32_t W, int32_t C, float* dx) {
  NN_ENTRY({
    NN_REQUIRE(dcol && dx && n > 0 && H > 0 && W > 0 && C > 0 && H % 2 == 0 && W % 2 == 0, "col2im arguments");
    nn_col2im(dcol, n, H, W, C, dx, s);
  });
}

sbr_status sbr_nn_col2im_relu_backward(sbr_context_t ctx, const float* dcol, int32_t n, int32_t H, int32_t W,
                                       int32_t C, const void* y, void* dz) {
  NN_ENTRY({
    NN_REQUIRE(dcol && y && dz && n > 0 && H > 0 && W > 0 && C > 0 && H % 2 == 0 && W % 2 == 0,
               "col2im_relu_backward arguments");
    nn_col2im(dcol, n, H, W, C, nullptr, s, y, dz);
  });
}

sbr_status sbr_nn_fourier(sbr_context_t ctx, const float* x, int64_t n, int32_t D, int32_t L, const void* emb,
                          int32_t E, const int32_t* scene, const float* extra, int32_t X, int32_t F, void* out) {
  NN_ENTRY({
    NN_REQUIRE(x && out && n >= 0 && D >= 0 && L >= 0 && L <= 30 && E >= 0 && X >= 0 &&
                   F >= E + D + 2 * D * L + X,
               "fourier arguments");
    NN_REQUIRE(E == 0 || (emb && scene), "fourier embedding");
    NN_REQUIRE(X == 0 || extra, "fourier extra columns");
    if (n > 0) nn_fourier(x, n, D, L, emb, E, scene, extra, X, F, out, s);
  });
}

sbr_status sbr_nn_mlp_infer(sbr_context_t ctx, int64_t n, const void* shared, const void* emb,
                            const int32_t* scene, const void* wt, const float* bias, int32_t depth, const void* out_w,
                            const float* out_b, int32_t T, float* out) {
  NN_ENTRY({
    NN_REQUIRE(n >= 0 && depth >= 1 && depth <= 64 && T >= 1 && T <= 64, "mlp_infer sizes");
    NN_REQUIRE(n == 0 || (shared && emb && scene && wt && bias && out_w && out_b && out), "mlp_infer arguments");
    NN_REQUIRE(n == 0 || ((reinterpret_cast<uintptr_t>(shared) | reinterpret_cast<uintptr_t>(emb) |
                           reinterpret_cast<uintptr_t>(wt)) & 15) == 0,
               "mlp_infer: shared, emb and wt must be 16-byte aligned");
    nn_mlp_fused(n, shared, emb, scene, wt, bias, depth, out_w, out_b, T, out, s);
  });
}

sbr_status sbr_nn_transpose_bf16(sbr_context_t ctx, const void* src, int32_t rows, int32_t cols, void* dst) {
  NN_ENTRY({
    NN_REQUIRE(src && dst && rows >= 0 && cols >= 0 && src != dst, "transpose arguments");
    if ((int64_t)rows * cols > 0) nn_transpose(src, rows, cols, dst, s);
  });
}

sbr_status sbr_nn_link_features(sbr_context_t ctx, const float* raw, int64_t n, const int32_t* scene,
                                const void* hmap, int32_t H, float half_extent_m, int32_t samples, float* x,
                                float* extra) {
  NN_ENTRY({
    NN_REQUIRE(raw && scene && hmap && x && extra && n >= 0 && H >= 2 && half_extent_m > 0.0f && samples >= 1,
               "link_features arguments");
    if (n > 0) nn_link_features(raw, n, scene, hmap, H, half_extent_m, samples, x, extra, s);
  });
}

sbr_status sbr_nn_relu_backward(sbr_context_t ctx, const float* g, const void* y, int64_t n, float* gout, void* gbf) {
  NN_ENTRY({
    NN_REQUIRE(g && y && n >= 0 && (gout || gbf), "relu_backward arguments");
    if (n > 0) nn_relu_bwd(g, y, n, gout, gbf, s);
  });
}

sbr_status sbr_nn_cast_bf16(sbr_context_t ctx, const float* a, int64_t n, void* b) {
  NN_ENTRY({
    NN_REQUIRE(a && b && n >= 0, "cast arguments");
    if (n > 0) nn_cast(a, n, b, s);
  });
}

sbr_status sbr_nn_mse(sbr_context_t ctx, const float* pred, int64_t ldp, const float* target, const float* weight,
                      int64_t n, int32_t T, float scale, float* dpred, int64_t ldd, double* loss) {
  NN_ENTRY({
    NN_REQUIRE(pred && target && dpred && loss && n >= 0 && T > 0, "mse arguments");
    nn_mse(pred, ldp, target, weight, n, T, scale, dpred, ldd, loss, s);
  });
}

sbr_status sbr_nn_relu_backward_colsum(sbr_context_t ctx, const float* g, const void* y, int64_t M, int32_t N,
                                       float* gout, void* gbf, float* colsum) {
  NN_ENTRY({
    NN_REQUIRE(g && y && colsum && M >= 0 && N >= 1 && N <= 256 && (gout || gbf),
               "relu_backward_colsum arguments (1 <= N <= 256)");
    nn_relu_bwd_colsum(g, y, M, N, gout, gbf, colsum, s);
  });
}

sbr_status sbr_nn_colsum(sbr_context_t ctx, const float* g, int64_t M, int32_t N, int64_t ld, float* out,
                         int32_t accumulate) {
  NN_ENTRY({
    NN_REQUIRE(g && out && M >= 0 && N > 0, "colsum arguments");
    nn_colsum(g, M, N, ld, out, accumulate, s);
  });
}

sbr_status sbr_nn_adam(sbr_context_t ctx, float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float wd, int32_t step, void* wbf) {
  NN_ENTRY({
    NN_REQUIRE(w && g && m && v && n >= 0 && step >= 1, "adam arguments");
    if (n > 0) nn_adam(w, g, m, v, n, lr, b1, b2, eps, wd, step, wbf, s);
  });
}

sbr_status sbr_nn_ensemble(sbr_context_t ctx, const float* out, int32_t E, int64_t member_stride, int64_t n,
                           int64_t ld, int32_t t, float threshold, float* mean, float* spread, uint8_t* mask) {
  NN_ENTRY({
    NN_REQUIRE(out && mean && E >= 1 && n >= 0 && t >= 0 && t < ld, "ensemble arguments");
    if (n > 0) nn_ensemble(out, E, member_stride, n, ld, t, threshold, mean, spread, mask, s);
  });
}

sbr_status sbr_nn_gather_rows(sbr_context_t ctx, const void* src, int64_t row_bytes, const int64_t* idx, int64_t n,
                              void* dst) {
  NN_ENTRY({
    NN_REQUIRE(src && idx && dst && n >= 0 && row_bytes > 0 && row_bytes % 4 == 0, "gather arguments");
    if (n > 0) nn_gather_rows(src, row_bytes, idx, n, dst, s);
  });
}

sbr_status sbr_nn_onehot_bf16(sbr_context_t ctx, const int32_t* idx, int64_t n, int32_t width, void* out) {
  NN_ENTRY({
    NN_REQUIRE(idx && out && n >= 0 && width > 0, "onehot arguments");
    if (n > 0) nn_onehot(idx, n, width, out, s);
  });
}

}  // extern "C"
