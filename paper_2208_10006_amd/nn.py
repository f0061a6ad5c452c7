"""Python binding of the surrogate kernels (include/sbr_nn.h), argument
marshalling only.  All tensors are torch tensors on the context's GPU; the
functions keep the C entry point names and return nothing (results are
written into the output tensors, in stream order)."""
from __future__ import annotations

import ctypes as C

import torch

from . import sbr as S

L = S._lib
P, I32, I64, U32, F = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_float
_SIG = {
    "sbr_nn_gemm_bf16": [P, I32, I32, I32, P, I64, I64, P, I64, I64, P, P, I64, U32],
    "sbr_nn_gemm_bf16_ex": [P, I32, I32, I32, P, I64, I64, P, I64, I64, P, P, I64, U32, P, I64, P],
    "sbr_nn_im2col": [P, P, I32, I32, I32, I32, P],
    "sbr_nn_col2im": [P, P, I32, I32, I32, I32, P],
    "sbr_nn_col2im_relu_backward": [P, P, I32, I32, I32, I32, P, P],
    "sbr_nn_fourier": [P, P, I64, I32, I32, P, I32, P, P, I32, I32, P],
    "sbr_nn_link_features": [P, P, I64, P, P, I32, F, I32, P, P],
    "sbr_nn_relu_backward": [P, P, P, I64, P, P],
    "sbr_nn_cast_bf16": [P, P, I64, P],
    "sbr_nn_mse": [P, P, I64, P, P, I64, I32, F, P, I64, P],
    "sbr_nn_colsum": [P, P, I64, I32, I64, P, I32],
    "sbr_nn_relu_backward_colsum": [P, P, P, I64, I32, P, P, P],
    "sbr_nn_adam": [P, P, P, P, P, I64, F, F, F, F, F, I32, P],
    "sbr_nn_ensemble": [P, P, I32, I64, I64, I64, I32, F, P, P, P],
    "sbr_nn_gather_rows": [P, P, I64, P, I64, P],
    "sbr_nn_onehot_bf16": [P, P, I64, I32, P],
    "sbr_nn_mlp_infer": [P, I64, P, P, P, P, P, I32, P, P, I32, P],
    "sbr_nn_transpose_bf16": [P, P, I32, I32, P],
}
for _n, _a in _SIG.items():
    _f = getattr(L, _n)
    _f.argtypes = _a
    _f.restype = C.c_int

RELU, OUT_BF16, ACCUMULATE = 1, 2, 4


def _p(t):
    if t is None:
        return None
    assert t.is_cuda, "surrogate kernels take device tensors"
    return C.c_void_p(t.data_ptr())


def sbr_nn_gemm_bf16(ctx, M, N, K, A, a_si, a_sk, B, b_sk, b_sj, bias, Cout, ldc, flags=0):
    S._call("sbr_nn_gemm_bf16", ctx.h, M, N, K, _p(A), a_si, a_sk, _p(B), b_sk, b_sj, _p(bias), _p(Cout), ldc, flags)


def sbr_nn_gemm_bf16_ex(ctx, M, N, K, A, a_si, a_sk, B, b_sk, b_sj, bias, Cout, ldc, flags=0, relu_mask=None,
                        ld_mask=0, bsum=None):
    S._call("sbr_nn_gemm_bf16_ex", ctx.h, M, N, K, _p(A), a_si, a_sk, _p(B), b_sk, b_sj, _p(bias), _p(Cout), ldc,
            flags, _p(relu_mask), ld_mask, _p(bsum))


def sbr_nn_im2col(ctx, x, n, H, W, Cch, col):
    S._call("sbr_nn_im2col", ctx.h, _p(x), n, H, W, Cch, _p(col))


def sbr_nn_col2im(ctx, dcol, n, H, W, Cch, dx):
    S._call("sbr_nn_col2im", ctx.h, _p(dcol), n, H, W, Cch, _p(dx))


def sbr_nn_col2im_relu_backward(ctx, dcol, n, H, W, Cch, y, dz):
    S._call("sbr_nn_col2im_relu_backward", ctx.h, _p(dcol), n, H, W, Cch, _p(y), _p(dz))


def sbr_nn_fourier(ctx, x, n, D, Lb, emb, E, scene, Fw, out, extra=None, X=0):
    S._call("sbr_nn_fourier", ctx.h, _p(x), n, D, Lb, _p(emb), E, _p(scene), _p(extra), X, Fw, _p(out))


def sbr_nn_link_features(ctx, raw, n, scene, hmap, H, half, samples, x, extra):
    S._call("sbr_nn_link_features", ctx.h, _p(raw), n, _p(scene), _p(hmap), H, float(half), samples, _p(x), _p(extra))


def sbr_nn_relu_backward(ctx, g, y, n, gout=None, gbf=None):
    S._call("sbr_nn_relu_backward", ctx.h, _p(g), _p(y), n, _p(gout), _p(gbf))


def sbr_nn_cast_bf16(ctx, a, n, b):
    S._call("sbr_nn_cast_bf16", ctx.h, _p(a), n, _p(b))


def sbr_nn_mse(ctx, pred, ldp, target, weight, n, T, scale, dpred, ldd, loss):
    S._call("sbr_nn_mse", ctx.h, _p(pred), ldp, _p(target), _p(weight), n, T, float(scale), _p(dpred), ldd, _p(loss))


def sbr_nn_relu_backward_colsum(ctx, g, y, M, N, colsum, gout=None, gbf=None):
    S._call("sbr_nn_relu_backward_colsum", ctx.h, _p(g), _p(y), M, N, _p(gout), _p(gbf), _p(colsum))


def sbr_nn_colsum(ctx, g, M, N, ld, out, accumulate=0):
    S._call("sbr_nn_colsum", ctx.h, _p(g), M, N, ld, _p(out), accumulate)


def sbr_nn_adam(ctx, w, g, m, v, n, lr, b1, b2, eps, wd, step, wbf=None):
    S._call("sbr_nn_adam", ctx.h, _p(w), _p(g), _p(m), _p(v), n, float(lr), float(b1), float(b2), float(eps),
            float(wd), int(step), _p(wbf))


def sbr_nn_ensemble(ctx, out, E, member_stride, n, ld, t, threshold, mean, spread=None, mask=None):
    S._call("sbr_nn_ensemble", ctx.h, _p(out), E, member_stride, n, ld, t, float(threshold), _p(mean), _p(spread),
            _p(mask))


def sbr_nn_gather_rows(ctx, src, row_bytes, idx, n, dst):
    S._call("sbr_nn_gather_rows", ctx.h, _p(src), row_bytes, _p(idx), n, _p(dst))


def sbr_nn_onehot_bf16(ctx, idx, n, width, out):
    S._call("sbr_nn_onehot_bf16", ctx.h, _p(idx), n, width, _p(out))


def sbr_nn_mlp_infer(ctx, n, shared, emb, scene, wt, bias, depth, out_w, out_b, T, out):
    S._call("sbr_nn_mlp_infer", ctx.h, n, _p(shared), _p(emb), _p(scene), _p(wt), _p(bias), depth, _p(out_w),
            _p(out_b), T, _p(out))


def sbr_nn_transpose_bf16(ctx, src, rows, cols, dst):
    S._call("sbr_nn_transpose_bf16", ctx.h, _p(src), rows, cols, _p(dst))
