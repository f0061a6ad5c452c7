"""The allocation-free capacity entry point (for callers that cannot
allocate device memory) against sbr_capacity, through the C-ABI: the same
values on two calls in a row, the second smaller than the first, and its
size limits rejected before any work is queued."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _h(shape, seed, scale=1e-5):
    rng = np.random.default_rng(seed)
    return ((rng.normal(size=shape) + 1j * rng.normal(size=shape)) * scale).astype(np.complex64)


@pytest.mark.parametrize("normalize", [1, 0])
def test_noalloc_capacity_matches_capacity(normalize):
    import torch
    from paper_2208_10006_amd import sbr as S
    ctx = S.Context(0)
    dev = torch.device("cuda", 0)
    snr = np.arange(0, 31, 5, dtype=np.float64)
    out = torch.full((64,), np.nan, dtype=torch.float64, device=dev)
    scale = 1e-5 if normalize else 1.0
    # each call is smaller than the one before it and has fewer SNR values;
    # the second takes the 128-wide elimination (64 < min(Nr, Nt) <= 128)
    for shape, ns, seed in [((48, 64, 256), 7, 1), ((16, 100, 128), 5, 3), ((5, 8, 3), 3, 2)]:
        banner("capacity noalloc", shape, ns, "normalize", normalize)
        H = _h(shape, seed, scale)
        ref = S.sbr_capacity(ctx, H, snr[:ns], normalize=normalize)
        Hd = torch.as_tensor(H).to(dev)
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        S.sbr_capacity_noalloc(ctx, Hd, snr[:ns], out, normalize=normalize)
        S.sbr_synchronize(ctx)
        got = out[:ns].cpu().numpy()
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12), (shape, got, ref)
        # nothing beyond the Nsnr outputs is written
        assert np.all(np.isnan(out[ns:].cpu().numpy()))


def test_noalloc_capacity_limits():
    import torch
    from paper_2208_10006_amd import sbr as S
    ctx = S.Context(0)
    dev = torch.device("cuda", 0)
    out = torch.zeros(70, dtype=torch.float64, device=dev)
    banner("capacity noalloc limits")
    for shape, ns in [((2, 129, 130), 3), ((2, 8, 8), 65), ((200000, 2, 2), 7)]:
        Hd = torch.zeros(shape, dtype=torch.complex64, device=dev)
        with pytest.raises(S.SbrError) as e:
            S.sbr_capacity_noalloc(ctx, Hd, np.zeros(ns), out)
        assert e.value.status == -4, e.value
