"""The allocation-free encode (ae_encode_noalloc) against ae_encode through the
C ABI: the same latent codes, per-patch (min, r) and FP8 scales, bit for bit,
on two calls in a row (the second on a smaller grid, so stale contents of the
shared static scratch would show), and the size limit of the static scratch
reported before any work is queued."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2304_04781_amd import _lib as L

pytestmark = pytest.mark.gpu


def grid_of(shape):
    nz, ny, nx = shape
    return L.make_grid(nz, ny, nx, 20.0, 1e-3, 10, 0, 1.0, 1, 0)


def encode_both(net, shape, fmt, seed):
    st = W.smooth_random_state(4, *shape, seed=seed).astype(np.float32)
    ts = torch.tensor(st, device="cuda")
    P = (shape[0] // 8) * (shape[1] // 8) * (shape[2] // 8)
    dt = torch.int16 if fmt == L.LATENT_BF16 else torch.uint8
    out = []
    for fn in (L.ae_encode, L.ae_encode_noalloc):
        lat = torch.full((P, 32), 0x55, dtype=dt, device="cuda")
        meta = torch.full((P, 4, 2), float("nan"), dtype=torch.float32, device="cuda")
        qs = torch.full((P,), float("nan"), dtype=torch.float32, device="cuda") if fmt == L.LATENT_FP8 else None
        fn(net, grid_of(shape), ts, fmt, lat, meta, qs)
        torch.cuda.synchronize()
        out.append((lat.cpu().numpy(), meta.cpu().numpy(), None if qs is None else qs.cpu().numpy()))
    return out


@pytest.mark.parametrize("fmt", [L.LATENT_FP8, L.LATENT_BF16])
def test_noalloc_encode_equals_encode_twice(fmt):
    prm = W.ae_init(seed=4)
    flat = np.concatenate([np.asarray(prm[k], np.float32).ravel() for k in
                           ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")])
    net = L.ae_create(2048, 512, 32, flat, np.full(4, 1e-7))
    try:
        # a larger grid first (several 128-patch work-groups and a ragged last one),
        # then a smaller one that reuses the scratch the first call left behind
        for shape, seed in (((64, 48, 88), 11), ((16, 24, 40), 12)):
            print(f"noalloc encode fmt={fmt} shape={shape} seed={seed}", flush=True)
            (lat_a, meta_a, qs_a), (lat_b, meta_b, qs_b) = encode_both(net, shape, fmt, seed)
            assert np.array_equal(lat_a, lat_b)
            assert np.array_equal(meta_a.view(np.uint32), meta_b.view(np.uint32))
            assert np.isfinite(meta_b).all()
            if fmt == L.LATENT_FP8:
                assert np.array_equal(qs_a.view(np.uint32), qs_b.view(np.uint32))
                assert (qs_b > 0).all()
    finally:
        L.ae_destroy(net)


def test_noalloc_encode_rejects_grids_beyond_the_scratch():
    prm = W.ae_init(seed=4)
    flat = np.concatenate([np.asarray(prm[k], np.float32).ravel() for k in
                           ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")])
    net = L.ae_create(2048, 512, 32, flat, np.full(4, 1e-7))
    try:
        # 512 x 512 x 264 cells = 135168 patches > 131072: rejected on the host,
        # before anything reads the (deliberately small) buffers below
        small = torch.zeros(16, device="cuda")
        lat = torch.zeros(16, dtype=torch.uint8, device="cuda")
        with pytest.raises(L.WvError) as e:
            L.ae_encode_noalloc(net, grid_of((264, 512, 512)), small, L.LATENT_FP8, lat, small, small)
        assert e.value.code == -1
        assert "static scratch" in L.wv_last_error()
    finally:
        L.ae_destroy(net)
