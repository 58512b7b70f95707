"""GPU: lco_permute_noalloc (no device allocation by the library; its workspace is a
fixed per-device array) equals lco_permute bit for bit, over consecutive calls whose
sizes and permutation methods differ, and rejects inputs beyond its maximum size."""
import numpy as np
import pytest

import lco_inputs as L
from conftest import gpu_create

pytestmark = pytest.mark.gpu


def _same_as_permute(lco_lib, ctx, t, perm):
    import torch
    ref = lco_lib.lco_permute(ctx, t, list(perm))
    livs = torch.empty(max(1, t.nnz), dtype=torch.int64, device="cuda")
    vals = torch.empty(max(1, t.nnz), dtype=torch.float64, device="cuda")
    livs.fill_(-1)
    vals.fill_(float("nan"))
    dims = lco_lib.lco_permute_noalloc(ctx, t, list(perm), livs, vals)
    ctx.synchronize()
    assert dims == list(ref.dims)
    n = t.nnz
    assert torch.equal(livs[:n], ref.livs())
    assert torch.equal(vals[:n].view(torch.int64), ref.vals().view(torch.int64))
    ref.destroy()


def test_noalloc_permute_consecutive_calls(lco_lib, gpu_ctx):
    rng = np.random.default_rng(20)
    # the largest input first, then smaller ones: what an earlier call left in the
    # workspace must not show up in a later one
    n = lco_lib.LCO_NOALLOC_MAX_NNZ
    dims = [64, 128, 32, 256]
    coords = np.unique(np.column_stack([rng.integers(0, d, n + n // 4) for d in dims]).astype(np.uint64), axis=0)
    coords = coords[rng.permutation(len(coords))[:n]]
    big = gpu_create(lco_lib, gpu_ctx, dims, coords, rng.uniform(-1, 1, len(coords)))
    assert big.nnz == n
    print("no-alloc permute: max-size random tensor (1,0,3,2), then a 3-D FD operator, then a 2-D one", flush=True)
    _same_as_permute(lco_lib, gpu_ctx, big, (1, 0, 3, 2))          # several LSD passes
    c, v = L.fd_laplacian(40, 3)
    fd = gpu_create(lco_lib, gpu_ctx, [40] * 6, c, v)
    _same_as_permute(lco_lib, gpu_ctx, fd, (4, 5, 3, 2, 0, 1))     # non-power-of-two dims, 64-bit shuffle
    c2, v2 = L.fd_laplacian(12, 2)
    fd2 = gpu_create(lco_lib, gpu_ctx, [12] * 4, c2, v2)
    _same_as_permute(lco_lib, gpu_ctx, fd2, (0, 2, 1, 3))          # common leading mode: segmented
    _same_as_permute(lco_lib, gpu_ctx, fd2, (2, 3, 0, 1))          # one tile in LDS
    for t in (fd2, fd, big):
        t.destroy()


def test_noalloc_permute_limits(lco_lib, gpu_ctx):
    import torch
    rng = np.random.default_rng(21)
    n = lco_lib.LCO_NOALLOC_MAX_NNZ + 1
    dims = [1 << 12, 1 << 12]
    coords = np.unique(np.column_stack([rng.integers(0, d, 2 * n) for d in dims]).astype(np.uint64), axis=0)[:n]
    t = gpu_create(lco_lib, gpu_ctx, dims, coords, rng.uniform(-1, 1, n))
    out_l = torch.empty(n, dtype=torch.int64, device="cuda")
    out_v = torch.empty(n, dtype=torch.float64, device="cuda")
    with pytest.raises(lco_lib.LcoError) as e:
        lco_lib.lco_permute_noalloc(gpu_ctx, t, [1, 0], out_l, out_v)
    assert e.value.code == 7  # LCO_E_UNSUPPORTED
    with pytest.raises(lco_lib.LcoError) as e:
        lco_lib.lco_permute_noalloc(gpu_ctx, t, [0, 0], out_l, out_v)
    assert e.value.code in (1, 7)
    t.destroy()
    empty = gpu_create(lco_lib, gpu_ctx, [5, 7], np.zeros((0, 2), np.uint64), np.zeros(0))
    assert lco_lib.lco_permute_noalloc(gpu_ctx, empty, [1, 0], out_l, out_v) == [7, 5]
    empty.destroy()
