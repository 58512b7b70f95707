"""GPU parity: sparse addition (permute + merge) vs the CPU oracle.

LIVs and patterns must be bit-exact.  The values are too: both sides round
alpha*a and beta*b separately and add them once, so the bound of 1e-12 relative
per entry is met with equality.  Cases span several merge tiles with ragged
tails, ties that straddle tile boundaries, every kind of overlap (identical,
disjoint, nested, interleaved patterns), empty operands, order 0, and operands
brought into the output's mode order by a permutation (power-of-two and other
dimensions).
"""
import itertools

import numpy as np
import pytest

import lco_inputs as L
from conftest import gpu_create

pytestmark = pytest.mark.gpu

TILE = 2048  # entries of the merged sequence per tile


def same(gt, ot, what=""):
    d, livs, vals = gt.to_numpy()
    assert d.tolist() == ot.dims.tolist(), what
    assert livs.shape == ot.livs.shape, (what, livs.shape, ot.livs.shape)
    assert np.array_equal(livs, ot.livs), what
    assert np.array_equal(vals.view(np.uint64), ot.vals.view(np.uint64)), what


def both(lco, ctx, ora, dims, coords, vals):
    return gpu_create(lco, ctx, dims, coords, vals), ora.create(dims, coords, vals)


@pytest.mark.parametrize("alpha,beta", [(1.0, 1.0), (1.0, -1.0), (0.75, -2.5)])
def test_add_label_orders(lco_lib, gpu_ctx, oracle_mod, alpha, beta):
    """Order 4 with non-power-of-two dimensions: b and c in several mode orders
    (b permuted, a permuted, both, neither)."""
    rng = np.random.default_rng(21)
    dims = [5, 6, 7, 9]
    lab = [10, 11, 12, 13]
    ca, va = L.random_sparse(rng, dims, 1500)
    ga, oa = both(lco_lib, gpu_ctx, oracle_mod, dims, ca, va)
    perms = [(0, 1, 2, 3), (1, 0, 3, 2), (3, 2, 1, 0), (2, 0, 3, 1)]
    for pb in perms:
        bd = [dims[q] for q in pb]
        cb, _ = L.random_sparse(rng, bd, 1200)
        # about a third of b's entries coincide with entries of a (b's mode r is a's mode pb[r])
        take = rng.choice(len(ca), 500, replace=False)
        cb = np.unique(np.concatenate([cb, ca[take][:, list(pb)]]), axis=0)
        vb = rng.uniform(-1, 1, len(cb))
        gb, ob = both(lco_lib, gpu_ctx, oracle_mod, bd, cb, vb)
        for pc in perms:
            bl = [lab[q] for q in pb]
            cl = [lab[q] for q in pc]
            print(f"add b{pb} c{pc} alpha={alpha} beta={beta}", flush=True)
            gc = lco_lib.lco_add(gpu_ctx, ga, lab, gb, bl, cl, alpha, beta)
            same(gc, oracle_mod.add(oa, lab, ob, bl, cl, alpha, beta), f"{pb} {pc}")
            gc.destroy()
        gb.destroy()
    ga.destroy()


def _keys_case(name, n):
    """Two strictly increasing key sets of an order-1 tensor with dimension 4n + 8."""
    k = np.arange(n, dtype=np.uint64)
    if name == "identical":
        return 2 * k, 2 * k
    if name == "disjoint":
        return 2 * k, 2 * k + 1
    if name == "nested":  # b is every third key of a
        return k, 3 * k[: n // 3]
    if name == "multiples":  # ties every sixth key
        return 2 * k, 3 * k
    if name == "blocks":  # alternating runs of 100 from each side, with shared block edges
        a = np.concatenate([np.arange(200 * r, 200 * r + 101) for r in range(n // 200 + 1)]).astype(np.uint64)
        b = np.concatenate([np.arange(200 * r + 100, 200 * r + 201) for r in range(n // 200 + 1)]).astype(np.uint64)
        return a, b
    raise ValueError(name)


@pytest.mark.parametrize("name", ["identical", "disjoint", "nested", "multiples", "blocks"])
@pytest.mark.parametrize("n", [1, TILE // 2, TILE // 2 + 1, TILE - 1, 3 * TILE + 5, 20000])
def test_add_overlap_structures(lco_lib, gpu_ctx, oracle_mod, name, n):
    a, b = _keys_case(name, n)
    dim = int(4 * n + 8 + 600)
    rng = np.random.default_rng(n)
    va = rng.uniform(-1, 1, len(a))
    vb = rng.uniform(-1, 1, len(b))
    ga, oa = both(lco_lib, gpu_ctx, oracle_mod, [dim], a.reshape(-1, 1), va)
    gb, ob = both(lco_lib, gpu_ctx, oracle_mod, [dim], b.reshape(-1, 1), vb)
    print(f"add {name} n={n} na={len(a)} nb={len(b)}", flush=True)
    for alpha, beta in [(1.0, 1.0), (1.0, -1.0)]:
        gc = lco_lib.lco_add(gpu_ctx, ga, [0], gb, [0], [0], alpha, beta)
        same(gc, oracle_mod.add(oa, [0], ob, [0], [0], alpha, beta), name)
        gc.destroy()
    ga.destroy()
    gb.destroy()


def test_add_self_cancels_keeping_pattern(lco_lib, gpu_ctx, oracle_mod):
    rng = np.random.default_rng(8)
    dims = [64, 32, 16]
    c, v = L.random_sparse(rng, dims, 9000)
    ga, oa = both(lco_lib, gpu_ctx, oracle_mod, dims, c, v)
    gc = lco_lib.lco_add(gpu_ctx, ga, [0, 1, 2], ga, [0, 1, 2], [0, 1, 2], 1.0, -1.0)
    d, livs, vals = gc.to_numpy()
    assert np.array_equal(livs, oa.livs) and np.all(vals == 0.0)
    gc.destroy()
    # a + its own transpose over the first two modes needs square modes: use a permuted copy instead
    gt = lco_lib.lco_permute(gpu_ctx, ga, [2, 0, 1])
    ot = oracle_mod.permute(oa, [2, 0, 1])
    gc = lco_lib.lco_add(gpu_ctx, ga, [0, 1, 2], gt, [2, 0, 1], [1, 2, 0], 2.0, 0.5)
    same(gc, oracle_mod.add(oa, [0, 1, 2], ot, [2, 0, 1], [1, 2, 0], 2.0, 0.5))
    gc.destroy()
    gt.destroy()
    ga.destroy()


def test_add_empty_and_order_zero(lco_lib, gpu_ctx, oracle_mod):
    dims = [7, 5]
    e_g, e_o = both(lco_lib, gpu_ctx, oracle_mod, dims, np.zeros((0, 2), np.uint64), np.zeros(0))
    c = np.array([[1, 2], [6, 4], [0, 0]], dtype=np.uint64)
    v = np.array([1.5, -2.0, 0.0])
    x_g, x_o = both(lco_lib, gpu_ctx, oracle_mod, dims, c, v)
    for (ga, oa), (gb, ob) in [((e_g, e_o), (x_g, x_o)), ((x_g, x_o), (e_g, e_o)), ((e_g, e_o), (e_g, e_o))]:
        gc = lco_lib.lco_add(gpu_ctx, ga, [0, 1], gb, [0, 1], [0, 1], 3.0, -1.0)
        same(gc, oracle_mod.add(oa, [0, 1], ob, [0, 1], [0, 1], 3.0, -1.0))
        gc.destroy()
    # an empty operand in another mode order: nothing to permute
    et_g, et_o = both(lco_lib, gpu_ctx, oracle_mod, [5, 7], np.zeros((0, 2), np.uint64), np.zeros(0))
    gc = lco_lib.lco_add(gpu_ctx, x_g, [0, 1], et_g, [1, 0], [1, 0], 1.0, 1.0)
    same(gc, oracle_mod.add(x_o, [0, 1], et_o, [1, 0], [1, 0], 1.0, 1.0))
    gc.destroy()
    import torch

    def scalar(x):  # order 0: one entry with LIV 0
        idx = torch.zeros(1, dtype=torch.int64, device="cuda")
        v = torch.tensor([x], dtype=torch.float64, device="cuda")
        return (lco_lib.lco_create(gpu_ctx, [], idx, v, lco_lib.LCO_SORTED),
                oracle_mod.create([], np.zeros((1, 0), np.uint64), np.array([x])))

    s1_g, s1_o = scalar(1.5)
    s2_g, s2_o = scalar(2.25)
    gc = lco_lib.lco_add(gpu_ctx, s1_g, [], s2_g, [], [], 1.0, 1.0)
    same(gc, oracle_mod.add(s1_o, [], s2_o, [], [], 1.0, 1.0))
    assert gc.to_numpy()[2].tolist() == [3.75]
    gc.destroy()
    for t in (e_g, x_g, et_g, s1_g, s2_g):
        t.destroy()


def test_add_large_ragged(lco_lib, gpu_ctx, oracle_mod):
    """About 1.4 M entries per operand (hundreds of tiles, ragged tail), 64-bit
    LIVs with the product of the dimensions equal to 2^64, b permuted."""
    rng = np.random.default_rng(77)
    dims = [1 << 16] * 4
    n = 1_400_003
    ca = rng.integers(0, 1 << 16, size=(n, 4), dtype=np.uint64)
    ca = np.unique(ca, axis=0)
    cb = np.concatenate([ca[::3][:, [2, 3, 0, 1]], rng.integers(0, 1 << 16, size=(n // 2, 4), dtype=np.uint64)])
    cb = np.unique(cb, axis=0)
    va = rng.uniform(-1, 1, len(ca))
    vb = rng.uniform(-1, 1, len(cb))
    ga, oa = both(lco_lib, gpu_ctx, oracle_mod, dims, ca, va)
    gb, ob = both(lco_lib, gpu_ctx, oracle_mod, dims, cb, vb)
    print(f"add large na={len(ca)} nb={len(cb)}", flush=True)
    gc = lco_lib.lco_add(gpu_ctx, ga, [0, 1, 2, 3], gb, [2, 3, 0, 1], [0, 1, 2, 3], 1.0, -1.0)
    same(gc, oracle_mod.add(oa, [0, 1, 2, 3], ob, [2, 3, 0, 1], [0, 1, 2, 3], 1.0, -1.0))
    gc.destroy()
    ga.destroy()
    gb.destroy()


def test_add_errors(lco_lib, gpu_ctx):
    a = gpu_create(lco_lib, gpu_ctx, [2, 3], np.array([[0, 0]], np.uint64), np.array([1.0]))
    b = gpu_create(lco_lib, gpu_ctx, [3, 2], np.array([[0, 0]], np.uint64), np.array([1.0]))
    c = gpu_create(lco_lib, gpu_ctx, [2, 3, 1], np.array([[0, 0, 0]], np.uint64), np.array([1.0]))
    cases = [
        ((a, [0, 1], b, [0, 1], [0, 1]), 3),     # same labels, different dimensions
        ((a, [0, 1], b, [1, 2], [0, 1]), 1),     # label sets differ
        ((a, [0, 0], b, [0, 1], [0, 1]), 1),     # repeated label
        ((a, [0, 1], c, [0, 1, 2], [0, 1]), 1),  # different orders
    ]
    for (x, lx, y, ly, lc), code in cases:
        with pytest.raises(lco_lib.LcoError) as e:
            lco_lib.lco_add(gpu_ctx, x, lx, y, ly, lc)
        assert e.value.code == code
    ok = lco_lib.lco_add(gpu_ctx, a, [0, 1], b, [1, 0], [0, 1])
    assert ok.nnz == 1 and ok.to_numpy()[2].tolist() == [2.0]
    for t in (ok, a, b, c):
        t.destroy()
