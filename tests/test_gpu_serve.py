"""GPU: the continuous-batching server.  Every result equals the plain per-call result on the
same operands bit for bit (and the oracle), whether it ran alone or batched with others."""
import numpy as np
import pytest

import lco_inputs as L
from conftest import gpu_create

pytestmark = pytest.mark.gpu


def fd_item(lco, ctx, oracle_mod, side, dim):
    c, v = L.fd_laplacian(side, dim)
    g = gpu_create(lco, ctx, [side] * (2 * dim), c, v)
    la, lb = list(range(2 * dim)), list(range(dim, 3 * dim))
    lc = list(range(dim)) + list(range(2 * dim, 3 * dim))
    o = oracle_mod.create([side] * (2 * dim), c, v)
    return (g, la, g, lb, lc), oracle_mod.contract(o, la, o, lb, lc), [g]


def mixed_requests(lco, ctx, oracle_mod):
    reqs, refs, keep = [], [], []
    for side, dim in ((8, 2), (13, 2), (30, 2), (6, 3), (9, 3), (17, 3)):
        it, ref, k = fd_item(lco, ctx, oracle_mod, side, dim)
        reqs.append(it)
        refs.append(ref)
        keep += k
    # hyper-sparse pair (outer-product path) and a product needing operand and output rearrangement
    ops = []
    for seed in (1, 2):
        c, v = L.kronecker_hypersparse(5, 1 << 9, seed)
        ops.append((gpu_create(lco, ctx, [32] * 4, c, v, lco.LCO_COORDS | lco.LCO_SUM_DUPLICATES),
                    oracle_mod.create([32] * 4, c, v, sum_duplicates=True)))
    (ga, oa), (gb, ob) = ops
    keep += [ga, gb]
    reqs.append((ga, [0, 1, 2, 3], gb, [2, 3, 4, 5], [0, 1, 4, 5]))
    refs.append(oracle_mod.contract(oa, [0, 1, 2, 3], ob, [2, 3, 4, 5], [0, 1, 4, 5]))
    rng = np.random.default_rng(77)
    ca, va = L.random_sparse(rng, [9, 12, 7], 300)
    cb, vb = L.random_sparse(rng, [7, 12, 10], 300)
    gra, grb = gpu_create(lco, ctx, [9, 12, 7], ca, va), gpu_create(lco, ctx, [7, 12, 10], cb, vb)
    keep += [gra, grb]
    ora, orb = oracle_mod.create([9, 12, 7], ca, va), oracle_mod.create([7, 12, 10], cb, vb)
    reqs.append((gra, [0, 1, 2], grb, [2, 1, 3], [3, 0]))
    refs.append(oracle_mod.contract(ora, [0, 1, 2], orb, [2, 1, 3], [3, 0]))
    return reqs, refs, keep


def check_against(lco, ctx, reqs, refs, outs):
    for it, ref, out in zip(reqs, refs, outs):
        alone = lco.lco_contract(ctx, *it)
        _, la, va = alone.to_numpy()
        alone.destroy()
        _, lo, vo = out
        assert np.array_equal(lo, la)
        assert np.array_equal(vo.view(np.uint64), va.view(np.uint64))
        assert np.array_equal(lo, ref.livs)
        tol = 1e-12 * np.maximum(np.abs(ref.vals), ref.absum)
        assert np.all(np.abs(vo - ref.vals) <= tol)


def collect(srv, n):
    srv.drain()
    got = {}
    for r in srv.poll():
        assert r["status"] == 0, r
        got[r["ticket"]] = (r["out"].to_numpy(), r["batch_size"])
        r["out"].destroy()
    assert sorted(got) == list(range(n))
    return [got[i][0] for i in range(n)], [got[i][1] for i in range(n)]


def test_served_in_mix_equals_alone(lco_lib, gpu_ctx, oracle_mod):
    reqs, refs, keep = mixed_requests(lco_lib, gpu_ctx, oracle_mod)
    gpu_ctx.synchronize()
    srv = lco_lib.Server(0, workers=2, max_batch=64)
    try:
        for rep in range(3):  # the same requests three times, interleaved, in one burst
            for it in reqs:
                srv.submit(*it)
        outs, sizes = collect(srv, 3 * len(reqs))
    finally:
        srv.destroy()
    print("batch sizes", sizes, flush=True)
    assert max(sizes) > 1  # some requests did run batched
    for rep in range(3):
        check_against(lco_lib, gpu_ctx, reqs, refs, outs[rep * len(reqs):(rep + 1) * len(reqs)])
    for t in keep:
        t.destroy()


def test_plain_mode_and_tiny_budget(lco_lib, gpu_ctx, oracle_mod):
    reqs, refs, keep = mixed_requests(lco_lib, gpu_ctx, oracle_mod)
    gpu_ctx.synchronize()
    for kw in (dict(workers=1, plain=True), dict(workers=2, hbm_budget=1)):
        srv = lco_lib.Server(0, **kw)
        try:
            for it in reqs:
                srv.submit(*it)
            outs, sizes = collect(srv, len(reqs))
        finally:
            srv.destroy()
        assert max(sizes) == 1  # plain calls, or a budget that admits one request at a time
        check_against(lco_lib, gpu_ctx, reqs, refs, outs)
    for t in keep:
        t.destroy()


def test_continuous_batching_burst(lco_lib, gpu_ctx):
    """A burst of 300 small requests on one worker: the worker takes what arrived while it was
    busy, so later batches hold many requests; all results are the expected sizes."""
    items = []
    keep = []
    for side in range(8, 28):
        c, v = L.fd_laplacian(side, 2)
        g = gpu_create(lco_lib, gpu_ctx, [side] * 4, c, v)
        keep.append((g, side))
    gpu_ctx.synchronize()
    srv = lco_lib.Server(0, workers=1, max_batch=128)
    sizes = []
    try:
        tickets = []
        for k in range(300):
            g, side = keep[k % len(keep)]
            tickets.append((srv.submit(g, [0, 1, 2, 3], g, [2, 3, 4, 5], [0, 1, 4, 5]), side))
        srv.drain()
        res = {r["ticket"]: r for r in srv.poll()}
        for t, s in tickets:
            r = res[t]
            assert r["status"] == 0
            assert r["out"].nnz == s * s + 4 * s * (s - 1) + 4 * (s - 1) ** 2 + 4 * s * (s - 2)
            sizes.append(r["batch_size"])
            r["out"].destroy()
    finally:
        srv.destroy()
    print("max batch", max(sizes), "batches", len(set(sizes)), flush=True)
    assert max(sizes) > 8
    for g, _ in keep:
        g.destroy()


def test_submit_errors(lco_lib, gpu_ctx):
    c, v = L.fd_laplacian(6, 2)
    g = gpu_create(lco_lib, gpu_ctx, [6] * 4, c, v)
    srv = lco_lib.Server(0, workers=1)
    try:
        with pytest.raises(lco_lib.LcoError):
            srv.submit(g, [0, 1, 2, 3], g, [2, 3, 4, 5], [0, 1, 4])  # summed free label 5
        t = srv.submit(g, [0, 1, 2, 3], g, [2, 3, 4, 5], [0, 1, 4, 5])
        srv.drain()
        r = srv.poll()
        assert len(r) == 1 and r[0]["ticket"] == t and r[0]["status"] == 0
        r[0]["out"].destroy()
    finally:
        srv.destroy()
    with pytest.raises(lco_lib.LcoError):
        lco_lib.Server(0, workers=0)
    g.destroy()
