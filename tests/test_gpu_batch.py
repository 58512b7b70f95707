"""GPU: batched contraction equals the per-call path bit for bit (and the oracle).

The batch mixes FD compositions of different grids and orders (the batched
path), products that need operand or output rearrangement, no-accumulator
instances, and instances that must fall back to the per-call path (outer
product, doubly compressed, long rows, empty operands).
"""
import numpy as np
import pytest

import lco_inputs as L
from conftest import gpu_create

pytestmark = pytest.mark.gpu


def np_of(t):
    d, l_, v = t.to_numpy()
    return d.tolist(), l_, v.view(np.uint64)


def test_batch_mixed_instances_equal_per_call(lco_lib, gpu_ctx, oracle_mod):
    rng = np.random.default_rng(4096)
    items, refs = [], []
    keep = []
    # FD compositions (batched, accumulator path)
    for side, dim in ((8, 2), (13, 2), (31, 2), (8, 3), (11, 3), (20, 3)):
        c, v = L.fd_laplacian(side, dim)
        g = gpu_create(lco_lib, gpu_ctx, [side] * (2 * dim), c, v)
        keep.append(g)
        la = list(range(2 * dim))
        lb = list(range(dim, 3 * dim))
        lc = list(range(dim)) + list(range(2 * dim, 3 * dim))
        items.append((g, la, g, lb, lc))
        o = oracle_mod.create([side] * (2 * dim), c, v)
        refs.append(oracle_mod.contract(o, la, o, lb, lc))
    # random products: rearranged operands and outputs, no-accumulator forced, fallbacks
    ca, va = L.random_sparse(rng, [9, 12, 7], 300)
    cb, vb = L.random_sparse(rng, [7, 12, 10], 300)
    ga, gb = gpu_create(lco_lib, gpu_ctx, [9, 12, 7], ca, va), gpu_create(lco_lib, gpu_ctx, [7, 12, 10], cb, vb)
    keep += [ga, gb]
    oa, ob = oracle_mod.create([9, 12, 7], ca, va), oracle_mod.create([7, 12, 10], cb, vb)
    for (la, lb, lc, flags) in (([0, 1, 2], [2, 1, 3], [0, 3], 0),
                                ([0, 1, 2], [2, 1, 3], [3, 0], 0),
                                ([0, 1, 2], [2, 1, 3], [0, 3], lco_lib.ALGO_IDS["CSRNA"]),
                                ([0, 1, 2], [2, 1, 3], [3, 0], lco_lib.ALGO_IDS["CSCNA"]),
                                ([0, 1, 2], [2, 1, 3], [0, 3], lco_lib.ALGO_IDS["DCSR"]),
                                ([0, 1, 2], [2, 1, 3], [0, 3], lco_lib.ALGO_IDS["SOP"]),
                                ([0, 1, 2], [3, 4, 5], [0, 1, 2, 3, 4, 5], 0)):
        items.append((ga, la, gb, lb, lc, flags))
        refs.append(oracle_mod.contract(oa, la, ob, lb, lc))
    # a long-row instance (falls back) and an empty one
    cl, vl = L.random_sparse(rng, [40, 200], 4000)
    cm, vm = L.random_sparse(rng, [200, 150], 6000)
    gl, gm = gpu_create(lco_lib, gpu_ctx, [40, 200], cl, vl), gpu_create(lco_lib, gpu_ctx, [200, 150], cm, vm)
    ge = gpu_create(lco_lib, gpu_ctx, [200, 150], np.zeros((0, 2), np.uint64), np.zeros(0))
    keep += [gl, gm, ge]
    ol, om = oracle_mod.create([40, 200], cl, vl), oracle_mod.create([200, 150], cm, vm)
    items.append((gl, [0, 1], gm, [1, 2], [0, 2]))
    refs.append(oracle_mod.contract(ol, [0, 1], om, [1, 2], [0, 2]))
    items.append((gl, [0, 1], ge, [1, 2], [0, 2]))
    refs.append(None)

    # a batch of fewer than 32 instances that the persistent engine could take runs in the chunked engine
    small = lco_lib.lco_contract_batch(gpu_ctx, items)
    b_small, p_small, q_small = lco_lib.lco_batch_stats(gpu_ctx)
    assert q_small == 0 and b_small >= 6
    for it, out in zip(items, small):
        single = lco_lib.lco_contract(gpu_ctx, *it[:5], it[5] if len(it) > 5 else 0)
        got, alone = np_of(out), np_of(single)
        assert np.array_equal(got[1], alone[1]) and np.array_equal(got[2], alone[2])
        single.destroy()
    for out in small:
        out.destroy()
    items, refs = items * 4, refs * 4  # enough instances for the persistent engine
    outs = lco_lib.lco_contract_batch(gpu_ctx, items)
    batched, per_call, persistent = lco_lib.lco_batch_stats(gpu_ctx)
    print(f"batched={batched} per_call={per_call} persistent={persistent}", flush=True)
    assert batched >= 24 and per_call >= 16  # FD compositions batch; long rows / DCSR / SOP fall back
    assert persistent >= 28  # the FD compositions and the long-row instance (sent on to the per-call path)
    for it, out, ref in zip(items, outs, refs):
        single = lco_lib.lco_contract(gpu_ctx, *it[:5], it[5] if len(it) > 5 else 0)
        got, alone = np_of(out), np_of(single)
        assert got[0] == alone[0]
        assert np.array_equal(got[1], alone[1]) and np.array_equal(got[2], alone[2])
        if ref is None:
            assert out.nnz == 0
        else:
            assert np.array_equal(got[1], ref.livs)
            assert np.array_equal(got[2], ref.vals.view(np.uint64))
        single.destroy()
    # outputs share one allocation; releasing them in any order is safe
    for out in outs[::2] + outs[1::2]:
        out.destroy()


def test_batch_mixed_column_widths(lco_lib, gpu_ctx, oracle_mod):
    """A batch in which one instance has 2^34 columns and the others fewer than
    2^32: the batched row kernels then check the width per row (64-bit hash keys
    for that instance, 32-bit table rows for the others).  Equal to per-call
    products and to the oracle bit for bit."""
    rng = np.random.default_rng(34)
    items, refs, keep = [], [], []
    for side, dim in ((9, 2), (12, 3)):
        c, v = L.fd_laplacian(side, dim)
        g = gpu_create(lco_lib, gpu_ctx, [side] * (2 * dim), c, v)
        keep.append(g)
        la, lb = list(range(2 * dim)), list(range(dim, 3 * dim))
        lc = list(range(dim)) + list(range(2 * dim, 3 * dim))
        items.append((g, la, g, lb, lc))
        o = oracle_mod.create([side] * (2 * dim), c, v)
        refs.append(oracle_mod.contract(o, la, o, lb, lc))
    da, db = [1 << 14, 1 << 14, 64], [64, 1 << 17, 1 << 17]
    heads = np.column_stack([rng.integers(0, da[0], 80), rng.integers(0, da[1], 80)]).astype(np.uint64)
    ca = np.unique(np.column_stack([heads[rng.integers(0, 80, 240)], rng.integers(0, 64, 240).astype(np.uint64)]),
                   axis=0)
    cb = np.column_stack([rng.integers(0, 64, 150), rng.integers(0, db[1], 150), rng.integers(0, db[2], 150)])
    cb = np.unique(cb.astype(np.uint64), axis=0)
    va, vb = rng.uniform(-1, 1, len(ca)), rng.uniform(-1, 1, len(cb))
    ga, gb = gpu_create(lco_lib, gpu_ctx, da, ca, va), gpu_create(lco_lib, gpu_ctx, db, cb, vb)
    keep += [ga, gb]
    # row by row (forced CSR), so that the wide side is the column side
    items.append((ga, [0, 1, 2], gb, [2, 3, 4], [0, 1, 3, 4], lco_lib.ALGO_IDS["CSR"]))
    refs.append(oracle_mod.contract(oracle_mod.create(da, ca, va), [0, 1, 2], oracle_mod.create(db, cb, vb),
                                    [2, 3, 4], [0, 1, 3, 4]))
    items, refs = items * 16, refs * 16
    outs = lco_lib.lco_contract_batch(gpu_ctx, items)
    batched, per_call, persistent = lco_lib.lco_batch_stats(gpu_ctx)
    print(f"batched={batched} per_call={per_call} persistent={persistent}", flush=True)
    # the wide instances' rows of A' are mostly empty: they run in the chunked engine
    assert batched == 48 and per_call == 0 and persistent == 32
    for it, out, ref in zip(items, outs, refs):
        single = lco_lib.lco_contract(gpu_ctx, *it[:5], it[5] if len(it) > 5 else 0)
        got, alone = np_of(out), np_of(single)
        assert got[0] == alone[0]
        assert np.array_equal(got[1], alone[1]) and np.array_equal(got[2], alone[2])
        assert np.array_equal(got[1], ref.livs) and np.array_equal(got[2], ref.vals.view(np.uint64))
        single.destroy()
    for out in outs:
        out.destroy()
    for t in keep:
        t.destroy()


def test_batch_many_small_fd(lco_lib, gpu_ctx, oracle_mod):
    """200 uneven 2-D / 3-D FD compositions (sides 4..24) in one batch: every result equals its
    closed-form size and the per-call result."""
    rng = np.random.default_rng(7)
    items, sizes = [], []
    for _ in range(200):
        dim = int(rng.integers(2, 4))
        side = int(rng.integers(4, 25 if dim == 2 else 13))
        c, v = L.fd_laplacian(side, dim)
        g = gpu_create(lco_lib, gpu_ctx, [side] * (2 * dim), c, v)
        items.append((g, list(range(2 * dim)), g, list(range(dim, 3 * dim)),
                      list(range(dim)) + list(range(2 * dim, 3 * dim))))
        s = side
        sizes.append(s * s + 4 * s * (s - 1) + 4 * (s - 1) ** 2 + 4 * s * (s - 2) if dim == 2 else
                     s**3 + 6 * s * s * (s - 1) + 12 * s * (s - 1) ** 2 + 6 * s * s * (s - 2))
    outs = lco_lib.lco_contract_batch(gpu_ctx, items)
    assert lco_lib.lco_batch_stats(gpu_ctx) == (200, 0, 200)
    for it, out, n in zip(items, outs, sizes):
        assert out.nnz == n
    for k in (0, 57, 199):
        single = lco_lib.lco_contract(gpu_ctx, *items[k])
        a, b = np_of(outs[k]), np_of(single)
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def _planned_items(lco_lib, gpu_ctx, rng):
    items, keep = [], []
    for side, dim in ((7, 2), (12, 2), (29, 2), (5, 3), (10, 3)):
        c, v = L.fd_laplacian(side, dim)
        g = gpu_create(lco_lib, gpu_ctx, [side] * (2 * dim), c, v)
        keep.append(g)
        items.append((g, list(range(2 * dim)), g, list(range(dim, 3 * dim)),
                      list(range(dim)) + list(range(2 * dim, 3 * dim))))
    # rows of at most 64 products (every instance of a plan runs batched)
    ca, va = L.random_sparse(rng, [40, 12, 7], 200)
    cb, vb = L.random_sparse(rng, [7, 12, 30], 200)
    ga, gb = gpu_create(lco_lib, gpu_ctx, [40, 12, 7], ca, va), gpu_create(lco_lib, gpu_ctx, [7, 12, 30], cb, vb)
    keep += [ga, gb]
    # operand rearrangement, output rearrangement, forced sort-based branches
    items += [(ga, [0, 1, 2], gb, [2, 1, 3], [0, 3]),
              (ga, [0, 1, 2], gb, [2, 1, 3], [3, 0]),
              (ga, [0, 1, 2], gb, [2, 1, 3], [0, 3], lco_lib.ALGO_IDS["CSRNA"]),
              (ga, [0, 1, 2], gb, [2, 1, 3], [3, 0], lco_lib.ALGO_IDS["CSCNA"])]
    return items, keep


def _check_plan_outputs(lco_lib, gpu_ctx, plan, items):
    for out, it in zip(plan.outputs(), items):
        single = lco_lib.lco_contract(gpu_ctx, *it[:5], it[5] if len(it) > 5 else 0)
        a, b = np_of(out), np_of(single)
        single.destroy()
        assert a[0] == b[0]
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_batch_plan_execute_and_graph_replays(lco_lib, gpu_ctx):
    """A planned batch equals per-call products; after the operands' values change in place,
    execute() and every replay of the captured graph equal per-call products on the new values."""
    rng = np.random.default_rng(99)
    items, keep = _planned_items(lco_lib, gpu_ctx, rng)
    plan = lco_lib.BatchPlan(gpu_ctx, items)
    try:
        info = plan.launches()
        print("launches", info, flush=True)
        assert info and all(x["branch"] in ("CSR", "CSRNA") for x in info)
        _check_plan_outputs(lco_lib, gpu_ctx, plan, items)
        for step, scale in enumerate((-1.5, 0.25, 3.0, -2.0)):
            for t in keep:
                t.vals().mul_(scale)
            if step == 0:
                plan.execute()
            else:
                plan.graph_launch()
            gpu_ctx.synchronize()
            _check_plan_outputs(lco_lib, gpu_ctx, plan, items)
    finally:
        plan.destroy()
    for t in keep:
        t.destroy()


def test_batch_plan_rejects_outer_product_and_entrywise(lco_lib, gpu_ctx):
    ops = []
    for seed in (1, 2):
        c, v = L.kronecker_hypersparse(5, 1 << 9, seed)
        ops.append(gpu_create(lco_lib, gpu_ctx, [32] * 4, c, v, lco_lib.LCO_COORDS | lco_lib.LCO_SUM_DUPLICATES))
    with pytest.raises(lco_lib.LcoError) as e:
        lco_lib.BatchPlan(gpu_ctx, [(ops[0], [0, 1, 2, 3], ops[1], [2, 3, 4, 5], [0, 1, 4, 5])])
    assert e.value.code == 7
    # an entrywise label (block-diagonal product) is not planned either
    with pytest.raises(lco_lib.LcoError) as e:
        lco_lib.BatchPlan(gpu_ctx, [(ops[0], [0, 1, 2, 3], ops[1], [0, 1, 2, 4], [0, 1, 3, 4])])
    assert e.value.code == 7
    for t in ops:
        t.destroy()


def test_batch_clustered_rows_with_fd_instances(lco_lib, gpu_ctx, oracle_mod):
    """A forced row-by-row (CSR) instance whose B' rows are the first and last 300
    of 2^22 -- about 4.2 million empty row pointers, written by whole waves in the
    batched pointer fill -- batched together with FD compositions: every output
    equals the per-call product and the oracle bit for bit."""
    rng = np.random.default_rng(92)
    items, refs, keep = [], [], []
    for side, dim in ((10, 2), (9, 3)):
        c, v = L.fd_laplacian(side, dim)
        g = gpu_create(lco_lib, gpu_ctx, [side] * (2 * dim), c, v)
        keep.append(g)
        la, lb = list(range(2 * dim)), list(range(dim, 3 * dim))
        lc = list(range(dim)) + list(range(2 * dim, 3 * dim))
        items.append((g, la, g, lb, lc))
        o = oracle_mod.create([side] * (2 * dim), c, v)
        refs.append(oracle_mod.contract(o, la, o, lb, lc))
    m, k, n = 512, 1 << 22, 40
    brows = np.concatenate([np.arange(300), np.arange(k - 300, k)])
    cb = np.array(sorted({(int(j), int(c)) for j in brows for c in rng.choice(n, 1 + int(j) % 3, replace=False)}),
                  dtype=np.uint64)
    vb = rng.uniform(-1, 1, len(cb))
    ca = np.array(sorted({(int(i), int(j)) for i in range(m) for j in rng.choice(brows, 4, replace=False)}),
                  dtype=np.uint64)
    va = rng.uniform(-1, 1, len(ca))
    ga, gb = gpu_create(lco_lib, gpu_ctx, [m, k], ca, va), gpu_create(lco_lib, gpu_ctx, [k, n], cb, vb)
    keep += [ga, gb]
    items.append((ga, [0, 1], gb, [1, 2], [0, 2], lco_lib.ALGO_IDS["CSR"]))
    refs.append(oracle_mod.contract(oracle_mod.create([m, k], ca, va), [0, 1], oracle_mod.create([k, n], cb, vb),
                                    [1, 2], [0, 2]))
    items.append(items[0])
    refs.append(refs[0])
    items, refs = items * 8, refs * 8
    outs = lco_lib.lco_contract_batch(gpu_ctx, items)
    batched, per_call, persistent = lco_lib.lco_batch_stats(gpu_ctx)
    print(f"batched={batched} per_call={per_call} persistent={persistent}", flush=True)
    assert batched == 32 and per_call == 0 and persistent == 32
    for it, out, ref in zip(items, outs, refs):
        single = lco_lib.lco_contract(gpu_ctx, *it[:5], it[5] if len(it) > 5 else 0)
        got, alone = np_of(out), np_of(single)
        assert np.array_equal(got[1], alone[1]) and np.array_equal(got[2], alone[2])
        assert np.array_equal(got[1], ref.livs) and np.array_equal(got[2], ref.vals.view(np.uint64))
        single.destroy()
    for out in outs:
        out.destroy()
    for t in keep:
        t.destroy()


@pytest.mark.slow
def test_batch_large_persistent_closed_form_and_oracle(lco_lib, gpu_ctx, oracle_mod):
    """A batch of 3-D and 2-D FD self-compositions with more than 2^26 A' entries
    in total (more than one chunk of the chunked engine holds), all in the
    persistent engine: every output of every instance equals the closed-form
    composed stencil (checked on the device); the first and last instance and
    the instances holding each eighth of the rows (where the work queues of
    the XCDs meet) equal the oracle bit for bit; a planned batch of the same
    instances gives the same outputs, also after a graph replay."""
    import torch
    from fd_closed_form import fd_square_matches
    inst = [(3, 40)] + [(3, 64)] * 36 + [(3, 40)] * 3 + [(2, 40 + (i % 21)) for i in range(30)] + \
        [(3, 64)] * 3 + [(3, 41)]
    distinct = {}
    for dim, side in sorted(set(inst)):
        c, v = L.fd_laplacian(side, dim)
        distinct[(dim, side)] = (gpu_create(lco_lib, gpu_ctx, [side] * (2 * dim), c, v), c, v)
    ops = []
    for dim, side in inst:  # every instance owns its operand
        src = distinct[(dim, side)][0]
        ops.append(lco_lib.lco_create(gpu_ctx, src.dims, src.livs(), src.vals(), lco_lib.LCO_SORTED))
    items = []
    for a, (dim, _) in zip(ops, inst):
        items.append((a, list(range(2 * dim)), a, list(range(dim, 3 * dim)),
                      list(range(dim)) + list(range(2 * dim, 3 * dim))))
    entries = sum(a.nnz for a in ops)
    assert entries > 1 << 26
    rows = np.cumsum([side ** dim for dim, side in inst])
    eighths = sorted({int(np.searchsorted(rows, rows[-1] * q // 8, side="right")) for q in range(1, 8)})
    print(f"large batch: {len(items)} instances, {entries} entries, queue splits in instances {eighths}",
          flush=True)
    outs = lco_lib.lco_contract_batch(gpu_ctx, items)
    assert lco_lib.lco_batch_stats(gpu_ctx) == (len(items), 0, len(items))
    torch.cuda.synchronize()
    for i, (out, (dim, side)) in enumerate(zip(outs, inst)):
        assert fd_square_matches(torch, out.livs(), out.vals(), side, dim), (i, dim, side)
    for i in sorted({0, len(items) - 1} | set(eighths)):
        dim, side = inst[i]
        _, c, v = distinct[(dim, side)]
        o = oracle_mod.create([side] * (2 * dim), c, v)
        ref = oracle_mod.contract(o, *items[i][1:2], o, *items[i][3:5])
        got = np_of(outs[i])
        print(f"oracle check of instance {i} ({dim}-D, side {side})", flush=True)
        assert np.array_equal(got[1], ref.livs) and np.array_equal(got[2], ref.vals.view(np.uint64)), i
    plan = lco_lib.BatchPlan(gpu_ctx, items)
    try:
        info = plan.launches()
        print("plan buckets", [(x["bucket"], x["instances"], x["branch"], x["chunks_per_item"]) for x in info],
              flush=True)
        assert sum(x["instances"] for x in info) == len(items)
        for i, p in enumerate(plan.outputs()):
            assert torch.equal(p.livs(), outs[i].livs()), i
            assert torch.equal(p.vals().view(torch.int64), outs[i].vals().view(torch.int64)), i
        for rep in range(2):
            plan.graph_launch()
            torch.cuda.synchronize()
            for i, p in enumerate(plan.outputs()):
                assert torch.equal(p.vals().view(torch.int64), outs[i].vals().view(torch.int64)), (rep, i)
    finally:
        plan.destroy()
    for out in outs:
        out.destroy()
    for a in ops:
        a.destroy()
    for g, _, _ in distinct.values():
        g.destroy()
