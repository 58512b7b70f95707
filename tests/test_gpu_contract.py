"""GPU parity: contraction (every algorithm of the poly-algorithm) vs the CPU oracle.

Indices and sparsity patterns must be bit-exact.  FP64 values must agree to
1e-12 relative per entry; where an entry's terms cancel (|c| < 1e-3 * sum|terms|)
the bound is 1e-12 * sum|terms|.  Integer-valued inputs (the FD operators) must
be bit-exact, and so must every case where both sides sum in the same order
(ascending contracted index in the first operand's mode order, from 0.0).
"""
import itertools

import numpy as np
import pytest

import lco_inputs as L
from conftest import gpu_create

pytestmark = pytest.mark.gpu

FORCED = ["CSC", "CSR", "DCSC", "DCSR", "CSCNA", "CSRNA", "SOP"]
TOL = 1e-12


@pytest.fixture(scope="module")
def paper_ctx(lco_lib):
    """A context whose selector is the paper's table as is."""
    c = lco_lib.lco_ctx_create(0)
    lco_lib.lco_ctx_use_paper_selector(c)
    yield c
    c.destroy()


def to_np(t):
    d, livs, vals = t.to_numpy()
    return d, livs, vals


def check(gt, ot, exact=False, what=""):
    d, livs, vals = to_np(gt)
    assert d.tolist() == ot.dims.tolist(), what
    assert livs.shape == ot.livs.shape, (what, livs.shape, ot.livs.shape)
    assert np.array_equal(livs, ot.livs), what
    if exact:
        assert np.array_equal(vals.view(np.uint64), ot.vals.view(np.uint64)), what
        return
    err = np.abs(vals - ot.vals)
    cancel = np.abs(ot.vals) < 1e-3 * ot.absum
    bound = np.where(cancel, TOL * ot.absum, TOL * np.abs(ot.vals))
    bad = err > bound
    assert not bad.any(), (what, int(bad.sum()), float(err.max()))


def pair(lco, ctx, ora, dims, coords, vals):
    return gpu_create(lco, ctx, dims, coords, vals), ora.create(dims, coords, vals)


def run_all(lco, ctx, ora, ga, oa, la, gb, ob, lb, lc, exact=False, algos=("auto",) + tuple(FORCED)):
    ref = ora.contract(oa, la, ob, lb, lc)
    first = None
    for name in algos:
        flags = 0 if name == "auto" else lco.ALGO_IDS[name]
        print(f"contract {la}x{lb}->{lc} algo={name} nnz={oa.nnz},{ob.nnz}", flush=True)
        gc = lco.lco_contract(ctx, ga, la, gb, lb, lc, flags)
        check(gc, ref, exact, f"{name} {la} {lb} {lc}")
        if first is None:
            first = to_np(gc)
        gc.destroy()
    return ref


# ---------------------------------------------------------------- small FD config
def test_small_fd_config_all_algorithms(lco_lib, gpu_ctx, oracle_mod):
    """32x32 grid operator composed with itself over modes (3,4)x(1,2): 12,676 entries, exact,
    and equal to the dense 1024x1024 matrix product."""
    c, v = L.fd_laplacian(32, 2)
    g, o = pair(lco_lib, gpu_ctx, oracle_mod, [32] * 4, c, v)
    plan = lco_lib.lco_plan_info(gpu_ctx, g, [0, 1, 2, 3], g, [2, 3, 4, 5], [0, 1, 4, 5])
    assert lco_lib.ALGOS[plan.algo] == "CSC" and plan.permute_a + plan.permute_b + plan.permute_c == 0
    ref = run_all(lco_lib, gpu_ctx, oracle_mod, g, o, [0, 1, 2, 3], g, o, [2, 3, 4, 5], [0, 1, 4, 5], exact=True)
    assert ref.nnz == 12676
    M = np.zeros((1024, 1024))
    M[(c[:, 0] + 32 * c[:, 1]).astype(int), (c[:, 2] + 32 * c[:, 3]).astype(int)] = v
    gc = lco_lib.lco_contract(gpu_ctx, g, [0, 1, 2, 3], g, [2, 3, 4, 5], [0, 1, 4, 5])
    _, livs, vals = to_np(gc)
    D = np.zeros_like(M)
    D[(livs % 1024).astype(int), (livs // 1024).astype(int)] = vals
    assert np.array_equal(D, M @ M)


# ---------------------------------------------------------------- all index matchings
def matchings(n):
    out = []
    for i in range(n + 1):
        for sa in itertools.combinations(range(n), i):
            for sb in itertools.permutations(range(n), i):
                out.append(list(zip(sa, sb)))
    return out


@pytest.mark.parametrize("n", [2, 3])
def test_all_matchings_every_algorithm(lco_lib, gpu_ctx, oracle_mod, n):
    rng = np.random.default_rng(40 + n)
    for mi, match in enumerate(matchings(n)):
        dims_a = [int(x) for x in rng.integers(2, 7, n)]
        dims_b = [int(x) for x in rng.integers(2, 7, n)]
        for (ia, ib) in match:
            dims_b[ib] = dims_a[ia]
        ca, va = L.random_sparse(rng, dims_a, 30, integer_values=True)
        cb, vb = L.random_sparse(rng, dims_b, 30, integer_values=True)
        ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, dims_a, ca, va)
        gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, dims_b, cb, vb)
        la = list(range(n))
        lb = [n + j for j in range(n)]
        for (ia, ib) in match:
            lb[ib] = la[ia]
        lc = [la[i] for i in range(n) if i not in {x for x, _ in match}] + \
             [lb[j] for j in range(n) if j not in {y for _, y in match}]
        if mi % 3 == 1:
            lc = lc[::-1]
        elif mi % 3 == 2 and len(lc) > 2:
            lc = lc[1:] + lc[:1]
        run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, la, gb, ob, lb, lc, exact=True)
        ga.destroy()
        gb.destroy()


@pytest.mark.parametrize("n", [2, 3])
def test_entrywise_matchings_every_algorithm(lco_lib, gpu_ctx, oracle_mod, n):
    """Every matching of the modes of two order-n tensors with at least one pair
    entrywise (in a, b and the output): every algorithm, several output orders."""
    import itertools
    rng = np.random.default_rng(60 + n)
    k = 0
    for match in matchings(n):
        for roles in itertools.product((0, 1), repeat=len(match)):
            if not any(roles):
                continue
            dims_a = [int(x) for x in rng.integers(2, 7, n)]
            dims_b = [int(x) for x in rng.integers(2, 7, n)]
            for (ia, ib) in match:
                dims_b[ib] = dims_a[ia]
            ca, va = L.random_sparse(rng, dims_a, 40, integer_values=True)
            cb, vb = L.random_sparse(rng, dims_b, 40, integer_values=True)
            ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, dims_a, ca, va)
            gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, dims_b, cb, vb)
            la = list(range(n))
            lb = [n + j for j in range(n)]
            for (ia, ib) in match:
                lb[ib] = la[ia]
            role = {ia: r for (ia, _), r in zip(match, roles)}
            lc = [la[i] for i in range(n) if role.get(i, 1) == 1] + \
                 [lb[j] for j in range(n) if j not in {y for _, y in match}]
            k += 1
            if k % 3 == 1:
                lc = lc[::-1]
            elif k % 3 == 2 and len(lc) > 2:
                lc = lc[1:] + lc[:1]
            run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, la, gb, ob, lb, lc, exact=True)
            ga.destroy()
            gb.destroy()


def test_entrywise_batched_matrix_products(lco_lib, gpu_ctx, oracle_mod):
    """c_hik = a_hij b_hjk: 48 sparse 60x50 by 50x40 products at once (random FP64,
    several tiles), the Hadamard product c_ij = a_ij b_ij, per-batch dot products
    c_h = a_hi b_hi, and the batch label in other positions and output orders."""
    rng = np.random.default_rng(77)
    H, I_, J_, K_ = 48, 60, 50, 40
    ca, va = L.random_sparse(rng, [H, I_, J_], 20000)
    cb, vb = L.random_sparse(rng, [H, J_, K_], 20000)
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, [H, I_, J_], ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, [H, J_, K_], cb, vb)
    plan = lco_lib.lco_plan_info(gpu_ctx, ga, [0, 1, 2], gb, [0, 2, 3], [0, 1, 3])
    assert plan.num_entrywise == 1 and plan.num_contracted == 1
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1, 2], gb, ob, [0, 2, 3], [0, 1, 3])
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1, 2], gb, ob, [0, 2, 3], [3, 1, 0])
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1, 2], gb, ob, [0, 2, 3], [1, 3, 0])
    # the batch mode last in a, first in b
    gt = lco_lib.lco_permute(gpu_ctx, ga, [1, 2, 0])
    ot = oracle_mod.permute(oa, [1, 2, 0])
    run_all(lco_lib, gpu_ctx, oracle_mod, gt, ot, [1, 2, 0], gb, ob, [0, 2, 3], [1, 3, 0])
    # Hadamard product (nothing contracted) and dot products per batch index
    cx, vx = L.random_sparse(rng, [H, I_], 1500)
    cy, vy = L.random_sparse(rng, [H, I_], 1500)
    gx, ox = pair(lco_lib, gpu_ctx, oracle_mod, [H, I_], cx, vx)
    gy, oy = pair(lco_lib, gpu_ctx, oracle_mod, [H, I_], cy, vy)
    run_all(lco_lib, gpu_ctx, oracle_mod, gx, ox, [0, 1], gy, oy, [0, 1], [0, 1])
    run_all(lco_lib, gpu_ctx, oracle_mod, gx, ox, [0, 1], gy, oy, [0, 1], [0])
    gyt = lco_lib.lco_permute(gpu_ctx, gy, [1, 0])
    run_all(lco_lib, gpu_ctx, oracle_mod, gx, ox, [0, 1], gyt, oracle_mod.permute(oy, [1, 0]), [1, 0], [1, 0])
    # a batch of instances with an entrywise label runs per call, bit-identical
    outs = lco_lib.lco_contract_batch(gpu_ctx, [(ga, [0, 1, 2], gb, [0, 2, 3], [0, 1, 3]),
                                                (gx, [0, 1], gy, [0, 1], [0])])
    one = lco_lib.lco_contract(gpu_ctx, ga, [0, 1, 2], gb, [0, 2, 3], [0, 1, 3])
    assert np.array_equal(outs[0].to_numpy()[1], one.to_numpy()[1])
    assert np.array_equal(outs[0].to_numpy()[2].view(np.uint64), one.to_numpy()[2].view(np.uint64))
    for t in outs + [one, ga, gb, gt, gx, gy, gyt]:
        t.destroy()


# ---------------------------------------------------------------- random FP64, multi-tile
@pytest.mark.parametrize("seed", [0, 1])
def test_random_fp64_every_algorithm(lco_lib, gpu_ctx, oracle_mod, seed):
    rng = np.random.default_rng(seed)
    dims_a, dims_b = [30, 40, 25], [25, 40, 35]
    ca, va = L.random_sparse(rng, dims_a, 9000)
    cb, vb = L.random_sparse(rng, dims_b, 9000)
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, dims_a, ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, dims_b, cb, vb)
    # a_ijk b_kjl -> c_il : contracted (j, k) in a's order -> bit-exact against the oracle
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1, 2], gb, ob, [2, 1, 3], [0, 3], exact=True)
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1, 2], gb, ob, [2, 1, 3], [3, 0], exact=True)


def test_long_rows_global_path(lco_lib, gpu_ctx, oracle_mod):
    """Rows with more than 64 products (about 3000 here: the in-LDS sort of up to 4096)."""
    rng = np.random.default_rng(9)
    ca, va = L.random_sparse(rng, [60, 300], 6000)
    cb, vb = L.random_sparse(rng, [300, 200], 9000)
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, [60, 300], ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, [300, 200], cb, vb)
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, [1, 2], [0, 2], exact=True)
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, [1, 2], [2, 0], exact=True)


@pytest.mark.parametrize("wide", [False, True])
def test_long_rows_every_bin(lco_lib, gpu_ctx, oracle_mod, wide):
    """Long rows in every bin of the long-row paths: in-LDS sorts of up to 256,
    1024 and 4096 products, and the global sort above that (rows of about 4500
    and 12000 products), beside rows of more than 64 entries with few or no
    products.  Row 0 of B has 2500 entries: a doubly compressed B' finds its end
    by a galloping search across many windows of 64 entries.  With 2^52 or more columns the (column, product) keys no longer
    fit 63 bits and every long row takes the global sort."""
    rng = np.random.default_rng(123)
    m, k = 240, 2000
    dims_b = [k, 1 << 26, 1 << 27] if wide else [k, 3000]
    ncols = int(np.prod(dims_b[1:], dtype=np.float64)) if not wide else None
    b_rows = []
    for j in range(k):
        if j % 10 == 9:
            continue  # empty rows of B
        ln = 2500 if j == 0 else int(rng.integers(1, 61))  # row 0: a doubly compressed row over 39 windows
        if wide:
            cols = np.unique(rng.integers(0, 1 << 20, ln)) * np.uint64(1 << 33) + np.uint64(j % 7)
        else:
            cols = rng.choice(ncols, ln, replace=False)
        b_rows += [(j, int(c)) for c in cols]
    nb = np.array(b_rows, dtype=np.uint64)
    if wide:  # column c -> coordinates (c mod 2^26, c div 2^26)
        cb = np.stack([nb[:, 0], nb[:, 1] % np.uint64(1 << 26), nb[:, 1] // np.uint64(1 << 26)], axis=1)
    else:
        cb = nb
    vb = rng.integers(-3, 4, len(cb)).astype(np.float64)
    vb[vb == 0] = 0.5
    empty = np.array([j for j in range(k) if j % 10 == 9])
    a_rows = []
    for i in range(m):
        t = [2, 5, 20, 60, 150, 400, 90][i % 7]
        if i % 7 == 6:  # many entries, most of them selecting empty rows of B
            full = np.setdiff1d(np.arange(k), empty)
            cols = np.concatenate([rng.choice(empty, t - 5, replace=False), rng.choice(full, 5, replace=False)])
        else:
            cols = rng.choice(k, t, replace=False)
        a_rows += [(i, int(c)) for c in cols]
    ca = np.array(a_rows, dtype=np.uint64)
    va = rng.uniform(-1, 1, len(ca))
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, [m, k], ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, dims_b, cb, vb)
    lb = [1, 2] if not wide else [1, 2, 3]
    lc = [0, 2] if not wide else [0, 2, 3]
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, lb, lc, exact=True,
            algos=("auto", "CSR", "DCSR", "CSRNA", "CSC", "DCSC"))
    for t in (ga, gb):
        t.destroy()


def _colliding_columns(n_cols, wide, slot, count, rng):
    """`count` distinct columns below n_cols that the row passes' LDS hash sends to
    one home slot: Fibonacci hashing of the column (32-bit product for columns
    below 2^32, 64-bit otherwise), top 7 bits."""
    out = np.zeros(0, dtype=np.uint64)
    while len(out) < count:
        c = np.unique(rng.integers(0, n_cols, 1 << 16, dtype=np.uint64))
        if wide:
            h = (c * np.uint64(0x9E3779B97F4A7C15)) >> np.uint64(57)
        else:
            h = ((c * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)) >> np.uint64(25)
        out = np.union1d(out, c[h == np.uint64(slot)])
    return rng.permutation(out)[:count]


@pytest.mark.parametrize("wide", [False, True])
def test_row_hash_collisions(lco_lib, gpu_ctx, oracle_mod, wide):
    """Rows whose columns all share one home slot of the row passes' 128-slot LDS
    hash (and rows that mix two neighbouring home slots), so that probe runs
    reach 64 slots: table rows of 2 and 7 entries (up to 64 distinct columns),
    rows of 16 entries, search-shaped rows, and entries that repeat each other's
    columns (lanes holding one column probe in lockstep and exactly one inserts
    it).  Exact against the oracle under CSR, DCSR, CSRNA and the automatic
    choice; with 2^40 columns the hash is the 64-bit one and no row is a table
    row."""
    rng = np.random.default_rng(2024 + int(wide))
    n_cols = (1 << 40) if wide else (1 << 20)
    s5 = _colliding_columns(n_cols, wide, 5, 64, rng)
    s6 = _colliding_columns(n_cols, wide, 6, 32, rng)
    b_rows = {
        0: s5[0:32], 1: s5[16:48], 2: s5[32:64], 3: np.concatenate([s6[0:16], s5[0:16]]),
    }
    for j in range(4, 12):  # rows of 8, overlapping by half
        b_rows[j] = s5[4 * (j - 4):4 * (j - 4) + 8]
    for j in range(12, 28):  # rows of 4
        b_rows[j] = np.concatenate([s5[2 * (j - 12):2 * (j - 12) + 2], s6[2 * (j - 12) % 32:2 * (j - 12) % 32 + 2]])
    both = np.concatenate([s5, s6])
    for j, ln in zip(range(28, 33), (20, 3, 17, 1, 23)):  # uneven rows: the search shape
        b_rows[j] = rng.choice(both, ln, replace=False)
    k = 40
    cb = np.array([(j, int(c)) for j in sorted(b_rows) for c in np.sort(b_rows[j])], dtype=np.uint64)
    vb = rng.uniform(-1, 1, len(cb))
    a_sets = [[0, 1], [0, 2], [1, 3], [2, 3], list(range(4, 11)), list(range(12, 28)), list(range(28, 33)),
              [0], [3, 30], list(range(4, 12)) + [0]]
    ca = np.array([(i, j) for i, js in enumerate(a_sets) for j in js], dtype=np.uint64)
    va = rng.uniform(-1, 1, len(ca))
    if wide:  # column c -> coordinates (c mod 2^20, c div 2^20)
        dims_b = [k, 1 << 20, 1 << 20]
        cbc = np.stack([cb[:, 0], cb[:, 1] % np.uint64(1 << 20), cb[:, 1] // np.uint64(1 << 20)], axis=1)
        lb, lc = [1, 2, 3], [0, 2, 3]
    else:
        dims_b = [k, n_cols]
        cbc = cb
        lb, lc = [1, 2], [0, 2]
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, [len(a_sets), k], ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, dims_b, cbc, vb)
    ref = run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, lb, lc, exact=True,
                  algos=("auto", "CSR", "DCSR", "CSRNA"))
    assert ref.nnz == sum(len(np.unique(np.concatenate([b_rows[j] for j in js]))) for js in a_sets)
    for t in (ga, gb):
        t.destroy()


def test_row_classes_mixed(lco_lib, gpu_ctx, oracle_mod):
    """Every row class of the row engine in one product: single-entry rows whose
    B' row is short or long (more than 64 products: the scaled-copy class),
    rows of 2-4 entries with at most 16 products (one lane per row), rows of the
    one-wave classes, and long rows; values include signed zeros (an output of
    one product -0.0 must come out +0.0, as a sum started from 0.0)."""
    rng = np.random.default_rng(31)
    m, k, n = 400, 120, 700
    b_rows = []
    for j in range(k):
        ln = [1, 2, 3, 5, 9, 17, 40, 70, 150][j % 9]
        cols = rng.choice(n, ln, replace=False)
        b_rows += [(j, c) for c in cols]
    cb = np.array(b_rows, dtype=np.uint64)
    vb = rng.integers(-3, 4, len(cb)).astype(np.float64)
    vb[vb == 0] = -0.0
    a_rows = []
    for i in range(m):
        t = [1, 1, 2, 3, 4, 6, 30][i % 7]
        cols = rng.choice(k, t, replace=False)
        a_rows += [(i, c) for c in cols]
    ca = np.array(a_rows, dtype=np.uint64)
    va = rng.integers(-2, 3, len(ca)).astype(np.float64)
    va[va == 0] = 0.5
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, [m, k], ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, [k, n], cb, vb)
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, [1, 2], [0, 2], exact=True)
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, [1, 2], [2, 0], exact=True)
    # outer products: every row is one entry times the other operand's only row
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, [2, 3], [0, 1, 2, 3], exact=True,
            algos=("auto", "CSR", "CSC", "CSRNA", "DCSR"))
    for t in (ga, gb):
        t.destroy()


def test_dense_rows_with_empty_rows(lco_lib, gpu_ctx, oracle_mod):
    """A' with at most twice as many rows as entries takes its row starts over all
    rows: here every third row is empty and so are the last 100 (and the last row),
    with more than 16384 entries (not the one-block setup)."""
    rng = np.random.default_rng(55)
    m, k, n = 9000, 300, 400
    rows = [i for i in range(m - 100) if i % 3]
    ca = np.array([(i, int(c)) for i in rows for c in rng.choice(k, 3, replace=False)], dtype=np.uint64)
    va = rng.integers(-3, 4, len(ca)).astype(np.float64)
    va[va == 0] = 1.0
    cb, vb = L.random_sparse(rng, [k, n], 2400, integer_values=True)
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, [m, k], ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, [k, n], cb, vb)
    assert m <= 2 * len(ca) and len(ca) > 16384
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, [1, 2], [0, 2], exact=True,
            algos=("auto", "CSR", "CSRNA", "DCSR"))
    for t in (ga, gb):
        t.destroy()


@pytest.mark.parametrize("lc", [[0, 2], [2, 0]])
def test_many_entry_rows_and_row_table(lco_lib, gpu_ctx, oracle_mod, lc):
    """Rows of more than 64 entries (up to 700; their product counts are summed
    by a whole wave), some of which select only empty rows of the other operand
    and so have no products, in 300 rows (a ragged last wave).  The contracted
    index has 2^20 values and few non-empty rows, so a doubly compressed operand
    is located through its hash table of row ids: clustered rows (long probe
    runs), rows at both ends of the range, and absent rows.  B has a column of
    150 entries, a many-entry row of the column-wise orientation."""
    rng = np.random.default_rng(77)
    m, k, n = 300, 1 << 20, 500
    brows = np.unique(np.concatenate([np.arange(200), [k - 1, k - 2, k - 5000], rng.integers(0, k, 300)]))
    bset = set(int(j) for j in brows)
    cb = {(int(j), int(c)) for j in brows for c in rng.choice(n, 1 + int(j) % 3, replace=False)}
    cb |= {(int(j), 7) for j in brows[:150]}
    cb = np.array(sorted(cb), dtype=np.uint64)
    vb = rng.integers(-4, 5, len(cb)).astype(np.float64)
    vb[vb == 0] = 0.25
    absent = [j for j in range(200, 2048)] + [k - 3, k - 4, k - 4999] + [int(j) for j in rng.integers(0, k, 3000)]
    absent = np.array(sorted(set(absent) - bset), dtype=np.uint64)
    a_rows = []
    for i in range(m):
        t = [1, 3, 64, 65, 100, 257, 700][i % 7]
        if i % 13 == 5:  # every column selects an empty row of B
            cols = rng.choice(absent, t, replace=False)
        else:
            h = t // 2
            cols = np.concatenate([rng.choice(brows, t - h, replace=False), rng.choice(absent, h, replace=False)])
        a_rows += [(i, int(c)) for c in cols]
    ca = np.array(a_rows, dtype=np.uint64)
    va = rng.uniform(-1, 1, len(ca))
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, [m, k], ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, [k, n], cb, vb)
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, [1, 2], lc, exact=True)
    for t in (ga, gb):
        t.destroy()


@pytest.mark.parametrize("lc", [[0, 2], [2, 0]])
def test_doubly_compressed_ids_near_2e57(lco_lib, gpu_ctx, oracle_mod, lc):
    """A contracted index of 2^57 values: no row pointer array fits, so only the doubly compressed
    (and outer-product) algorithms run. The hash table of B's rows holds ids at both ends of the
    range (0, 1, 2^57 - 1, 2^57 - 2), ids one apart and 2^40 apart, and ids that no entry of A
    selects; A selects absent ids as well."""
    rng = np.random.default_rng(57)
    m, k, n = 70, 1 << 57, 90
    ids = [0, 1, 2, k - 1, k - 2, k - 3] + [(1 << 40) * i for i in range(1, 40)] + \
          [int(x) for x in rng.integers(0, k, 200, dtype=np.int64)]
    ids = sorted(set(ids))
    cb = np.array(sorted({(j, int(c)) for j in ids for c in rng.choice(n, 1 + j % 5, replace=False)}), dtype=np.uint64)
    vb = rng.uniform(-1, 1, len(cb))
    absent = sorted(set(int(x) for x in rng.integers(0, k, 300, dtype=np.int64)) - set(ids))
    ca = np.array(sorted({(i, int(c)) for i in range(m)
                          for c in list(rng.choice(ids, 4 + i % 9, replace=False)) + list(rng.choice(absent, 3, replace=False))}),
                  dtype=np.uint64)
    va = rng.uniform(-1, 1, len(ca))
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, [m, k], ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, [k, n], cb, vb)
    p = lco_lib.lco_plan_info(gpu_ctx, ga, [0, 1], gb, [1, 2], lc)
    assert lco_lib.ALGOS[p.algo] in ("DCSC", "DCSR")
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, [1, 2], lc, exact=True,
            algos=("auto", "DCSC", "DCSR", "SOP"))
    for t in (ga, gb):
        t.destroy()


@pytest.mark.parametrize("lc", [[0, 2], [2, 0]])
def test_clustered_rows_long_pointer_runs(lco_lib, gpu_ctx, oracle_mod, lc):
    """Rows clustered at both ends of their ranges leave runs of thousands of
    empty rows between them, which whole waves write: B's rows are the first and
    last 300 of 2^22 (about 4.2 million empty row pointers of a singly
    compressed B'; a doubly compressed one finds them in its hash table),
    and A's rows are the first and last 150 of 4096 with 2400 entries (its row
    starts are taken over all 4096 rows)."""
    rng = np.random.default_rng(91)
    m, k, n = 4096, 1 << 22, 300
    brows = np.concatenate([np.arange(300), np.arange(k - 300, k)])
    cb = np.array(sorted({(int(j), int(c)) for j in brows for c in rng.choice(n, 1 + int(j) % 3, replace=False)}),
                  dtype=np.uint64)
    vb = rng.integers(-4, 5, len(cb)).astype(np.float64)
    vb[vb == 0] = 0.5
    arows = np.concatenate([np.arange(150), np.arange(m - 150, m)])
    absent = rng.choice(np.arange(300, k - 300), 4000, replace=False)
    ca = np.array([(int(i), int(c)) for i in arows
                   for c in np.concatenate([rng.choice(brows, 5, replace=False), rng.choice(absent, 3, replace=False)])],
                  dtype=np.uint64)
    va = rng.uniform(-1, 1, len(ca))
    assert m <= 2 * len(ca)
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, [m, k], ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, [k, n], cb, vb)
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, [1, 2], lc, exact=True)
    for t in (ga, gb):
        t.destroy()


@pytest.mark.parametrize("lc", [[0, 1, 3, 4], [3, 4, 0, 1]])
def test_wide_columns_every_algorithm(lco_lib, gpu_ctx, oracle_mod, lc):
    """Columns of the product beyond 2^32 (m' = 2^28 rows, n' = 2^34 columns):
    row-by-row passes key their hash with 64-bit columns and rank outputs by
    readlane, so no row uses the 32-bit table (column-by-column algorithms see
    the transposed shape).  Rows of A hold up to about 10 entries, so the
    lane-mask sums are covered too."""
    rng = np.random.default_rng(11)
    da, db = [1 << 14, 1 << 14, 64], [64, 1 << 17, 1 << 17]
    heads = np.column_stack([rng.integers(0, da[0], 60), rng.integers(0, da[1], 60)]).astype(np.uint64)
    ca = np.column_stack([heads[rng.integers(0, 60, 500)], rng.integers(0, 64, 500).astype(np.uint64)])
    ca = np.unique(ca, axis=0)
    cb = np.column_stack([rng.integers(0, 64, 300), rng.integers(0, db[1], 300), rng.integers(0, db[2], 300)])
    cb = np.unique(cb.astype(np.uint64), axis=0)
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, da, ca, rng.uniform(-1, 1, len(ca)))
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, db, cb, rng.uniform(-1, 1, len(cb)))
    plan = lco_lib.lco_plan_info(gpu_ctx, ga, [0, 1, 2], gb, [2, 3, 4], lc)
    assert plan.num_contracted == 1
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1, 2], gb, ob, [2, 3, 4], lc, exact=True)
    ga.destroy()
    gb.destroy()


@pytest.mark.parametrize("b_len", [1, 2, 4])
def test_tiny_rows_staged_and_direct(lco_lib, gpu_ctx, oracle_mod, b_len):
    """Rows of at most 4 entries and 16 products only (one lane per row): with
    short B' rows a wave's 64 rows have few outputs and are staged through LDS;
    with 4 x 4 disjoint products a wave's outputs exceed the staging buffer and
    are written directly.  Also a ragged last group of rows."""
    rng = np.random.default_rng(40 + b_len)
    m, k = 64 * 37 + 13, 4 * 64
    n = 4 * k
    cb = np.array([(j, (j * 4 + q) % n) for j in range(k) for q in range(b_len)], dtype=np.uint64)
    vb = rng.integers(-4, 5, len(cb)).astype(np.float64)
    ca = np.array([(i, (i * 4 + e) % k) for i in range(m) for e in range(1 + i % 4)], dtype=np.uint64)
    va = rng.uniform(-1, 1, len(ca))
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, [m, k], ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, [k, n], cb, vb)
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, [1, 2], [0, 2], exact=True,
            algos=("auto", "CSR", "CSRNA", "DCSR"))
    for t in (ga, gb):
        t.destroy()


def test_selector_crossovers(lco_lib, gpu_ctx, oracle_mod):
    """A new context selects with the values measured on MI355X; the paper's
    table is one call away.  Against the paper's table: a column-sparsity of 4
    takes CSC instead of DCSC, a column-sparsity of 64 keeps DCSC, an
    index-sparsity of 20 takes CSC or CSR instead of SOP, and one of 64 takes
    DCSC or DCSR instead of SOP (or SOP again when the index cell is set to it).
    Results are bit-identical throughout; bad values are rejected."""
    rng = np.random.default_rng(90)
    ctx2 = lco_lib.lco_ctx_create(0)
    try:
        assert lco_lib.lco_ctx_get_crossovers(ctx2) == lco_lib.MI355X_CROSSOVERS
        assert lco_lib.lco_ctx_get_index_algorithm(ctx2) == lco_lib.MI355X_INDEX_ALGORITHM == "DCSC"
        cases = []
        # a_ijk b_ljk: A is N x N^2 with N^2 / nnz = 4 (A column-sparse, B row-sparse)
        ca, va = L.random_sparse(rng, [64, 64, 64], 1024)
        cb, vb = L.random_sparse(rng, [64, 64, 64], 1024)
        cases.append(([64, 64, 64], ca, va, [64, 64, 64], cb, vb, ("CSC", "CSR")))
        # the same with N^2 / nnz = 64: DCSC stays
        ca, va = L.random_sparse(rng, [64, 64, 64], 64)
        cb, vb = L.random_sparse(rng, [64, 64, 64], 64)
        cases.append(([64, 64, 64], ca, va, [64, 64, 64], cb, vb, None))
        # square N^2 x N^2 operands with index-sparsity 20, then 64
        for nnz, to in ((205, ("CSC", "CSR")), (64, ("DCSC", "DCSR"))):
            ca, va = L.random_sparse(rng, [4096, 64, 64], nnz)
            cb, vb = L.random_sparse(rng, [4096, 64, 64], nnz)
            cases.append(([4096, 64, 64], ca, va, [4096, 64, 64], cb, vb, to))
        la, lb, lc = [0, 1, 2], [3, 1, 2], [0, 3]
        for da, ca, va, db, cb, vb, to in cases:
            ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, da, ca, va)
            gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, db, cb, vb)
            ref = oracle_mod.contract(oa, la, ob, lb, lc)
            lco_lib.lco_ctx_use_paper_selector(ctx2)
            assert lco_lib.lco_ctx_get_crossovers(ctx2) == lco_lib.PAPER_CROSSOVERS
            paper = lco_lib.lco_plan_info(ctx2, ga, la, gb, lb, lc).as_dict()
            got_p = lco_lib.lco_contract(ctx2, ga, la, gb, lb, lc)
            lco_lib.lco_ctx_use_mi355x_selector(ctx2)
            tuned = lco_lib.lco_plan_info(ctx2, ga, la, gb, lb, lc).as_dict()
            got_t = lco_lib.lco_contract(ctx2, ga, la, gb, lb, lc)
            print("selector", paper["algo_name"], "->", tuned["algo_name"], flush=True)
            if to is None:
                assert tuned["algo_name"] == paper["algo_name"]
            else:
                assert paper["algo_name"] != tuned["algo_name"] and tuned["algo_name"] in to
            outs = [got_p, got_t]
            if paper["algo_name"] == "SOP" and to[0] == "DCSC":
                # the measured crossovers with SOP in the index cell: SOP again
                lco_lib.lco_ctx_set_index_algorithm(ctx2, "SOP")
                assert lco_lib.lco_plan_info(ctx2, ga, la, gb, lb, lc).as_dict()["algo_name"] == "SOP"
                outs.append(lco_lib.lco_contract(ctx2, ga, la, gb, lb, lc))
                lco_lib.lco_ctx_set_index_algorithm(ctx2, "DCSR")
                assert lco_lib.lco_ctx_get_index_algorithm(ctx2) == "DCSC"
            for t in outs:
                check(t, ref, exact=True)
            for t in outs + [ga, gb]:
                t.destroy()
        for bad in [(2.9, 3, 3), (3, 3, float("inf")), (3, float("nan"), 3)]:
            with pytest.raises(lco_lib.LcoError):
                lco_lib.lco_ctx_set_crossovers(ctx2, *bad)
        for bad in ("CSC", "CSRNA", "auto"):
            with pytest.raises(lco_lib.LcoError):
                lco_lib.lco_ctx_set_index_algorithm(ctx2, bad)
        assert lco_lib.lco_ctx_get_crossovers(ctx2) == lco_lib.MI355X_CROSSOVERS
        assert lco_lib.lco_ctx_get_index_algorithm(ctx2) == "DCSC"
    finally:
        ctx2.destroy()


# ---------------------------------------------------------------- hyper-sparse cells of the table
def test_rowsparse_times_colsparse_uses_no_accumulator(lco_lib, gpu_ctx, oracle_mod):
    """a_ijk b_lmk (Section 5.2.4): A row-sparse, B column-sparse -> CSCNA/CSRNA."""
    rng = np.random.default_rng(21)
    d = [128, 128, 128]
    ca, va = L.random_sparse(rng, d, 3000)
    cb, vb = L.random_sparse(rng, d, 3000)
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, d, ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, d, cb, vb)
    la, lb, lc = [0, 1, 2], [3, 4, 2], [0, 1, 3, 4]
    p = lco_lib.lco_plan_info(gpu_ctx, ga, la, gb, lb, lc)
    assert (p.a_class, p.b_class) == (lco_lib.LCO_ROW_SPARSE, lco_lib.LCO_COL_SPARSE)
    assert lco_lib.ALGOS[p.algo] in ("CSCNA", "CSRNA")
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, la, gb, ob, lb, lc, exact=True)


def test_colsparse_times_rowsparse_uses_doubly_compressed(lco_lib, gpu_ctx, paper_ctx, oracle_mod):
    """a_ijk b_ljk (Section 5.2.3): A column-sparse, B row-sparse -> DCSC/DCSR in the paper's
    table (a column-sparsity of 5.5, below the crossover measured on MI355X, where a new context
    takes CSC)."""
    rng = np.random.default_rng(22)
    d = [128, 128, 128]
    ca, va = L.random_sparse(rng, d, 3000)
    cb, vb = L.random_sparse(rng, d, 3000)
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, d, ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, d, cb, vb)
    la, lb, lc = [0, 1, 2], [3, 1, 2], [0, 3]
    p = lco_lib.lco_plan_info(paper_ctx, ga, la, gb, lb, lc)
    assert (p.a_class, p.b_class) == (lco_lib.LCO_COL_SPARSE, lco_lib.LCO_ROW_SPARSE)
    assert lco_lib.ALGOS[p.algo] in ("DCSC", "DCSR")
    assert lco_lib.ALGOS[lco_lib.lco_plan_info(gpu_ctx, ga, la, gb, lb, lc).algo] in ("CSC", "CSR")
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, la, gb, ob, lb, lc, exact=True)


@pytest.mark.parametrize("lc", [[0, 1, 4, 5], [0, 4, 1, 5]])
@pytest.mark.parametrize("bits,draws", [(6, 3000), (10, 60000)])
def test_kronecker_index_sparse_sop(lco_lib, gpu_ctx, paper_ctx, oracle_mod, bits, draws, lc):
    """Scaled-down hyper-sparse Kronecker pair contracted over (3,4)x(1,2): index-sparse x
    index-sparse -> SOP, with the second operand rearranged; the output modes in order, or
    interleaved (a general output-LIV key)."""
    ca, va = L.kronecker_hypersparse(bits, draws, seed=1)
    cb, vb = L.kronecker_hypersparse(bits, draws, seed=2)
    dims = [2**bits] * 4
    flags = lco_lib.LCO_COORDS | lco_lib.LCO_SUM_DUPLICATES
    ga = gpu_create(lco_lib, gpu_ctx, dims, ca, va, flags)
    gb = gpu_create(lco_lib, gpu_ctx, dims, cb, vb, flags)
    oa = oracle_mod.create(dims, ca, va, sum_duplicates=True)
    ob = oracle_mod.create(dims, cb, vb, sum_duplicates=True)
    la, lb = [0, 1, 2, 3], [2, 3, 4, 5]
    if bits == 10:
        p = lco_lib.lco_plan_info(paper_ctx, ga, la, gb, lb, lc)
        assert lco_lib.ALGOS[p.algo] == "SOP" and p.permute_b == 1
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, la, gb, ob, lb, lc, exact=True)


def test_diagonal_tensor_splits(lco_lib, gpu_ctx, oracle_mod):
    c, v = L.diagonal(4, 10)
    g, o = pair(lco_lib, gpu_ctx, oracle_mod, [10] * 4, c, v)
    for lb, lc in (([2, 3, 4, 5], [0, 1, 4, 5]), ([1, 2, 3, 4], [0, 4]), ([4, 0, 1, 2], [3, 4])):
        ref = run_all(lco_lib, gpu_ctx, oracle_mod, g, o, [0, 1, 2, 3], g, o, lb, lc, exact=True)
        assert ref.nnz == 10


# ---------------------------------------------------------------- edge cases
def test_edge_cases(lco_lib, gpu_ctx, oracle_mod):
    rng = np.random.default_rng(3)
    ca, va = L.random_sparse(rng, [6, 7], 20)
    cb, vb = L.random_sparse(rng, [7, 5], 20)
    ga, oa = pair(lco_lib, gpu_ctx, oracle_mod, [6, 7], ca, va)
    gb, ob = pair(lco_lib, gpu_ctx, oracle_mod, [7, 5], cb, vb)
    # full contraction to a scalar (order-0 output)
    gs, os_ = pair(lco_lib, gpu_ctx, oracle_mod, [7, 5], *L.random_sparse(rng, [7, 5], 15))
    ref = oracle_mod.contract(ob, [0, 1], os_, [0, 1], [])
    got = lco_lib.lco_contract(gpu_ctx, gb, [0, 1], gs, [0, 1], [])
    check(got, ref)
    # outer product (nothing contracted)
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, [2, 3], [0, 1, 2, 3], exact=True)
    run_all(lco_lib, gpu_ctx, oracle_mod, ga, oa, [0, 1], gb, ob, [2, 3], [2, 0, 3, 1], exact=True)
    # empty operand
    ge = gpu_create(lco_lib, gpu_ctx, [7, 5], np.zeros((0, 2), np.uint64), np.zeros(0))
    r = lco_lib.lco_contract(gpu_ctx, ga, [0, 1], ge, [1, 2], [0, 2])
    assert r.nnz == 0 and r.dims == [6, 5]
    # products that cancel exactly are kept as explicit zeros
    a = gpu_create(lco_lib, gpu_ctx, [2, 2], np.array([[0, 0], [0, 1]], np.uint64), np.array([1.0, 1.0]))
    b = gpu_create(lco_lib, gpu_ctx, [2, 2], np.array([[0, 0], [1, 0]], np.uint64), np.array([1.0, -1.0]))
    for name in ["auto"] + FORCED:
        r = lco_lib.lco_contract(gpu_ctx, a, [0, 1], b, [1, 2], [0, 2], 0 if name == "auto" else lco_lib.ALGO_IDS[name])
        _, l_, v_ = to_np(r)
        assert l_.tolist() == [0] and v_.tolist() == [0.0], name
    # errors are reported before any device work
    with pytest.raises(lco_lib.LcoError) as e:
        lco_lib.lco_contract(gpu_ctx, ga, [0, 1], gb, [1, 2], [0])  # label 2 of b summed alone
    assert e.value.code == 7
    with pytest.raises(lco_lib.LcoError) as e:
        lco_lib.lco_contract(gpu_ctx, ga, [0, 1], ga, [1, 2], [0, 2])
    assert e.value.code == 3


def test_deterministic(lco_lib, gpu_ctx, oracle_mod):
    rng = np.random.default_rng(77)
    ca, va = L.random_sparse(rng, [40, 50, 40], 20000)
    g, _ = pair(lco_lib, gpu_ctx, oracle_mod, [40, 50, 40], ca, va)
    outs = []
    for _ in range(2):
        for name in FORCED:
            r = lco_lib.lco_contract(gpu_ctx, g, [0, 1, 2], g, [2, 1, 3], [0, 3], lco_lib.ALGO_IDS[name])
            outs.append(to_np(r))
            r.destroy()
    for o in outs[1:]:
        assert np.array_equal(o[1], outs[0][1])
        assert np.array_equal(o[2].view(np.uint64), outs[0][2].view(np.uint64))


# ---------------------------------------------------------------- full-size configurations
def squared_laplacian_values(livs, side, dim):
    co = np.stack(np.unravel_index(livs.astype(np.int64), [side] * (2 * dim), order="F"), 1)
    p, q = co[:, :dim], co[:, dim:]
    d = q - p
    l1 = np.abs(d).sum(1)
    deg = np.zeros(len(p), np.int64)
    for ax in range(dim):
        deg += (p[:, ax] > 0).astype(np.int64) + (p[:, ax] < side - 1).astype(np.int64)
    return np.where(l1 == 0, 4 * dim * dim + deg,
                    np.where(l1 == 1, -4 * dim, np.where(np.abs(d).max(1) == 2, 1, 2))).astype(np.float64)


@pytest.mark.slow
def test_3d_fd_config_full_size(lco_lib, gpu_ctx, oracle_mod):
    """128^3 grid (14,581,760 entries): permute (4,5,6,1,2,3), then compose over 3 modes:
    51,742,208 entries, every value equal to the closed form, sampled rows equal to the oracle."""
    s = 128
    c, v = L.fd_laplacian(s, 3)
    g = gpu_create(lco_lib, gpu_ctx, [s] * 6, c, v)
    p = lco_lib.lco_permute(gpu_ctx, g, [3, 4, 5, 0, 1, 2])
    la, lb, lc = [0, 1, 2, 3, 4, 5], [3, 4, 5, 6, 7, 8], [0, 1, 2, 6, 7, 8]
    for name in ("auto", "CSR", "CSRNA"):
        flags = 0 if name == "auto" else lco_lib.ALGO_IDS[name]
        print(f"full 3-D composition algo={name}", flush=True)
        r = lco_lib.lco_contract(gpu_ctx, p, la, p, lb, lc, flags)
        _, livs, vals = to_np(r)
        assert livs.shape[0] == 51742208
        assert np.all(livs[1:] > livs[:-1])
        assert np.array_equal(vals, squared_laplacian_values(livs, s, 3))
        r.destroy()
    # oracle on sampled rows (output grid points), incl. corners and faces
    rng = np.random.default_rng(2)
    rows = np.unique(np.concatenate([rng.integers(0, s**3, 3000), [0, s - 1, s**3 - 1, s * s * 64 + 64 * s]]))
    o = oracle_mod.create([s] * 6, c, v)
    keep = np.isin(o.livs % np.uint64(s**3), rows.astype(np.uint64))
    sub = oracle_mod.Tensor(o.dims, o.livs[keep], o.vals[keep])
    ref = oracle_mod.contract(sub, la, o, lb, lc, mode="sort")
    r = lco_lib.lco_contract(gpu_ctx, p, la, p, lb, lc)
    _, livs, vals = to_np(r)
    pick = np.isin(livs % np.uint64(s**3), rows.astype(np.uint64))
    assert np.array_equal(livs[pick], ref.livs)
    assert np.array_equal(vals[pick], ref.vals)


@pytest.mark.slow
def test_hypersparse_kronecker_full_size(lco_lib, gpu_ctx, oracle_mod):
    """Order-4 Kronecker pair, 2^16 per mode, 2^24 draws each (seeds 1, 2), contracted over (3,4)x(1,2)
    by DCSC (the selector measured on MI355X) and by SOP (the paper's table), bit-identical; sampled
    output rows against the oracle."""
    bits, draws = 16, 1 << 24
    ca, va = L.kronecker_hypersparse(bits, draws, seed=1)
    cb, vb = L.kronecker_hypersparse(bits, draws, seed=2)
    dims = [2**bits] * 4
    flags = lco_lib.LCO_COORDS | lco_lib.LCO_SUM_DUPLICATES
    ga = gpu_create(lco_lib, gpu_ctx, dims, ca, va, flags)
    gb = gpu_create(lco_lib, gpu_ctx, dims, cb, vb, flags)
    la, lb, lc = [0, 1, 2, 3], [2, 3, 4, 5], [0, 1, 4, 5]
    plan = lco_lib.lco_plan_info(gpu_ctx, ga, la, gb, lb, lc)
    assert lco_lib.ALGOS[plan.algo] == "DCSC" and plan.permute_a + plan.permute_b + plan.permute_c == 0
    r = lco_lib.lco_contract(gpu_ctx, ga, la, gb, lb, lc)
    _, livs, vals = to_np(r)
    # the paper's table takes SOP here: the same bits
    sop = lco_lib.lco_contract(gpu_ctx, ga, la, gb, lb, lc, lco_lib.ALGO_IDS["SOP"])
    _, livs_s, vals_s = to_np(sop)
    sop.destroy()
    assert np.array_equal(livs, livs_s) and np.array_equal(vals.view(np.uint64), vals_s.view(np.uint64))
    del livs_s, vals_s
    assert np.all(livs[1:] > livs[:-1])
    # sampled rows: output entries whose (mode 0, mode 1) pair lies in a random sample
    oa = oracle_mod.create(dims, ca, va, sum_duplicates=True)
    ob = oracle_mod.create(dims, cb, vb, sum_duplicates=True)
    rng = np.random.default_rng(5)
    rows = np.unique(oa.livs[rng.integers(0, oa.nnz, 20000)] % np.uint64(2**32))
    keep = np.isin(oa.livs % np.uint64(2**32), rows)
    sub = oracle_mod.Tensor(oa.dims, oa.livs[keep], oa.vals[keep])
    ref = oracle_mod.contract(sub, la, ob, lb, lc, mode="sort")
    pick = np.isin(livs % np.uint64(2**32), rows)
    assert np.array_equal(livs[pick], ref.livs)
    err = np.abs(vals[pick] - ref.vals)
    cancel = np.abs(ref.vals) < 1e-3 * ref.absum
    assert np.all(err <= np.where(cancel, TOL * ref.absum, TOL * np.abs(ref.vals)))
    assert np.array_equal(vals[pick].view(np.uint64), ref.vals.view(np.uint64))
