"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: the worked LIV
example printed in the paper, dense brute force (numpy transpose / einsum /
matmul on tiny tensors), closed-form finite-difference stencils, involutions and
exhaustively enumerated index matchings.  None of them calls the HIP library.
"""
import itertools
import math
import os

import numpy as np
import pytest

import lco_inputs as L

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_of(t):
    """Dense array of an oracle tensor, decoding LIVs with plain numpy div/mod."""
    dims = [int(d) for d in t.dims]
    out = np.zeros(dims if dims else (), dtype=np.float64)
    rem = t.livs.copy()
    idx = []
    for d in dims:
        idx.append((rem % np.uint64(d)).astype(np.int64))
        rem = rem // np.uint64(d)
    if dims:
        out[tuple(idx)] = t.vals
    elif t.nnz:
        out[()] = t.vals[0]
    return out


def dense_from_coords(dims, coords, vals):
    out = np.zeros([int(d) for d in dims], dtype=np.float64)
    np.add.at(out, tuple(coords[:, r].astype(np.int64) for r in range(len(dims))), vals)
    return out


# ---------------------------------------------------------------- LIV codec
def test_table_sparse_formats_example(oracle_mod):
    """Section 3.1, Table on CO vs LCO formats: 4x4x4 example LIVs 1, 18, 20, 43, 49, 58."""
    rows = []
    dims = None
    for line in open(os.path.join(GOLDEN, "table_sparse_formats.txt")):
        if line.startswith("#") or not line.strip():
            continue
        if line.startswith("dims"):
            dims = [int(x) for x in line.split()[1:]]
            continue
        rows.append([int(x) for x in line.split()])
    rows = np.array(rows, dtype=np.uint64)
    livs = oracle_mod.linearise(dims, rows[:, :3])
    assert livs.tolist() == rows[:, 3].tolist()
    back = oracle_mod.delinearise(dims, livs)
    assert np.array_equal(back, rows[:, :3])


def test_liv_full_64bit_range(oracle_mod):
    """Unsigned LIVs cover a product of dims of exactly 2^64 (dims (2^16)^4)."""
    dims = [1 << 16] * 4
    c = np.array([[65535] * 4, [0, 0, 0, 1], [1, 0, 0, 0], [12345, 54321, 7, 65535]], dtype=np.uint64)
    livs = oracle_mod.linearise(dims, c)
    expect = [sum(int(x) << (16 * r) for r, x in enumerate(row)) for row in c]
    assert [int(v) for v in livs] == expect
    assert int(livs[0]) == 2**64 - 1
    assert np.array_equal(oracle_mod.delinearise(dims, livs), c)


def test_overflow_rejected(oracle_mod):
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.linearise([1 << 32, (1 << 32) + 1], [[0, 0]])
    assert e.value.code == 2
    oracle_mod.linearise([1 << 32, 1 << 32], [[0, 0]])


# ---------------------------------------------------------------- construction
def test_create_sums_duplicates_in_input_order(oracle_mod):
    rng = np.random.default_rng(7)
    dims = [3, 4, 2]
    coords = np.stack([rng.integers(0, d, 200) for d in dims], axis=1).astype(np.uint64)
    vals = rng.uniform(-1, 1, 200)
    t = oracle_mod.create(dims, coords, vals, sum_duplicates=True)
    # brute force: python dict in input order, keys ordered by (k, j, i)
    acc = {}
    for c, v in zip(coords.tolist(), vals.tolist()):
        key = (c[2], c[1], c[0])
        acc[key] = acc[key] + v if key in acc else v
    keys = sorted(acc)
    assert t.nnz == len(keys)
    assert t.livs.tolist() == [k[2] + 3 * (k[1] + 4 * k[0]) for k in keys]
    assert t.vals.tolist() == [acc[k] for k in keys]  # bit-exact: same order of addition
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.create(dims, coords, vals, sum_duplicates=False)
    assert e.value.code == 5


def test_create_rejects_out_of_range(oracle_mod):
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.create([2, 2], np.array([[0, 2]], np.uint64), [1.0])


# ---------------------------------------------------------------- permutation
@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_permute_vs_dense_transpose_all_perms(oracle_mod, order):
    rng = np.random.default_rng(100 + order)
    dims = [int(x) for x in rng.integers(1, 6, order)]
    coords, vals = L.random_sparse(rng, dims, 40)
    t = oracle_mod.create(dims, coords, vals)
    dense = dense_from_coords(dims, coords, vals)
    for perm in itertools.permutations(range(order)):
        p = oracle_mod.permute(t, perm)
        assert p.dims.tolist() == [dims[q] for q in perm]
        assert p.nnz == t.nnz
        assert np.all(np.diff(p.livs.astype(np.float64)) > 0) or p.nnz < 2
        assert np.array_equal(dense_of(p), np.transpose(dense, perm))


def test_permute_involution_and_inverse(oracle_mod):
    rng = np.random.default_rng(5)
    dims = [5, 3, 4, 6]
    coords, vals = L.random_sparse(rng, dims, 150)
    t = oracle_mod.create(dims, coords, vals)
    swap = [2, 3, 0, 1]
    p = oracle_mod.permute(oracle_mod.permute(t, swap), swap)
    assert np.array_equal(p.livs, t.livs) and np.array_equal(p.vals, t.vals)
    for perm in itertools.permutations(range(4)):
        inv = list(np.argsort(perm))
        q = oracle_mod.permute(oracle_mod.permute(t, perm), inv)
        assert np.array_equal(q.livs, t.livs) and np.array_equal(q.vals, t.vals)


def test_permute_symmetric_fd_operator_is_fixed_point(oracle_mod):
    """The FD Laplacian is symmetric, so swapping row and column modes reproduces it exactly."""
    c, v = L.fd_laplacian(6, 3)
    t = oracle_mod.create([6] * 6, c, v)
    p = oracle_mod.permute(t, [3, 4, 5, 0, 1, 2])
    assert np.array_equal(p.livs, t.livs) and np.array_equal(p.vals, t.vals)


# ---------------------------------------------------------------- contraction
def partial_permutation_count(n):
    """Section 3.1: number of inner/outer index matchings of two order-n tensors."""
    return sum(math.factorial(i) * math.comb(n, i) ** 2 for i in range(n + 1))


def matchings(n):
    """All partial bijections between the modes of two order-n tensors."""
    out = []
    for i in range(n + 1):
        for sa in itertools.combinations(range(n), i):
            for sb in itertools.permutations(range(n), i):
                out.append(list(zip(sa, sb)))
    return out


@pytest.mark.parametrize("n", [1, 2, 3])
def test_all_matchings_vs_einsum(oracle_mod, n):
    assert len(matchings(n)) == partial_permutation_count(n)
    assert [partial_permutation_count(k) for k in (1, 2, 3, 4)] == [2, 7, 34, 209]
    rng = np.random.default_rng(10 + n)
    letters = "abcdefghij"
    for mi, match in enumerate(matchings(n)):
        dims_a = [int(x) for x in rng.integers(1, 5, n)]
        dims_b = [int(x) for x in rng.integers(1, 5, n)]
        for (ia, ib) in match:
            dims_b[ib] = dims_a[ia]
        ca, va = L.random_sparse(rng, dims_a, 12, integer_values=True)
        cb, vb = L.random_sparse(rng, dims_b, 12, integer_values=True)
        a = oracle_mod.create(dims_a, ca, va)
        b = oracle_mod.create(dims_b, cb, vb)
        la = list(range(n))
        lb = [n + j for j in range(n)]
        for (ia, ib) in match:
            lb[ib] = la[ia]
        matched_a = {ia for ia, _ in match}
        matched_b = {ib for _, ib in match}
        lc = [la[i] for i in range(n) if i not in matched_a] + [lb[j] for j in range(n) if j not in matched_b]
        if mi % 2:
            lc = lc[::-1]  # exercise a non-default output order too
        c = oracle_mod.contract(a, la, b, lb, lc)
        spec = "".join(letters[x] for x in la) + "," + "".join(letters[x] for x in lb) + "->" + \
            "".join(letters[x] for x in lc)
        Da = dense_from_coords(dims_a, ca, va)
        Db = dense_from_coords(dims_b, cb, vb)
        expect = np.einsum(spec, Da, Db)
        got = dense_of(c)
        assert np.array_equal(got, expect), (match, lc)
        # structural pattern: positions reached by at least one product
        patt = np.einsum(spec, (Da != 0).astype(np.float64), (Db != 0).astype(np.float64)) > 0
        got_patt = np.zeros_like(patt)
        if c.nnz and patt.ndim:
            got_patt[np.unravel_index(c.livs.astype(np.int64), patt.shape, order="F")] = True
        elif c.nnz:
            got_patt[()] = True
        assert np.array_equal(got_patt, patt)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_entrywise_labels_vs_einsum(oracle_mod, n):
    """Every matching of the modes of two order-n tensors, each matched pair either
    summed (contracted) or kept in the output (entrywise: the product pairs only
    entries that agree on it, as numpy einsum does with a label in both inputs and
    the output), in two output orders; values and structural pattern."""
    rng = np.random.default_rng(40 + n)
    letters = "abcdefghij"
    cases = 0
    for match in matchings(n):
        for roles in itertools.product((0, 1), repeat=len(match)):  # 1: entrywise
            dims_a = [int(x) for x in rng.integers(1, 5, n)]
            dims_b = [int(x) for x in rng.integers(1, 5, n)]
            for (ia, ib) in match:
                dims_b[ib] = dims_a[ia]
            ca, va = L.random_sparse(rng, dims_a, 14, integer_values=True)
            cb, vb = L.random_sparse(rng, dims_b, 14, integer_values=True)
            a = oracle_mod.create(dims_a, ca, va)
            b = oracle_mod.create(dims_b, cb, vb)
            la = list(range(n))
            lb = [n + j for j in range(n)]
            for (ia, ib) in match:
                lb[ib] = la[ia]
            matched_a = {ia: r for (ia, _), r in zip(match, roles)}
            matched_b = {ib for _, ib in match}
            lc = [la[i] for i in range(n) if i not in matched_a or matched_a[i] == 1] + \
                 [lb[j] for j in range(n) if j not in matched_b]
            for order in (lc, lc[::-1]):
                c = oracle_mod.contract(a, la, b, lb, order)
                spec = "".join(letters[x] for x in la) + "," + "".join(letters[x] for x in lb) + "->" + \
                    "".join(letters[x] for x in order)
                Da = dense_from_coords(dims_a, ca, va)
                Db = dense_from_coords(dims_b, cb, vb)
                assert np.array_equal(dense_of(c), np.einsum(spec, Da, Db)), (match, roles, order)
                patt = np.einsum(spec, (Da != 0).astype(np.float64), (Db != 0).astype(np.float64)) > 0
                got_patt = np.zeros_like(patt)
                if c.nnz and patt.ndim:
                    got_patt[np.unravel_index(c.livs.astype(np.int64), patt.shape, order="F")] = True
                elif c.nnz:
                    got_patt[()] = True
                assert np.array_equal(got_patt, patt), (match, roles, order)
                cases += 1
    assert cases == 2 * sum(2 ** len(m) for m in matchings(n))


def test_map_and_sort_modes_agree(oracle_mod):
    rng = np.random.default_rng(3)
    dims = [7, 5, 6]
    ca, va = L.random_sparse(rng, dims, 120)
    cb, vb = L.random_sparse(rng, [6, 5, 4], 90)
    a = oracle_mod.create(dims, ca, va)
    b = oracle_mod.create([6, 5, 4], cb, vb)
    m = oracle_mod.contract(a, [0, 1, 2], b, [2, 1, 3], [3, 0])
    s = oracle_mod.contract(a, [0, 1, 2], b, [2, 1, 3], [3, 0], mode="sort")
    assert np.array_equal(m.livs, s.livs) and np.array_equal(m.vals, s.vals)
    assert np.array_equal(m.absum, s.absum)


# ---------------------------------------------------------------- real-valued contraction pins
#
# Every pin above uses small integer values, whose sums are exact in any float
# format.  The pins below use uniform(-1, 1) FP64 values and compare the oracle
# with references computed independently of it: an exactly rounded sum of each
# output entry's products (math.fsum over a brute-force enumeration of the
# products, Section 2's definition of the product), and a dense (or
# scipy.sparse) matrix product of the matricised operands (Section 5.2).  The
# bound is that of recursive summation: an entry with k products, each rounded
# once and added one at a time from 0.0, is within (k + 1) * u * sum|terms|
# of the exact sum (u = 2^-53).  An oracle that summed in float32, dropped or
# doubled a term, flipped a sign or transposed an operand misses it by orders of
# magnitude.
U64 = 2.0 ** -53


def brute_products(dims_a, ca, va, la, dims_b, cb, vb, lb, lc):
    """Dictionary output-LIV -> list of products, by enumerating every pair of
    entries that agree on the shared labels (plain Python loops)."""
    dims_of = {}
    for lab, d in zip(la, dims_a):
        dims_of[lab] = int(d)
    for lab, d in zip(lb, dims_b):
        dims_of[lab] = int(d)
    shared = [x for x in la if x in lb]
    out = {}
    for i in range(len(va)):
        ka = {lab: int(ca[i][r]) for r, lab in enumerate(la)}
        for j in range(len(vb)):
            kb = {lab: int(cb[j][r]) for r, lab in enumerate(lb)}
            if any(ka[x] != kb[x] for x in shared):
                continue
            coord = {**ka, **kb}
            liv, w = 0, 1
            for lab in lc:  # default order: the first output mode is the least significant
                liv += coord[lab] * w
                w *= dims_of[lab]
            out.setdefault(liv, []).append(float(va[i]) * float(vb[j]))
    return out


@pytest.mark.parametrize("n", [2, 3])
def test_real_values_vs_exact_sums(oracle_mod, n):
    """Random FP64 operands over every partial-permutation matching of two order-n
    tensors (contracted pairs), two output orders: each output entry is within the
    recursive-summation bound of the exactly rounded sum of its products, its
    Σ|products| matches, and the pattern is the set of positions with a product."""
    rng = np.random.default_rng(700 + n)
    checked = 0
    for mi, match in enumerate(matchings(n)):
        dims_a = [int(x) for x in rng.integers(2, 6, n)]
        dims_b = [int(x) for x in rng.integers(2, 6, n)]
        for (ia, ib) in match:
            dims_b[ib] = dims_a[ia]
        ca, va = L.random_sparse(rng, dims_a, 40)
        cb, vb = L.random_sparse(rng, dims_b, 40)
        a = oracle_mod.create(dims_a, ca, va)
        b = oracle_mod.create(dims_b, cb, vb)
        la = list(range(n))
        lb = [n + j for j in range(n)]
        for (ia, ib) in match:
            lb[ib] = la[ia]
        matched_a = {ia for ia, _ in match}
        matched_b = {ib for _, ib in match}
        lc = [la[i] for i in range(n) if i not in matched_a] + [lb[j] for j in range(n) if j not in matched_b]
        for order in ((lc, lc[::-1]) if len(lc) > 1 else (lc,)):
            c = oracle_mod.contract(a, la, b, lb, order)
            prods = brute_products(dims_a, ca, va, la, dims_b, cb, vb, lb, order)
            assert sorted(prods) == [int(x) for x in c.livs], (match, order)
            for liv, val, absum in zip(c.livs.tolist(), c.vals.tolist(), c.absum.tolist()):
                terms = prods[int(liv)]
                exact = math.fsum(terms)
                mag = math.fsum(abs(t) for t in terms)
                bound = (len(terms) + 1) * U64 * mag
                assert abs(val - exact) <= bound, (match, order, liv, val, exact)
                assert abs(absum - mag) <= bound
                checked += 1
    assert checked > (150 if n == 2 else 1000)


@pytest.mark.parametrize("bits", [4, 5, 6])
def test_kronecker_pairs_real_values_vs_matrix_product(oracle_mod, bits):
    """Scaled-down instances of the hyper-sparse Kronecker pair (2^bits per mode,
    2^(bits+6) draws each, seeds 1 and 2, duplicates summed, uniform(-1, 1)
    values), contracted over modes (3,4) x (1,2): the matricised product A @ B
    computed by scipy.sparse in FP64, with |A| @ |B| as the magnitude of each
    entry's terms; values within 1e-12 of that magnitude (the gate of the GPU
    parity tests), the structural pattern exact, and the entries with the most
    products within the recursive-summation bound of math.fsum."""
    import scipy.sparse as sp
    side = 1 << bits
    n2 = side * side
    draws = 1 << (bits + 6)
    ops = []
    for seed in (1, 2):
        co, va = L.kronecker_hypersparse(bits, draws, seed)
        ops.append((co, va, oracle_mod.create([side] * 4, co, va, sum_duplicates=True)))
    (ca, va, a), (cb, vb, b) = ops
    c = oracle_mod.contract(a, [0, 1, 2, 3], b, [2, 3, 4, 5], [0, 1, 4, 5])
    # matricise from the raw coordinates (duplicates summed by the sparse constructor)
    ra = ca[:, 0].astype(np.int64) + side * ca[:, 1].astype(np.int64)
    ka = ca[:, 2].astype(np.int64) + side * ca[:, 3].astype(np.int64)
    kb = cb[:, 0].astype(np.int64) + side * cb[:, 1].astype(np.int64)
    nb = cb[:, 2].astype(np.int64) + side * cb[:, 3].astype(np.int64)
    MA = sp.csr_matrix((va, (ra, ka)), shape=(n2, n2))
    MB = sp.csr_matrix((vb, (kb, nb)), shape=(n2, n2))
    MA.sum_duplicates()
    MB.sum_duplicates()
    ones_a = sp.csr_matrix((np.ones(MA.nnz), MA.indices, MA.indptr), shape=MA.shape)
    ones_b = sp.csr_matrix((np.ones(MB.nnz), MB.indices, MB.indptr), shape=MB.shape)
    P = (ones_a @ ones_b).tocoo()          # structural pattern (count of products per entry)
    C = (MA @ MB).tocsr()
    M = (abs(MA) @ abs(MB)).tocsr()
    livs = P.row.astype(np.uint64) + np.uint64(n2) * P.col.astype(np.uint64)
    order = np.argsort(livs)
    livs = livs[order]
    rows, cols = P.row[order], P.col[order]
    assert c.nnz == livs.size > 0
    assert np.array_equal(c.livs, livs)
    ref = np.asarray(C[rows, cols]).ravel()
    mag = np.asarray(M[rows, cols]).ravel()
    assert np.all(np.abs(c.vals - ref) <= 1e-12 * mag)
    assert np.all(np.abs(c.absum - mag) <= 1e-12 * mag)
    # exactly rounded sums of the entries with the most products
    count = P.data[order]
    top = np.argsort(-count, kind="stable")[:32]
    dA, dB = MA.tolil(), MB.tocsc()
    for t in top:
        i, j = int(rows[t]), int(cols[t])
        arow = dA.rows[i]
        terms = [float(dA[i, kk]) * float(dB[kk, j]) for kk in arow if dB[kk, j] != 0]
        assert len(terms) == int(count[t])
        exact = math.fsum(terms)
        bound = (len(terms) + 1) * U64 * math.fsum(abs(x) for x in terms)
        assert abs(c.vals[t] - exact) <= bound


def test_contract_errors(oracle_mod):
    a = oracle_mod.create([3, 4], np.array([[0, 0]], np.uint64), [1.0])
    b = oracle_mod.create([5, 2], np.array([[0, 0]], np.uint64), [1.0])
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.contract(a, [0, 1], b, [1, 2], [0, 2])
    assert e.value.code == 3  # contracted dims 4 vs 5
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.contract(a, [0, 1], b, [2, 3], [0, 2, 3])
    assert e.value.code == 7  # a label of a in neither b nor the output (a summed free label)
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.contract(a, [0, 1], b, [0, 2], [0, 1, 2])
    assert e.value.code == 3  # entrywise label with dims 3 vs 5


def test_diagonal_products(oracle_mod):
    """Diagonal tensors (Section 5.1 hyper-sparsity figure): products stay diagonal."""
    n = 10
    c, v = L.diagonal(4, n)
    a = oracle_mod.create([n] * 4, c, v)
    # a_ijkl a_klmn (2+2 split: index-sparse) -> diagonal with squared values
    r = oracle_mod.contract(a, [0, 1, 2, 3], a, [2, 3, 4, 5], [0, 1, 4, 5])
    assert r.nnz == n
    assert np.array_equal(r.vals, v * v)
    assert np.array_equal(oracle_mod.delinearise(r.dims, r.livs), np.stack([np.arange(n)] * 4, 1).astype(np.uint64))
    # a_ijkl a_jklm (1+3 / 3+1 splits: column- and row-sparse)
    r = oracle_mod.contract(a, [0, 1, 2, 3], a, [1, 2, 3, 4], [0, 4])
    assert r.nnz == n and np.array_equal(r.vals, v * v)


# ------------------------------------------------- closed-form FD compositions
def _squared_laplacian_check(t, side, dim):
    """Closed form of (Dirichlet FD Laplacian)^2 entries.

    With L = -2d on the diagonal and 1 for in-grid neighbours:
    diagonal = 4d^2 + deg(p); |q-p| = 1 -> -4d; two unit steps on different
    axes -> 2; two unit steps on one axis -> 1.
    """
    co = np.stack(np.unravel_index(t.livs.astype(np.int64), [side] * (2 * dim), order="F"), 1)
    p, q = co[:, :dim], co[:, dim:]
    d = q - p
    l1 = np.abs(d).sum(1)
    deg = np.zeros(len(p), np.int64)
    for ax in range(dim):
        deg += (p[:, ax] > 0).astype(np.int64) + (p[:, ax] < side - 1).astype(np.int64)
    expect = np.where(l1 == 0, 4 * dim * dim + deg,
                      np.where(l1 == 1, -4 * dim,
                               np.where(np.abs(d).max(1) == 2, 1, 2))).astype(np.float64)
    assert np.all(l1 <= 2)
    assert np.array_equal(t.vals, expect)


def biharmonic_nnz(s):
    return s * s + 4 * s * (s - 1) + 4 * (s - 1) ** 2 + 4 * s * (s - 2)


def squared_laplacian_3d_nnz(s):
    return s**3 + 6 * s * s * (s - 1) + 12 * s * (s - 1) ** 2 + 6 * s * s * (s - 2)


@pytest.mark.parametrize("side", [2, 3, 5, 32])
def test_biharmonic_closed_form(oracle_mod, side):
    c, v = L.fd_laplacian(side, 2)
    assert len(v) == 5 * side * side - 4 * side
    t = oracle_mod.create([side] * 4, c, v)
    r = oracle_mod.contract(t, [0, 1, 2, 3], t, [2, 3, 4, 5], [0, 1, 4, 5])
    assert r.nnz == biharmonic_nnz(side)
    _squared_laplacian_check(r, side, 2)
    if side >= 3:
        # interior rows carry the 13-point biharmonic stencil 20 / -8 / 2 / 1
        assert set(np.unique(r.vals)) >= {20.0, -8.0, 2.0, 1.0}


@pytest.mark.parametrize("side", [2, 4, 7])
def test_squared_3d_laplacian_closed_form(oracle_mod, side):
    c, v = L.fd_laplacian(side, 3)
    assert len(v) == 7 * side**3 - 6 * side**2
    t = oracle_mod.create([side] * 6, c, v)
    r = oracle_mod.contract(t, [0, 1, 2, 3, 4, 5], t, [3, 4, 5, 6, 7, 8], [0, 1, 2, 6, 7, 8])
    assert r.nnz == squared_laplacian_3d_nnz(side)
    _squared_laplacian_check(r, side, 3)


def test_small_fd_config_equals_dense_product(oracle_mod):
    """32x32 grid: the composed operator equals the dense 1024x1024 matrix product exactly."""
    s = 32
    c, v = L.fd_laplacian(s, 2)
    M = np.zeros((s * s, s * s))
    rows = (c[:, 0] + s * c[:, 1]).astype(np.int64)
    cols = (c[:, 2] + s * c[:, 3]).astype(np.int64)
    M[rows, cols] = v
    t = oracle_mod.create([s] * 4, c, v)
    p = oracle_mod.permute(t, [2, 3, 0, 1])
    Mp = np.zeros_like(M)
    Mp[(p.livs % (s * s)).astype(np.int64), (p.livs // (s * s)).astype(np.int64)] = p.vals
    assert np.array_equal(Mp, M.T)
    r = oracle_mod.contract(t, [0, 1, 2, 3], t, [2, 3, 4, 5], [0, 1, 4, 5])
    D = np.zeros_like(M)
    D[(r.livs % (s * s)).astype(np.int64), (r.livs // (s * s)).astype(np.int64)] = r.vals
    assert np.array_equal(D, M @ M)
    assert r.nnz == int(np.count_nonzero((M != 0).astype(float) @ (M != 0).astype(float)))
    assert r.nnz == 12676


def test_kronecker_generator_recipe(oracle_mod):
    """Small Kronecker instance: duplicates summed, values bounded, order-4 outer structure."""
    coords, vals = L.kronecker_hypersparse(6, 4096, seed=1)
    assert coords.max() < 64
    t = oracle_mod.create([64] * 4, coords, vals, sum_duplicates=True)
    assert 0 < t.nnz <= 4096
    assert np.isclose(t.vals.sum(), vals.sum())
    dense = dense_from_coords([64] * 4, coords, vals)
    assert np.array_equal(np.count_nonzero(dense != 0) <= t.nnz, True)


# ---------------------------------------------------------------- addition
def _pattern_of(t):
    return set(int(x) for x in t.livs)


def _dense_pattern(t):
    """Boolean array: the positions the tensor stores (explicit zeros included)."""
    return dense_of(oracle_tensor_with_values(t, np.ones(t.nnz))) != 0


def oracle_tensor_with_values(t, vals):
    import oracle
    return oracle.Tensor(t.dims, t.livs, np.asarray(vals, dtype=np.float64))


@pytest.mark.parametrize("alpha,beta", [(1.0, 1.0), (1.0, -1.0), (0.5, 3.0)])
def test_add_vs_dense_all_label_orders(oracle_mod, alpha, beta):
    """Section 2 addition: c = alpha*a + beta*b where b's modes are named in any
    order; dense brute force (numpy transposes) for every order of b's labels and
    of c's labels, values and pattern (the union of the patterns, explicit zeros
    included)."""
    rng = np.random.default_rng(11)
    dims = [3, 4, 5]
    ca, va = L.random_sparse(rng, dims, 20, integer_values=True)
    va[:3] = 0.0  # explicit zeros stay structural
    a = oracle_mod.create(dims, ca, va)
    labels = [7, 8, 9]
    A = dense_of(a)
    Apat = _dense_pattern(a)
    for pb in itertools.permutations(range(3)):
        b_labels = [labels[q] for q in pb]
        b_dims = [dims[q] for q in pb]
        cb, vb = L.random_sparse(rng, b_dims, 25, integer_values=True)
        b = oracle_mod.create(b_dims, cb, vb)
        # B[b coords] -> a's mode order: a mode q is b mode pb.index(q)
        Bt = np.transpose(dense_of(b), [pb.index(q) for q in range(3)])
        Bpat = np.transpose(_dense_pattern(b), [pb.index(q) for q in range(3)])
        for pc in itertools.permutations(range(3)):
            c_labels = [labels[q] for q in pc]
            c = oracle_mod.add(a, labels, b, b_labels, c_labels, alpha, beta)
            assert [int(x) for x in c.dims] == [dims[q] for q in pc]
            assert np.all(np.diff(c.livs.astype(np.float64)) > 0)
            want = np.transpose(alpha * A + beta * Bt, pc)
            assert np.array_equal(dense_of(c), want)
            assert np.array_equal(_dense_pattern(c), np.transpose(Apat | Bpat, pc))


def test_add_cancellation_keeps_pattern_and_identities(oracle_mod):
    """a - a keeps every position with value 0.0; a + b = b + a; adding an empty
    tensor scales; a + a = 2a exactly."""
    rng = np.random.default_rng(3)
    dims = [6, 5, 4, 3]
    ca, va = L.random_sparse(rng, dims, 60)
    cb, vb = L.random_sparse(rng, dims, 70)
    a = oracle_mod.create(dims, ca, va)
    b = oracle_mod.create(dims, cb, vb)
    lab = [0, 1, 2, 3]
    z = oracle_mod.add(a, lab, a, lab, lab, 1.0, -1.0)
    assert np.array_equal(z.livs, a.livs) and np.all(z.vals == 0.0)
    two = oracle_mod.add(a, lab, a, lab, lab)
    assert np.array_equal(two.vals, 2.0 * a.vals)
    ab = oracle_mod.add(a, lab, b, lab, lab, 0.25, -3.0)
    ba = oracle_mod.add(b, lab, a, lab, lab, -3.0, 0.25)
    assert np.array_equal(ab.livs, ba.livs) and np.array_equal(ab.vals, ba.vals)
    assert _pattern_of(ab) == _pattern_of(a) | _pattern_of(b)
    empty = oracle_mod.create(dims, np.zeros((0, 4), np.uint64), np.zeros(0))
    e = oracle_mod.add(empty, lab, a, lab, lab, 1.0, -2.0)
    assert np.array_equal(e.livs, a.livs) and np.array_equal(e.vals, -2.0 * a.vals)


def test_add_errors(oracle_mod):
    a = oracle_mod.create([2, 3], [[0, 0]], [1.0])
    b = oracle_mod.create([3, 2], [[0, 0]], [1.0])
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.add(a, [0, 1], b, [0, 1], [0, 1])  # same labels, different dims
    assert e.value.code == 3
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.add(a, [0, 1], b, [1, 2], [0, 1])  # label sets differ
    assert e.value.code == 1
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.add(a, [0, 0], b, [0, 1], [0, 1])  # repeated label
    assert e.value.code == 1


# ------------------------------------------- combinatorial Laplacian (Section 2)
def test_fd_first_derivative_exact_on_quadratics():
    """The O(h^2) central, forward and backward differences of the FD matrix of
    Section 2 are exact on quadratics: D x^2 = 2x, D x = 1, D 1 = 0 (the last
    row must be (1, -4, 3)/2 for this to hold)."""
    for n in (3, 4, 7, 31):
        c, v = L.fd_first_derivative(n)
        assert len(v) == 2 * n + 2
        D = dense_from_coords([n, n], c, v)
        x = np.arange(n, dtype=np.float64)
        assert np.array_equal(D @ (x * x), 2 * x)
        assert np.array_equal(D @ x, np.ones(n))
        assert np.array_equal(D @ np.ones(n), np.zeros(n))


def combinatorial_laplacian_oracle(oracle_mod, n):
    """The design tensor a_ijlk = d_ii' delta_jl d_i'k + d_jj' delta_ik d_j'l of
    Section 2, executed left to right as binary products (two outer products with
    Kronecker deltas, two hyper-sparse contractions) and one addition whose
    second term is re-sorted into the first term's mode order."""
    I, J, K, Lb, I2, J2 = 0, 1, 2, 3, 4, 5
    cd, vd = L.fd_first_derivative(n)
    d = oracle_mod.create([n, n], cd, vd)
    ce, ve = L.diagonal(2, n, np.ones(n))
    delta = oracle_mod.create([n, n], ce, ve)
    by = oracle_mod.contract(d, [I, I2], delta, [J, Lb], [I, I2, J, Lb])
    ty = oracle_mod.contract(by, [I, I2, J, Lb], d, [I2, K], [I, J, Lb, K])
    bx = oracle_mod.contract(d, [J, J2], delta, [I, K], [J, J2, I, K])
    tx = oracle_mod.contract(bx, [J, J2, I, K], d, [J2, Lb], [J, I, K, Lb])
    a = oracle_mod.add(ty, [I, J, Lb, K], tx, [J, I, K, Lb], [I, J, Lb, K])
    return by, ty, tx, a


@pytest.mark.parametrize("n", [3, 7, 15])
def test_combinatorial_laplacian_closed_form(oracle_mod, n):
    """a = (D^2)_ik delta_jl + delta_ik (D^2)_jl: flattened with rows (i, j) and
    columns (k, l) it is kron(D^2, I) + kron(I, D^2) (dense numpy); the pattern
    is the union of the two terms' patterns."""
    by, ty, tx, a = combinatorial_laplacian_oracle(oracle_mod, n)
    c, v = L.fd_first_derivative(n)
    D = dense_from_coords([n, n], c, v)
    D2 = D @ D
    E = np.eye(n)
    want = (np.kron(D2, E) + np.kron(E, D2)).reshape(n, n, n, n)  # [i, j, k, l]
    got = dense_of(a).transpose(0, 1, 3, 2)  # a is stored (i, j, l, k)
    assert np.array_equal(got, want)
    pat2 = (np.abs(D) != 0).astype(np.int64) @ (np.abs(D) != 0).astype(np.int64) != 0  # structural D^2
    pat = (np.kron(pat2, E) + np.kron(E, pat2)) != 0
    assert a.nnz == int(pat.sum())
    assert by.nnz == (2 * n + 2) * n
    assert ty.nnz == int(pat2.sum()) * n and tx.nnz == ty.nnz
