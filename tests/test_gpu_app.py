"""GPU: the design tensor of the paper's Section 2 (the combinatorial Laplacian
a_ijlk = d_ii' delta_jl d_i'k + d_jj' delta_ik d_j'l) at N = 2^k - 1.

It is executed left to right as binary operations, as the paper describes:
two outer products with Kronecker deltas, the two hyper-sparse products of
Section 6 (an N^3 x N row-sparse operand times an N x N sparse matrix), and one
addition whose second term must first be re-sorted into the first term's order
(the {1,0,3,2} permutation of Section 3.2).  N = 2^k - 1 keeps every dimension
off a power of two, so the LIV codec runs its invariant-division path.

Small N: every intermediate equals the oracle bit for bit.  N = 2047 (the
paper's largest size): every entry of the two terms and of the sum is checked
against the closed form (D^2)_ik delta_jl + delta_ik (D^2)_jl, computed densely
with numpy (all values are short dyadic fractions, so every order of summation
gives the same bits).
"""
import numpy as np
import pytest

import lco_inputs as L
from conftest import gpu_create

pytestmark = pytest.mark.gpu

I, J, K, LL, I2, J2 = 0, 1, 2, 3, 4, 5


def same(gt, ot, what=""):
    d, livs, vals = gt.to_numpy()
    assert d.tolist() == ot.dims.tolist(), what
    assert np.array_equal(livs, ot.livs), what
    assert np.array_equal(vals.view(np.uint64), ot.vals.view(np.uint64)), what


def operands(lco, ctx, n):
    cd, vd = L.fd_first_derivative(n)
    ce, ve = L.diagonal(2, n, np.ones(n))
    return gpu_create(lco, ctx, [n, n], cd, vd), gpu_create(lco, ctx, [n, n], ce, ve)


def design_tensor(lco, ctx, d, delta):
    by = lco.lco_contract(ctx, d, [I, I2], delta, [J, LL], [I, I2, J, LL])
    ty = lco.lco_contract(ctx, by, [I, I2, J, LL], d, [I2, K], [I, J, LL, K])
    bx = lco.lco_contract(ctx, d, [J, J2], delta, [I, K], [J, J2, I, K])
    tx = lco.lco_contract(ctx, bx, [J, J2, I, K], d, [J2, LL], [J, I, K, LL])
    a = lco.lco_add(ctx, ty, [I, J, LL, K], tx, [J, I, K, LL], [I, J, LL, K])
    return by, ty, bx, tx, a


@pytest.mark.parametrize("n", [3, 7, 15, 31])
def test_design_tensor_vs_oracle(lco_lib, gpu_ctx, oracle_mod, n):
    print(f"design tensor n={n}", flush=True)
    d, delta = operands(lco_lib, gpu_ctx, n)
    got = design_tensor(lco_lib, gpu_ctx, d, delta)
    od = oracle_mod.create([n, n], *L.fd_first_derivative(n))
    oe = oracle_mod.create([n, n], *L.diagonal(2, n, np.ones(n)))
    oby = oracle_mod.contract(od, [I, I2], oe, [J, LL], [I, I2, J, LL])
    oty = oracle_mod.contract(oby, [I, I2, J, LL], od, [I2, K], [I, J, LL, K])
    obx = oracle_mod.contract(od, [J, J2], oe, [I, K], [J, J2, I, K])
    otx = oracle_mod.contract(obx, [J, J2, I, K], od, [J2, LL], [J, I, K, LL])
    oa = oracle_mod.add(oty, [I, J, LL, K], otx, [J, I, K, LL], [I, J, LL, K])
    for g, o, what in zip(got, (oby, oty, obx, otx, oa), ("by", "ty", "bx", "tx", "a")):
        same(g, o, f"{what} n={n}")
    for t in got + (d, delta):
        t.destroy()


def _liv(n, c0, c1, c2, c3):
    n = np.uint64(n)
    return c0 + n * (c1 + n * (c2 + n * c3))


def test_design_tensor_full_size_closed_form(lco_lib, gpu_ctx):
    n = 2047
    print(f"design tensor n={n}", flush=True)
    d, delta = operands(lco_lib, gpu_ctx, n)
    plan = lco_lib.lco_plan_info(gpu_ctx, d, [I, I2], delta, [J, LL], [I, I2, J, LL])
    assert plan.num_contracted == 0
    by, ty, bx, tx, a = design_tensor(lco_lib, gpu_ctx, d, delta)
    cd, vd = L.fd_first_derivative(n)
    D = np.zeros((n, n))
    D[cd[:, 0].astype(np.int64), cd[:, 1].astype(np.int64)] = vd
    P = (D != 0).astype(np.float64)
    D2 = D @ D
    P2 = (P @ P) != 0  # structural pattern of D^2 (kept even where values cancel)
    ik = np.argwhere(P2).astype(np.uint64)  # row-major: ascending (i, k)
    v2 = D2[P2]
    ar = np.arange(n, dtype=np.uint64)
    # by_{i i' j l} = D_ii' delta_jl
    assert by.nnz == (2 * n + 2) * n == 8_384_512
    # ty_{i j l k} = (D^2)_ik delta_jl
    ty_l = _liv(n, ik[:, 0][None, :], ar[:, None], ar[:, None], ik[:, 1][None, :]).ravel()
    ty_v = np.broadcast_to(v2[None, :], (n, len(v2))).ravel()
    o = np.argsort(ty_l)
    _, livs, vals = ty.to_numpy()
    assert np.array_equal(livs, ty_l[o]) and np.array_equal(vals, ty_v[o])
    # tx_{j i k l} = delta_ik (D^2)_jl: the same entries with the roles of the pairs swapped
    _, livs_x, vals_x = tx.to_numpy()
    assert np.array_equal(livs_x, ty_l[o]) and np.array_equal(vals_x, ty_v[o])
    # a_{i j l k} = (D^2)_ik delta_jl + delta_ik (D^2)_jl
    tx_l = _liv(n, ar[:, None], ik[:, 0][None, :], ik[:, 1][None, :], ar[:, None]).ravel()
    keys = np.concatenate([ty_l, tx_l])
    v = np.concatenate([ty_v, ty_v])
    uk, inv = np.unique(keys, return_inverse=True)
    s = np.zeros(len(uk))
    np.add.at(s, inv, v)
    _, livs_a, vals_a = a.to_numpy()
    assert a.nnz == len(uk)
    assert np.array_equal(livs_a, uk) and np.array_equal(vals_a, s)
    print(f"nnz by={by.nnz} ty={ty.nnz} a={a.nnz}", flush=True)
    for t in (by, ty, bx, tx, a, d, delta):
        t.destroy()


def design_tensor_ijkl(lco, ctx, n):
    """a_ijkl (modes in the order i, j, k, l), as the permutation experiment of Section 4.2 uses it."""
    d, delta = operands(lco, ctx, n)
    by, ty, bx, tx, a = design_tensor(lco, ctx, d, delta)
    a2 = lco.lco_add(ctx, ty, [I, J, LL, K], tx, [J, I, K, LL], [I, J, K, LL])
    for t in (by, ty, bx, tx, a, d, delta):
        t.destroy()
    return a2


def test_design_tensor_permutations_vs_oracle(lco_lib, gpu_ctx, oracle_mod):
    import itertools
    n = 15
    a = design_tensor_ijkl(lco_lib, gpu_ctx, n)
    _, livs, vals = a.to_numpy()
    oa = oracle_mod.Tensor(np.array([n] * 4, np.uint64), livs, vals)
    for perm in itertools.permutations(range(4)):
        print(f"permute design tensor n={n} perm={perm}", flush=True)
        p = lco_lib.lco_permute(gpu_ctx, a, list(perm))
        same(p, oracle_mod.permute(oa, list(perm)), str(perm))
        p.destroy()
    a.destroy()


def test_design_tensor_permutations_full_size(lco_lib, gpu_ctx):
    """n = 2896 (2^11.5 rounded, the size of the paper's permutation table): every
    permutation followed by its inverse gives the tensor back bit for bit and a
    strictly increasing LIV list; the three permutations of the table are also
    checked entry by entry against numpy (decode, move coordinates, re-linearise,
    sort)."""
    import itertools
    n = 2896
    print(f"permute design tensor n={n}", flush=True)
    a = design_tensor_ijkl(lco_lib, gpu_ctx, n)
    _, livs, vals = a.to_numpy()
    nn = np.uint64(n)
    coords = [(livs // nn**q) % nn for q in range(4)]
    for perm in itertools.permutations(range(4)):
        if perm == (0, 1, 2, 3):
            continue
        inv = [perm.index(q) for q in range(4)]
        p = lco_lib.lco_permute(gpu_ctx, a, list(perm))
        back = lco_lib.lco_permute(gpu_ctx, p, inv)
        _, pl, pv = p.to_numpy()
        _, bl, bv = back.to_numpy()
        assert np.all(pl[1:] > pl[:-1]), perm
        assert np.array_equal(bl, livs) and np.array_equal(bv.view(np.uint64), vals.view(np.uint64)), perm
        if perm in ((3, 1, 2, 0), (2, 1, 3, 0), (1, 0, 2, 3)):
            want = coords[perm[0]] + nn * (coords[perm[1]] + nn * (coords[perm[2]] + nn * coords[perm[3]]))
            o = np.argsort(want, kind="stable")
            assert np.array_equal(pl, want[o]) and np.array_equal(pv.view(np.uint64), vals[o].view(np.uint64))
        p.destroy()
        back.destroy()
    a.destroy()
