"""GPU parity: construction and radix permutation vs the CPU oracle (bit-exact).

LIVs and values must match the oracle exactly: construction sums duplicates in
input order on both sides, and permutation moves values without arithmetic.
"""
import itertools

import numpy as np
import pytest

import lco_inputs as L
from conftest import gpu_create

pytestmark = pytest.mark.gpu


def same(gt, ot):
    dims, livs, vals = gt.to_numpy()
    assert dims.tolist() == ot.dims.tolist()
    assert livs.shape == ot.livs.shape, (livs.shape, ot.livs.shape)
    assert np.array_equal(livs, ot.livs)
    assert np.array_equal(vals.view(np.uint64), ot.vals.view(np.uint64))


# ---------------------------------------------------------------- construction
@pytest.mark.parametrize("n", [0, 1, 100, 5000, 8192, 8193, 100000, 300001])
def test_create_with_duplicates(lco_lib, gpu_ctx, oracle_mod, n):
    print(f"create n={n}", flush=True)
    rng = np.random.default_rng(n)
    dims = [37, 5, 64, 3]
    coords = np.stack([rng.integers(0, d, n) for d in dims], axis=1).astype(np.uint64)
    vals = rng.uniform(-1, 1, n)
    g = gpu_create(lco_lib, gpu_ctx, dims, coords, vals, lco_lib.LCO_COORDS | lco_lib.LCO_SUM_DUPLICATES)
    o = oracle_mod.create(dims, coords, vals, sum_duplicates=True)
    same(g, o)
    g.destroy()


def test_create_errors(lco_lib, gpu_ctx):
    import torch
    dims = [4, 4]
    with pytest.raises(lco_lib.LcoError) as e:
        gpu_create(lco_lib, gpu_ctx, dims, [[0, 1], [0, 1]], [1.0, 2.0])
    assert e.value.code == 5
    with pytest.raises(lco_lib.LcoError) as e:
        gpu_create(lco_lib, gpu_ctx, dims, [[0, 4]], [1.0])
    assert e.value.code == 1
    livs = torch.tensor([3, 2], dtype=torch.int64, device="cuda")
    vals = torch.tensor([1.0, 2.0], dtype=torch.float64, device="cuda")
    with pytest.raises(lco_lib.LcoError) as e:
        lco_lib.lco_create(gpu_ctx, dims, livs, vals, lco_lib.LCO_SORTED)
    assert e.value.code == 4
    ok = lco_lib.lco_create(gpu_ctx, dims, livs, vals, 0)  # unsorted LIVs are sorted
    d, l_, v = ok.to_numpy()
    assert l_.tolist() == [2, 3] and v.tolist() == [2.0, 1.0]
    ok.destroy()
    with pytest.raises(lco_lib.LcoError) as e:
        lco_lib.lco_create(gpu_ctx, [2**40, 2**30], livs, vals, 0)
    assert e.value.code == 2


def test_create_full_64bit_range(lco_lib, gpu_ctx, oracle_mod):
    rng = np.random.default_rng(64)
    dims = [2**16] * 4
    n = 50000
    coords = np.stack([rng.integers(0, d, n, dtype=np.uint64) for d in dims], axis=1)
    coords[0] = [2**16 - 1] * 4
    vals = rng.uniform(-1, 1, n)
    g = gpu_create(lco_lib, gpu_ctx, dims, coords, vals, lco_lib.LCO_COORDS | lco_lib.LCO_SUM_DUPLICATES)
    o = oracle_mod.create(dims, coords, vals, sum_duplicates=True)
    same(g, o)
    assert int(o.livs[-1]) == 2**64 - 1
    g.destroy()


# ---------------------------------------------------------------- permutation
def _perm_case(lco_lib, gpu_ctx, oracle_mod, dims, coords, vals, perms):
    g = gpu_create(lco_lib, gpu_ctx, dims, coords, vals)
    o = oracle_mod.create(dims, coords, vals)
    for perm in perms:
        print(f"permute dims={dims} nnz={o.nnz} perm={perm}", flush=True)
        gp = lco_lib.lco_permute(gpu_ctx, g, list(perm))
        same(gp, oracle_mod.permute(o, list(perm)))
        gp.destroy()
    g.destroy()


def test_permute_small_fd_config(lco_lib, gpu_ctx, oracle_mod):
    """32x32 grid operator, modes (1,2,3,4) -> (3,4,1,2): single-tile LDS path."""
    c, v = L.fd_laplacian(32, 2)
    _perm_case(lco_lib, gpu_ctx, oracle_mod, [32] * 4, c, v, [(2, 3, 0, 1)])


@pytest.mark.parametrize("nnz", [3000, 60000, 250000])
def test_permute_all_4d_permutations(lco_lib, gpu_ctx, oracle_mod, nnz):
    """All 24 permutations of an order-4 tensor (the paper's 23 non-identity cases plus identity),
    on the LDS path and on the multi-tile global path with a ragged last tile."""
    rng = np.random.default_rng(nnz)
    dims = [29, 64, 7, 33]
    coords, vals = L.random_sparse(rng, dims, nnz)
    _perm_case(lco_lib, gpu_ctx, oracle_mod, dims, coords, vals, list(itertools.permutations(range(4))))


def test_permute_segmented_paths(lco_lib, gpu_ctx, oracle_mod):
    """A shared leading resting mode: small regions (segmented LDS path) and large regions
    (fallback to the global passes)."""
    rng = np.random.default_rng(11)
    small = [50, 40, 300, 20]          # regions of constant (mode 2, mode 3) hold <= 2000 entries
    coords, vals = L.random_sparse(rng, small, 200000)
    _perm_case(lco_lib, gpu_ctx, oracle_mod, small, coords, vals, [(1, 0, 2, 3), (2, 1, 0, 3)])
    big = [400, 300, 3]                 # regions of constant mode 2 hold ~67k entries
    coords, vals = L.random_sparse(rng, big, 200000)
    _perm_case(lco_lib, gpu_ctx, oracle_mod, big, coords, vals, [(1, 0, 2)])
    # regions of 2,300 entries on average, but one of 9,000: the tile sort is tried, gives up, and the
    # global passes run
    dims = [100, 100, 10]
    c0, _ = L.random_sparse(rng, [100, 100], 9000)
    c1, _ = L.random_sparse(rng, [100, 100, 9], 21000)
    coords = np.concatenate([np.concatenate([c0, np.zeros((9000, 1), np.uint64)], axis=1),
                             c1 + np.array([0, 0, 1], dtype=np.uint64)])
    vals = rng.uniform(-1, 1, len(coords))
    lco_lib.lco_timing_reset(gpu_ctx)
    lco_lib.lco_timing_enable(gpu_ctx, True)
    _perm_case(lco_lib, gpu_ctx, oracle_mod, dims, coords, vals, [(1, 0, 2)])
    lco_lib.lco_timing_enable(gpu_ctx, False)
    launched = {k for k in lco_lib.lco_timing_kernels(gpu_ctx) if lco_lib.lco_timing_query(gpu_ctx, k)[0]}
    lco_lib.lco_timing_reset(gpu_ctx)
    assert {"rx_segmented", "rx_scatter"} <= launched


def test_permute_segment_tiles_half_then_full(lco_lib, gpu_ctx, oracle_mod):
    """Segments of 4,000 and 100 entries alternating: half-size tiles (4096) are
    tried first and overflow where a short segment starts next to a long one;
    full-size tiles (8192) then hold them."""
    rng = np.random.default_rng(13)
    dims = [70, 70, 40]
    parts = []
    for m2 in range(0, 40, 2):
        n_here = 4000 if (m2 // 2) % 2 == 0 else 100
        c, _ = L.random_sparse(rng, [70, 70], n_here)
        parts.append(np.concatenate([c, np.full((len(c), 1), m2, np.uint64)], axis=1))
    coords = np.concatenate(parts)
    vals = rng.uniform(-1, 1, len(coords))
    _perm_case(lco_lib, gpu_ctx, oracle_mod, dims, coords, vals, [(1, 0, 2)])


def test_permute_short_segments(lco_lib, gpu_ctx, oracle_mod):
    """Segments of constant leading resting modes that hold a few entries each are
    ranked directly: a ragged last tile, equal keys inside a segment (a trailing
    resting mode below the key: the sort must be stable), and a tensor whose
    segments are short on average but one holds 60 entries (the tile sort takes
    over)."""
    rng = np.random.default_rng(12)
    dims = [6, 5, 70, 90]  # 6300 segments of constant (mode 2, mode 3), ~4.8 entries each
    coords, vals = L.random_sparse(rng, dims, 30001)
    _perm_case(lco_lib, gpu_ctx, oracle_mod, dims, coords, vals, [(1, 0, 2, 3)])
    dims = [3, 4, 5, 40, 50]  # key (mode 2, mode 1) above the resting mode 0
    coords, vals = L.random_sparse(rng, dims, 12000)
    _perm_case(lco_lib, gpu_ctx, oracle_mod, dims, coords, vals, [(0, 2, 1, 3, 4), (2, 1, 0, 3, 4)])
    full = np.array([(a, b, c, 7, 9) for a in range(3) for b in range(4) for c in range(5)], dtype=np.uint64)
    keep = ~((coords[:, 3] == 7) & (coords[:, 4] == 9))
    coords = np.concatenate([coords[keep], full])
    vals = np.concatenate([vals[keep], rng.uniform(-1, 1, len(full))])
    lco_lib.lco_timing_reset(gpu_ctx)
    lco_lib.lco_timing_enable(gpu_ctx, True)
    _perm_case(lco_lib, gpu_ctx, oracle_mod, dims, coords, vals, [(0, 2, 1, 3, 4)])
    lco_lib.lco_timing_enable(gpu_ctx, False)
    launched = {k for k in lco_lib.lco_timing_kernels(gpu_ctx) if lco_lib.lco_timing_query(gpu_ctx, k)[0]}
    lco_lib.lco_timing_reset(gpu_ctx)
    assert {"rx_smallseg", "rx_segmented"} <= launched  # the direct ranking gave up, the tile sort ran


def test_permute_size_one_modes_and_empty(lco_lib, gpu_ctx, oracle_mod):
    rng = np.random.default_rng(5)
    dims = [1, 70, 1, 90]
    coords, vals = L.random_sparse(rng, dims, 3000)
    _perm_case(lco_lib, gpu_ctx, oracle_mod, dims, coords, vals, [(1, 0, 2, 3), (2, 3, 0, 1), (3, 1, 0, 2)])
    e = gpu_create(lco_lib, gpu_ctx, [3, 4], np.zeros((0, 2), np.uint64), np.zeros(0))
    p = lco_lib.lco_permute(gpu_ctx, e, [1, 0])
    assert p.nnz == 0 and p.dims == [4, 3]


def test_permute_hypersparse_64bit(lco_lib, gpu_ctx, oracle_mod):
    """Order-4 Kronecker tensor with 2^16 per mode (full 64-bit LIVs): modes (3,4,1,2), 32-bit key."""
    coords, vals = L.kronecker_hypersparse(16, 1 << 18, seed=2)
    o = oracle_mod.create([2**16] * 4, coords, vals, sum_duplicates=True)
    g = gpu_create(lco_lib, gpu_ctx, [2**16] * 4, coords, vals, lco_lib.LCO_COORDS | lco_lib.LCO_SUM_DUPLICATES)
    same(g, o)
    gp = lco_lib.lco_permute(gpu_ctx, g, [2, 3, 0, 1])
    same(gp, oracle_mod.permute(o, [2, 3, 0, 1]))


def test_timing_filter(lco_lib, gpu_ctx, oracle_mod):
    """lco_timing_only: with a kernel name, only that kernel's launches are
    bracketed by events; with None, every kernel is again."""
    rng = np.random.default_rng(12)
    dims = [1 << 16] * 4
    coords, _ = L.random_sparse(rng, dims, 40000)
    vals = rng.uniform(-1, 1, len(coords))
    t = gpu_create(lco_lib, gpu_ctx, dims, coords, vals)

    def launched():
        return {k for k in lco_lib.lco_timing_kernels(gpu_ctx) if lco_lib.lco_timing_query(gpu_ctx, k)[0]}

    lco_lib.lco_timing_reset(gpu_ctx)
    lco_lib.lco_timing_only(gpu_ctx, "rx_scatter")
    lco_lib.lco_timing_enable(gpu_ctx, True)
    p = lco_lib.lco_permute(gpu_ctx, t, [3, 2, 1, 0])
    lco_lib.lco_timing_enable(gpu_ctx, False)
    assert launched() == {"rx_scatter"}
    n1, ms1 = lco_lib.lco_timing_query(gpu_ctx, "rx_scatter")
    assert n1 >= 2 and ms1 > 0
    p.destroy()
    lco_lib.lco_timing_reset(gpu_ctx)
    lco_lib.lco_timing_only(gpu_ctx, None)
    lco_lib.lco_timing_enable(gpu_ctx, True)
    p = lco_lib.lco_permute(gpu_ctx, t, [3, 2, 1, 0])
    lco_lib.lco_timing_enable(gpu_ctx, False)
    assert {"rx_scatter", "rx_count"} <= launched()
    lco_lib.lco_timing_reset(gpu_ctx)
    same = oracle_mod.permute(oracle_mod.create(dims, coords, vals), [3, 2, 1, 0])
    _, livs, v = p.to_numpy()
    assert np.array_equal(livs, same.livs) and np.array_equal(v.view(np.uint64), same.vals.view(np.uint64))
    p.destroy()
    t.destroy()


def test_permute_3d_fd_operator_order6(lco_lib, gpu_ctx, oracle_mod):
    c, v = L.fd_laplacian(24, 3)
    _perm_case(lco_lib, gpu_ctx, oracle_mod, [24] * 6, c, v, [(3, 4, 5, 0, 1, 2), (1, 0, 2, 3, 4, 5),
                                                             (5, 4, 3, 2, 1, 0)])


@pytest.mark.slow
def test_permute_large_recursive_scans(lco_lib, gpu_ctx):
    """140 M random entries of a 2^16-per-mode order-4 tensor: the radix passes
    (64-bit keys, 8 passes) scan digit-count arrays of 8.75 M entries, more
    than the two-launch scan takes, so the recursive scan runs.  All on the
    device: a permutation is strictly increasing, and permuting back restores
    the tensor bit for bit."""
    import torch
    n = 140_000_000
    dims = [1 << 16] * 4
    print(f"large permute n={n}", flush=True)
    g = torch.Generator(device="cuda").manual_seed(9)
    coords = torch.randint(0, 1 << 16, (n, 4), device="cuda", generator=g, dtype=torch.int64)
    vals = torch.rand(n, device="cuda", generator=g, dtype=torch.float64)
    t = lco_lib.lco_create(gpu_ctx, dims, coords.reshape(-1), vals, lco_lib.LCO_COORDS | lco_lib.LCO_SUM_DUPLICATES)
    del coords, vals
    lco_lib.lco_timing_reset(gpu_ctx)
    lco_lib.lco_timing_enable(gpu_ctx, True)
    p = lco_lib.lco_permute(gpu_ctx, t, [1, 0, 3, 2])
    lco_lib.lco_timing_enable(gpu_ctx, False)
    passes = lco_lib.lco_timing_query(gpu_ctx, "rx_scatter")[0]
    reduces = lco_lib.lco_timing_query(gpu_ctx, "scan_reduce")[0]
    lco_lib.lco_timing_reset(gpu_ctx)
    assert passes >= 2 and reduces == 2 * passes  # each pass's scan also reduces its tile sums
    back = lco_lib.lco_permute(gpu_ctx, p, [1, 0, 3, 2])
    pl = p.livs() ^ torch.iinfo(torch.int64).min  # order-preserving map of the unsigned LIVs to int64
    assert p.nnz == t.nnz and bool((pl[1:] > pl[:-1]).all())
    assert torch.equal(back.livs(), t.livs()) and torch.equal(back.vals().view(torch.int64), t.vals().view(torch.int64))
    for x in (back, p, t):
        x.destroy()


@pytest.mark.slow
def test_permute_3d_fd_full_size(lco_lib, gpu_ctx, oracle_mod):
    """128^3 grid operator (14,581,760 entries), modes (1..6) -> (4,5,6,1,2,3): bit-exact vs the oracle;
    the operator is symmetric, so the result also equals the input."""
    c, v = L.fd_laplacian(128, 3)
    o = oracle_mod.create([128] * 6, c, v)
    assert o.nnz == 14581760
    g = gpu_create(lco_lib, gpu_ctx, [128] * 6, c, v)
    same(g, o)
    gp = lco_lib.lco_permute(gpu_ctx, g, [3, 4, 5, 0, 1, 2])
    same(gp, oracle_mod.permute(o, [3, 4, 5, 0, 1, 2]))
    same(gp, o)
    gp2 = lco_lib.lco_permute(gpu_ctx, g, [3, 4, 5, 0, 1, 2])
    a1, a2 = gp.to_numpy(), gp2.to_numpy()
    assert np.array_equal(a1[1], a2[1]) and np.array_equal(a1[2], a2[2])  # deterministic


@pytest.mark.slow
@pytest.mark.parametrize("perm", [(4, 1, 2, 3, 0, 5), (0, 1, 2, 4, 3, 5), (4, 5, 3, 2, 0, 1)])
def test_permute_3d_fd_full_size_nontrivial(lco_lib, gpu_ctx, oracle_mod, perm):
    """The 128^3 grid operator (14,581,760 entries) under permutations that are
    not symmetries of it, so the correct output differs from the input: a global
    LSD key over rearranged modes, a common leading mode (segmented method), and
    a permutation that moves every mode (its row and column halves take
    different axis orders, so it is no symmetry of the grid).  Bit-exact vs the
    oracle, and the output LIVs differ from the input's."""
    import torch
    c, v = L.fd_laplacian(128, 3)
    o = oracle_mod.create([128] * 6, c, v)
    g = gpu_create(lco_lib, gpu_ctx, [128] * 6, c, v)
    print(f"full-size permute {perm}", flush=True)
    gp = lco_lib.lco_permute(gpu_ctx, g, list(perm))
    ref = oracle_mod.permute(o, list(perm))
    same(gp, ref)
    assert not np.array_equal(ref.livs, o.livs)
    assert not torch.equal(gp.livs(), g.livs())
    for x in (gp, g):
        x.destroy()
