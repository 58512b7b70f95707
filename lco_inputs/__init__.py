"""Seeded synthetic input generators shared by the tests, the oracle checks and the benchmark.

This module produces *coordinates and values only*: per-entry mode coordinates (an
``(nnz, order)`` uint64 array, unsorted) and FP64 values.  It holds none of the
method's arithmetic -- no linearisation, no sorting by linearised index, no
products -- so both the oracle and the HIP path start from exactly the same raw
input and each does its own linearisation.

Workloads (all synthetic, seeded, shaped like the paper's benchmark operators):

* ``fd_laplacian(side, dim)`` -- the finite-difference Laplacian on a ``side**dim``
  grid with Dirichlet boundary (neighbours outside the grid are dropped), as a
  tensor of order ``2*dim``: the first ``dim`` modes are the output grid point,
  the last ``dim`` modes the input grid point.  Centre value ``-2*dim``, each
  in-grid neighbour ``1``.  This is the high-order differential operator of the
  paper's Section 2 (the combinatorial Laplacian built from FD matrices),
  in its standard 5-point (2-D) / 7-point (3-D) form.
* ``kronecker_hypersparse(bits, draws, seed)`` -- a 4-mode Kronecker (R-MAT style)
  tensor with ``2**bits`` per mode: each draw picks, for every bit level and each
  mode pair (0,1), (2,3), one of four quadrants with probabilities
  ``[0.57, 0.19, 0.19, 0.05]``; values uniform(-1, 1).  Duplicated coordinates
  are left in (the consumer sums them on construction).  This is the recursive
  quadrant model that the paper's R-TENSOR generalises (Section 5.2.1).
* ``fd_first_derivative(n)`` -- the length-``n`` first-derivative FD matrix of the
  paper's Section 2 as an order-2 tensor: O(h^2) central differences (-1/2, +1/2)
  on interior rows, the O(h^2) one-sided forms (-3, 4, -1)/2 on the first row and
  (1, -4, 3)/2 on the last.  Its products with Kronecker deltas build the
  combinatorial Laplacian of the paper's Section 2 at ``n = 2**k - 1``.
* ``rtensor(bits, draws, seed)`` -- the third-order R-TENSOR of the paper's
  Section 5.2.1 (the R-MAT model generalised to octants): per bit level one
  octant is drawn with the base edge probabilities of Table r_tensor_probs
  ((1,1,1): .3, (2,2,2): .2, the six others .5/6 each), jittered once per tensor
  by uniform(-.1, .1) additions and renormalised; ``first_extra_bits`` extends the
  first mode (the M x N x N tensors with M = N^2 of the outer-product tests).
* ``random_sparse(rng, dims, nnz)`` -- distinct uniformly random coordinates.
* ``diagonal(order, n)`` -- the purely diagonal tensor of the paper's Figure on
  hyper-sparsity of matricised tensors (all-zero except i=j=...).
* ``batched_fd_instances(count, seed)`` -- the (dimension, grid side) of each
  instance of a batch of FD self-compositions: 2-D 5-point or 3-D 7-point
  (50/50), side uniform in 8..64.
* ``fd_laplacian_torch`` / ``kronecker_hypersparse_torch`` -- the same recipes
  producing coordinates directly in device memory with torch (for operand
  pools too large to generate on the host quickly).  The FD operator is the
  same set of entries as ``fd_laplacian`` (in another order); the Kronecker
  tensor follows the same quadrant recipe but draws from torch's generator,
  so it is not the PCG64 tensor of the same seed.
* ``serving_trace(seconds, rate, seed)`` -- a Poisson request stream: arrival
  times and, per request, its class (small 2-D FD composition, large 3-D FD
  composition, hyper-sparse Kronecker pair) and size parameter.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "fd_laplacian",
    "kronecker_hypersparse",
    "fd_first_derivative",
    "random_sparse",
    "rtensor",
    "RTENSOR_PROBS",
    "diagonal",
    "batched_fd_instances",
    "fd_laplacian_torch",
    "kronecker_hypersparse_torch",
    "serving_trace",
    "KRON_PROBS",
]

KRON_PROBS = (0.57, 0.19, 0.19, 0.05)
# octants (1,1,1), (1,1,2), (1,2,1), (1,2,2), (2,1,1), (2,1,2), (2,2,1), (2,2,2)
RTENSOR_PROBS = (0.3,) + (0.5 / 6,) * 6 + (0.2,)


def fd_laplacian(side: int, dim: int):
    """Coordinates and values of the ``dim``-D FD Laplacian on a ``side**dim`` grid.

    Returns ``(coords, vals)`` with ``coords`` of shape ``(nnz, 2*dim)`` (uint64):
    modes ``0..dim-1`` are the row grid point (x, y[, z]) and modes
    ``dim..2*dim-1`` the column grid point.  ``nnz = (2*dim+1)*side**dim -
    2*dim*side**(dim-1)``.
    """
    if side < 1 or dim < 1:
        raise ValueError("side and dim must be >= 1")
    axes = np.meshgrid(*[np.arange(side, dtype=np.int64)] * dim, indexing="ij")
    pts = np.stack([a.reshape(-1) for a in axes], axis=1)  # (side**dim, dim)
    coords = [np.concatenate([pts, pts], axis=1)]
    vals = [np.full(pts.shape[0], -2.0 * dim)]
    for ax in range(dim):
        for step in (-1, 1):
            nb = pts.copy()
            nb[:, ax] += step
            keep = (nb[:, ax] >= 0) & (nb[:, ax] < side)
            coords.append(np.concatenate([pts[keep], nb[keep]], axis=1))
            vals.append(np.ones(int(keep.sum())))
    return (np.ascontiguousarray(np.concatenate(coords).astype(np.uint64)),
            np.concatenate(vals).astype(np.float64))


def kronecker_hypersparse(bits: int, draws: int, seed: int, probs=KRON_PROBS):
    """Order-4 Kronecker tensor, ``2**bits`` per mode, ``draws`` quadrant draws.

    For each bit level ``b`` (low to high) and each mode pair ((0,1), then (2,3)) a
    uniform number picks quadrant ``q`` from the cumulative probabilities; the
    pair's first mode gets bit ``q >> 1`` and the second bit ``q & 1`` at level
    ``b``.  Values are drawn afterwards, uniform in (-1, 1).  Duplicate
    coordinates are kept.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    cum = np.cumsum(np.asarray(probs, dtype=np.float64))
    cols = [np.zeros(draws, dtype=np.uint64) for _ in range(4)]
    q = np.empty(draws, dtype=np.uint8)
    for b in range(bits):
        for (m0, m1) in ((0, 1), (2, 3)):
            u = rng.random(draws)
            # quadrant = how many cumulative probabilities are <= u (a right-sided search)
            np.less_equal(cum[0], u, out=q, casting="unsafe")
            for c in cum[1:]:
                q += u >= c
            cols[m0] |= (q >> 1).astype(np.uint64) << np.uint64(b)
            cols[m1] |= (q & 1).astype(np.uint64) << np.uint64(b)
    vals = rng.uniform(-1.0, 1.0, draws)
    return np.ascontiguousarray(np.stack(cols, axis=1)), vals


def rtensor(bits: int, draws: int, seed: int, first_extra_bits: int = 0, probs=RTENSOR_PROBS,
            jitter: float = 0.1):
    """Coordinates ``(draws, 3)`` and values of an R-TENSOR with ``2**bits`` per mode
    (the first mode ``2**(bits + first_extra_bits)``).

    The probabilities get one uniform(-jitter, jitter) addition each, negative
    results are clipped to 0, and they are renormalised to sum to 1.  For each bit
    level ``b`` (low to high) a uniform number picks octant ``o`` (index 4x + 2y + z
    of the octant (x+1, y+1, z+1)), which sets bit ``b`` of the three coordinates to
    x, y, z.  The extra high bits of the first mode are set with the first mode's
    marginal probability of its upper half.  Values are uniform in (-1, 1).
    Duplicate coordinates are kept (the consumer sums them on construction).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.asarray(probs, dtype=np.float64) + rng.uniform(-jitter, jitter, 8)
    p = np.clip(p, 0.0, None)
    p /= p.sum()
    cum = np.cumsum(p)
    coords = np.zeros((draws, 3), dtype=np.uint64)
    one = np.uint64(1)
    for b in range(bits):
        o = np.searchsorted(cum, rng.random(draws), side="right").astype(np.uint64)
        o = np.minimum(o, np.uint64(7))
        coords[:, 0] |= ((o >> np.uint64(2)) & one) << np.uint64(b)
        coords[:, 1] |= ((o >> one) & one) << np.uint64(b)
        coords[:, 2] |= (o & one) << np.uint64(b)
    p_hi = float(p[4:].sum())
    for b in range(first_extra_bits):
        coords[:, 0] |= (rng.random(draws) < p_hi).astype(np.uint64) << np.uint64(bits + b)
    vals = rng.uniform(-1.0, 1.0, draws)
    return coords, vals


def random_sparse(rng: np.random.Generator, dims, nnz: int, integer_values: bool = False):
    """``nnz`` distinct uniformly random coordinates in ``dims`` (fewer if the space is smaller).

    Values are uniform(-1, 1), or small integers in [-4, 4] \\ {0} when
    ``integer_values`` (useful where exact sums are wanted).
    """
    dims = [int(d) for d in dims]
    order = len(dims)
    if order == 0:
        n = min(nnz, 1)
        coords = np.zeros((n, 0), dtype=np.uint64)
    else:
        total = 1
        for d in dims:
            total *= d
        nnz = min(nnz, total)
        if nnz == 0:
            coords = np.zeros((0, order), dtype=np.uint64)
        else:
            got = np.zeros((0, order), dtype=np.uint64)
            while got.shape[0] < nnz:
                need = (nnz - got.shape[0]) * 2 + 8
                cand = np.stack([rng.integers(0, d, need, dtype=np.uint64) for d in dims], axis=1)
                got = np.unique(np.concatenate([got, cand]), axis=0)
            pick = rng.permutation(got.shape[0])[:nnz]
            coords = np.ascontiguousarray(got[pick])
    n = coords.shape[0]
    if integer_values:
        v = rng.integers(1, 5, n).astype(np.float64) * rng.choice([-1.0, 1.0], n)
    else:
        v = rng.uniform(-1.0, 1.0, n)
    return coords, v


def fd_first_derivative(n: int):
    """Coordinates ``(nnz, 2)`` (row, column) and values of the ``n x n`` O(h^2)
    first-derivative matrix (unit spacing), ``n >= 3``: 2n + 2 entries."""
    if n < 3:
        raise ValueError("the one-sided rows need n >= 3")
    rows, cols, vals = [0, 0, 0], [0, 1, 2], [-1.5, 2.0, -0.5]
    i = np.arange(1, n - 1, dtype=np.int64)
    r = np.concatenate([np.array(rows), np.repeat(i, 2), np.full(3, n - 1)])
    c = np.concatenate([np.array(cols), np.stack([i - 1, i + 1], axis=1).ravel(), np.array([n - 3, n - 2, n - 1])])
    v = np.concatenate([np.array(vals), np.tile([-0.5, 0.5], n - 2), np.array([0.5, -2.0, 1.5])])
    coords = np.ascontiguousarray(np.stack([r, c], axis=1).astype(np.uint64))
    return coords, v.astype(np.float64)


def diagonal(order: int, n: int, values=None):
    """The diagonal tensor of order ``order`` with ``n`` per mode (entries where all coordinates agree)."""
    c = np.arange(n, dtype=np.uint64)
    coords = np.ascontiguousarray(np.stack([c] * order, axis=1))
    vals = np.arange(1, n + 1, dtype=np.float64) if values is None else np.asarray(values, dtype=np.float64)
    return coords, vals


def batched_fd_instances(count: int = 4096, seed: int = 4096, lo: int = 8, hi: int = 64):
    """``[(dim, side), ...]``: each instance is the ``dim``-D FD Laplacian on a ``side**dim`` grid,
    composed with itself.  Sides are drawn first (uniform in ``lo..hi``), then the kinds
    (0: 2-D 5-point, 1: 3-D 7-point), from ``PCG64(seed)``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    side = rng.integers(lo, hi + 1, size=count)
    kind = rng.integers(0, 2, size=count)
    return [(2 + int(k), int(s)) for s, k in zip(side, kind)]


SERVE_CLASSES = ("fd2", "fd3", "kron")


def serving_trace(seconds: float = 60.0, rate: float = 200.0, seed: int = 5):
    """A Poisson request stream from ``PCG64(seed)``: exponential inter-arrival gaps of mean
    ``1/rate`` seconds up to ``seconds``; per request a uniform draw picks the class
    (70 % ``fd2``: 2-D 5-point FD composition with side U{16..96}; 25 % ``fd3``: 3-D 7-point
    with side U{64..128}; 5 % ``kron``: a hyper-sparse Kronecker pair with 2**L per mode,
    L U{12..16}).  Requests are drawn in blocks of 4096 (gaps, class draws, then the three
    size draws), so a shorter window is a prefix of a longer one.  Returns
    ``(arrival_s, cls, param)`` arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ts, cs, ps = [], [], []
    t_end = 0.0
    while t_end < seconds:
        gaps = rng.exponential(1.0 / rate, size=4096)
        u = rng.random(4096)
        p2 = rng.integers(16, 97, size=4096)
        p3 = rng.integers(64, 129, size=4096)
        pk = rng.integers(12, 17, size=4096)
        t = t_end + np.cumsum(gaps)
        t_end = float(t[-1])
        cls = np.where(u < 0.70, 0, np.where(u < 0.95, 1, 2)).astype(np.int64)
        ts.append(t)
        cs.append(cls)
        ps.append(np.where(cls == 0, p2, np.where(cls == 1, p3, pk)).astype(np.int64))
    t, cls, param = np.concatenate(ts), np.concatenate(cs), np.concatenate(ps)
    n = int(np.searchsorted(t, seconds))
    return t[:n], cls[:n], param[:n]


def fd_laplacian_torch(side: int, dim: int, device):
    """``(coords, vals)`` torch tensors on ``device``: the entries of ``fd_laplacian(side, dim)``
    (coordinates int64 of shape ``(nnz, 2*dim)``, row point then column point), unsorted."""
    import torch
    n = side**dim
    p = torch.arange(n, device=device, dtype=torch.int64)
    pts = [(p // side**a) % side for a in range(dim)]  # x, y[, z] of each grid point
    cs = [torch.stack(pts + pts, dim=1)]
    vs = [torch.full((n,), -2.0 * dim, dtype=torch.float64, device=device)]
    for a in range(dim):
        for step in (-1, 1):
            q = pts[a] + step
            ok = (q >= 0) & (q < side)
            row = list(pts)
            row[a] = q
            c = torch.stack(row + pts, dim=1)[ok]
            cs.append(c)
            vs.append(torch.ones(c.shape[0], dtype=torch.float64, device=device))
    return torch.cat(cs), torch.cat(vs)


def kronecker_hypersparse_torch(bits: int, draws: int, seed: int, device, probs=KRON_PROBS):
    """``(coords, vals)`` torch tensors on ``device``: the quadrant recipe of
    ``kronecker_hypersparse`` with uniform numbers from ``torch.Generator(device).manual_seed(seed)``.
    Duplicate coordinates are kept."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    cum = torch.tensor(np.cumsum(np.asarray(probs, dtype=np.float64)), dtype=torch.float64, device=device)
    coords = torch.zeros((draws, 4), dtype=torch.int64, device=device)
    for b in range(bits):
        for (m0, m1) in ((0, 1), (2, 3)):
            u = torch.rand(draws, generator=g, dtype=torch.float64, device=device)
            q = torch.bucketize(u, cum, right=True).clamp_(max=3)
            coords[:, m0] |= (q >> 1) << b
            coords[:, m1] |= (q & 1) << b
    vals = torch.rand(draws, generator=g, dtype=torch.float64, device=device) * 2.0 - 1.0
    return coords, vals
