"""Closed form of the squared FD Laplacian, checked on device arrays with torch.

The Dirichlet FD Laplacian L of a ``side**dim`` grid (centre -2*dim, each in-grid
neighbour 1) composed with itself has, for output (p, q):
  * 4*dim^2 + deg(p) where q = p (deg = in-grid neighbours of p),
  * -4*dim where q is a neighbour of p,
  * 2 where q differs from p by one step along each of two axes,
  * 1 where q is two steps from p along one axis,
and no other entries (the composed stencils of Section 2).  Used by the GPU
tests and the benchmark to check every entry of large batched outputs without
the oracle.
"""
from __future__ import annotations


def fd_square_nnz(dim: int, s: int) -> int:
    if dim == 2:
        return s * s + 4 * s * (s - 1) + 4 * (s - 1) ** 2 + 4 * s * (s - 2)
    return s**3 + 6 * s * s * (s - 1) + 12 * s * (s - 1) ** 2 + 6 * s * s * (s - 2)


def fd_square_matches(torch, livs, vals, side: int, dim: int) -> bool:
    """True iff the device arrays (int64 LIVs in the default order of ``[side] *
    (2*dim)``, float64 values) are exactly L^2: the closed-form count, strictly
    increasing LIVs, every entry on the composed stencil with its exact value."""
    n = livs.numel()
    if n != fd_square_nnz(dim, side) or vals.numel() != n:
        return False
    if n > 1 and not bool((livs[1:] > livs[:-1]).all()):
        return False
    rem = livs.clone()
    c = []
    for _ in range(2 * dim):
        c.append(rem % side)
        rem = rem // side
    if bool((rem != 0).any()):
        return False
    l1 = torch.zeros_like(livs)
    nz = torch.zeros_like(livs)
    deg = torch.zeros_like(livs)
    for a in range(dim):
        d = (c[dim + a] - c[a]).abs()
        l1 += d
        nz += (d != 0).to(livs.dtype)
        deg += (c[a] > 0).to(livs.dtype) + (c[a] < side - 1).to(livs.dtype)
    if bool((l1 > 2).any()):
        return False
    exp = torch.where(l1 == 0, (4 * dim * dim + deg).to(torch.float64),
                      torch.where(l1 == 1, torch.full_like(vals, -4.0 * dim),
                                  torch.where(nz == 2, torch.full_like(vals, 2.0), torch.full_like(vals, 1.0))))
    return bool(torch.equal(exp.view(torch.int64), vals.view(torch.int64)))
