"""CPU: the seeded input recipes (coordinates and values only)."""
import numpy as np
import pytest

import lco_inputs as L


def fd_out_nnz(dim, s):
    if dim == 2:
        return s * s + 4 * s * (s - 1) + 4 * (s - 1) ** 2 + 4 * s * (s - 2)
    return s**3 + 6 * s * s * (s - 1) + 12 * s * (s - 1) ** 2 + 6 * s * s * (s - 2)


@pytest.mark.parametrize("side,dim", [(1, 2), (2, 2), (5, 2), (2, 3), (7, 3)])
def test_fd_torch_is_the_same_operator(side, dim):
    torch = pytest.importorskip("torch")
    c, v = L.fd_laplacian(side, dim)
    ct, vt = L.fd_laplacian_torch(side, dim, torch.device("cpu"))
    a = sorted(zip(map(tuple, c.astype(np.int64).tolist()), v.tolist()))
    b = sorted(zip(map(tuple, ct.numpy().tolist()), vt.numpy().tolist()))
    assert a == b
    assert len(a) == (2 * dim + 1) * side**dim - 2 * dim * side ** (dim - 1)


def test_kronecker_torch_range_and_marginals():
    torch = pytest.importorskip("torch")
    c, v = L.kronecker_hypersparse_torch(6, 1 << 14, 3, torch.device("cpu"))
    c = c.numpy()
    assert c.shape == (1 << 14, 4) and c.min() >= 0 and c.max() < 64
    assert float(v.min()) >= -1.0 and float(v.max()) < 1.0
    # per bit, P(first mode bit set) = 0.19 + 0.05, P(second mode bit set) = 0.19 + 0.05
    for m in range(4):
        frac = ((c[:, m] >> 3) & 1).mean()
        assert abs(frac - 0.24) < 0.02
    c2, _ = L.kronecker_hypersparse_torch(6, 1 << 14, 3, torch.device("cpu"))
    assert np.array_equal(c, c2.numpy())  # seeded


def test_batched_recipe_sizes():
    inst = L.batched_fd_instances()
    assert len(inst) == 4096
    assert all(8 <= s <= 64 and d in (2, 3) for d, s in inst)
    n_in = sum((2 * d + 1) * s**d - 2 * d * s ** (d - 1) for d, s in inst)
    n_out = sum(fd_out_nnz(d, s) for d, s in inst)
    assert (n_in, n_out) == (1089900128, 3811424094)


def test_serving_trace_shape():
    t, cls, p = L.serving_trace(60.0)
    assert np.all(np.diff(t) > 0) and t[-1] < 60.0
    assert abs(len(t) / 60.0 - 200) < 10  # Poisson rate
    frac = np.bincount(cls, minlength=3) / len(t)
    assert abs(frac[0] - 0.70) < 0.02 and abs(frac[1] - 0.25) < 0.02 and abs(frac[2] - 0.05) < 0.01
    assert p[cls == 0].min() >= 16 and p[cls == 0].max() <= 96
    assert p[cls == 1].min() >= 64 and p[cls == 1].max() <= 128
    assert p[cls == 2].min() >= 12 and p[cls == 2].max() <= 16
    t20, c20, p20 = L.serving_trace(20.0)
    assert np.array_equal(t20, t[:len(t20)]) and np.array_equal(c20, cls[:len(t20)])  # a prefix
    assert np.array_equal(p20, p[:len(t20)]) and t[len(t20)] >= 20.0


def test_rtensor_recipe():
    """Octant draws: each mode's bit is 1 with the marginal of the jittered
    probabilities (about .5/6*3 + .2 = .45 before jitter), levels independent;
    seeded; the first mode's extra bits extend its range."""
    c, v = L.rtensor(10, 1 << 16, seed=3)
    assert c.shape == (1 << 16, 3) and c.max() < 1024 and np.all(np.abs(v) < 1)
    for m in range(3):
        frac = ((c[:, m] >> 4) & 1).mean()
        assert 0.2 < frac < 0.7
    assert abs(((c[:, 0] >> 2) & 1).mean() - ((c[:, 0] >> 7) & 1).mean()) < 0.02  # same law at every level
    c2, _ = L.rtensor(10, 1 << 16, seed=3)
    assert np.array_equal(c, c2)
    c3, _ = L.rtensor(6, 1 << 14, seed=4, first_extra_bits=6)
    assert c3[:, 0].max() >= 64 and c3[:, 0].max() < 4096 and c3[:, 1].max() < 64
    # no jitter: the marginal of the first mode's bit is exactly .5/6*3 + .2
    c4, _ = L.rtensor(1, 1 << 18, seed=5, jitter=0.0)
    assert abs((c4[:, 0] & 1).mean() - (0.25 + 0.2)) < 0.005
