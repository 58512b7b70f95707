"""GPU: a context that allocates device memory itself (no allocator callbacks: hipMalloc with the
released blocks reused in the order of its stream) gives the same bits as a torch-allocating one.
Outputs are kept alive across later calls, released out of order and from another thread, sizes
vary from a few to hundreds of thousands of entries, and the context changes stream half way."""
import threading

import numpy as np
import pytest

import lco_inputs as L
from conftest import gpu_create

pytestmark = pytest.mark.gpu


def fd_labels(dim):
    return list(range(2 * dim)), list(range(dim, 3 * dim)), list(range(dim)) + list(range(2 * dim, 3 * dim))


def same(x, y):
    dx, lx, vx = x.to_numpy()
    dy, ly, vy = y.to_numpy()
    return (np.array_equal(dx, dy) and np.array_equal(lx, ly)
            and np.array_equal(vx.view(np.uint64), vy.view(np.uint64)))


def test_library_allocator_matches_torch_allocator(lco_lib, gpu_ctx):
    import torch
    rng = np.random.default_rng(2024)
    lib_ctx = lco_lib.lco_ctx_create(0, allocator="library")
    held, made = [], []
    try:
        probe = gpu_create(lco_lib, lib_ctx, [4, 4], [[0, 1], [2, 3]], [1.0, 2.0])
        made.append(probe)
        with pytest.raises(KeyError):  # no torch views of library-allocated tensors
            probe.livs()
        ops = []
        for dim, side in [(2, 16), (2, 29), (2, 40), (3, 8), (3, 13), (3, 20)]:
            c, v = L.fd_laplacian(side, dim)
            dims = [side] * (2 * dim)
            ops.append(("fd", dim, gpu_create(lco_lib, gpu_ctx, dims, c, v), gpu_create(lco_lib, lib_ctx, dims, c, v)))
        flags = lco_lib.LCO_COORDS | lco_lib.LCO_SUM_DUPLICATES
        pair_t, pair_l = [], []
        for seed in (1, 2):
            c, v = L.kronecker_hypersparse(8, 3000, seed)
            pair_t.append(gpu_create(lco_lib, gpu_ctx, [256] * 4, c, v, flags))
            pair_l.append(gpu_create(lco_lib, lib_ctx, [256] * 4, c, v, flags))
        made += [o[2] for o in ops] + [o[3] for o in ops] + pair_t + pair_l
        torch.cuda.synchronize()
        for step in range(80):
            if step == 40:  # later work on another stream
                s2 = torch.cuda.Stream()
                lib_ctx.set_stream(s2)
            kind = rng.integers(0, 3)
            if kind == 0:
                _, dim, at, al = ops[rng.integers(0, len(ops))]
                la, lb, lc = fd_labels(dim)
                rt = lco_lib.lco_contract(gpu_ctx, at, la, at, lb, lc)
                rl = lco_lib.lco_contract(lib_ctx, al, la, al, lb, lc)
            elif kind == 1:
                _, dim, at, al = ops[rng.integers(0, len(ops))]
                perm = [int(x) for x in rng.permutation(2 * dim)]
                rt = lco_lib.lco_permute(gpu_ctx, at, perm)
                rl = lco_lib.lco_permute(lib_ctx, al, perm)
            else:
                algo = ["auto", "DCSC", "SOP", "CSR", "CSRNA"][rng.integers(0, 5)]
                f = 0 if algo == "auto" else lco_lib.ALGO_IDS[algo]
                la, lb, lc = [0, 1, 2, 3], [2, 3, 4, 5], [0, 1, 4, 5]
                rt = lco_lib.lco_contract(gpu_ctx, pair_t[0], la, pair_t[1], lb, lc, f)
                rl = lco_lib.lco_contract(lib_ctx, pair_l[0], la, pair_l[1], lb, lc, f)
            print(f"library allocator step {step} kind {kind} nnz {rl.nnz}", flush=True)
            assert same(rt, rl), step
            rt.destroy()
            held.append(rl)
            if len(held) > 6 and rng.random() < 0.5:  # release some held outputs, out of order
                k = int(rng.integers(1, 4))
                for i in sorted(rng.choice(len(held), k, replace=False), reverse=True):
                    held.pop(i).destroy()
            if step % 10 == 9:  # and some from another thread
                batch, held = held[: len(held) // 2], held[len(held) // 2:]
                t = threading.Thread(target=lambda b=batch: [x.destroy() for x in b])
                t.start()
                t.join()
    finally:
        for x in held + made:
            x.destroy()
        lib_ctx.destroy()
