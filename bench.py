"""Benchmark: one step = radix permutation of the order-6 FD Laplacian on a 128^3 grid
(14,581,760 non-zeros, modes (1..6) -> (4,5,6,1,2,3)) followed by the contraction of the
permuted operator with itself over three modes (51,742,208 output non-zeros), on one MI355X.

Prints ONE JSON line: output non-zeros per second of the whole step, the permutation's
effective GB/s against the HBM peak, per-step p50/p99, a roofline object for the dominant
kernel (HIP-event time of every launch in the timed region, algorithmic bytes per launch),
and the CPU oracle's throughput on a bounded sample of the same step.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, GB/s
SIDE = 128
PERM = [3, 4, 5, 0, 1, 2]
LA, LB, LC = [0, 1, 2, 3, 4, 5], [3, 4, 5, 6, 7, 8], [0, 1, 2, 6, 7, 8]


def algorithmic_bytes(kernel: str, sz: dict):
    """Bytes a launch of `kernel` must move at minimum for this workload (per launch)."""
    n, na, nb, nc, k, rows = sz["n"], sz["nnz_a"], sz["nnz_b"], sz["nnz_c"], sz["k"], sz["rows"]
    table = {
        # one stable radix pass: read LIV + value, write LIV + value
        "rx_scatter": 32 * n,
        "rx_count": 8 * n,
        "rx_single": 32 * n,
        "shuffle_copy": 32 * n,
        # numeric row pass: read A' and B' once, write C once, read the row pointers of B'
        # and the per-row metadata (list entry, start, id, output offset)
        "row_small_num": 16 * (na + nb + nc) + 4 * (k + 1) + 24 * rows,
        # symbolic row pass: LIVs of A' and B', row pointers, per-row metadata and counts
        "row_small_sym": 8 * (na + nb) + 4 * (k + 1) + 24 * rows,
        # per A' entry: read its LIV, write its product count and B' row start (32-bit each),
        # read the row pointers of B'
        "entry_len": 16 * na + 4 * (k + 1),
        # the same, plus the row starts (4 B) and ids (8 B) of all m' = rows rows of A'
        "dense_rows_len": 16 * na + 4 * (k + 1) + 12 * rows,
        "dense_ptr": 8 * nb + 4 * (k + 1),
        "seg_heads": 12 * na,
    }
    return table.get(kernel)


def source_digest() -> str:
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1802_02619_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode())
            h.update(f.read())
    return h.hexdigest()[:16]


MAIN_WORKLOAD = "fd3d_128_permute_contract"
APP_WORKLOAD = "laplacian_2047_design_tensor"


def measured_traffic(kernel: str, workload: str = MAIN_WORKLOAD):
    """HBM bytes per launch of `kernel` in `workload` from the committed rocprofv3 counter summary
    (profiles/traffic.json), if it was taken from the current sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != source_digest():
        return None
    e = t.get("workloads", {}).get(workload, {}).get("kernels", {}).get(kernel)
    return None if e is None else e.get("bytes_per_launch")


def copy_ceiling(torch, nbytes: int = 1 << 30, reps: int = 10):
    """Measured device-copy ceiling: a plain elementwise copy of `nbytes` (read + write) on the
    current stream, timed with HIP events; GB/s counts both directions."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for k in range(reps):
        torch.neg(src, out=dst)
        ev[k + 1].record()
    torch.cuda.synchronize()
    ms = statistics.median(ev[k].elapsed_time(ev[k + 1]) for k in range(reps))
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def note(msg: str):
    """One progress line on stderr (the JSON result is the only line on stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def host_cpu():
    """Model name and core counts of the host CPU (from /proc/cpuinfo and the OS)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cores": os.cpu_count(), "cores_available": len(os.sched_getaffinity(0))}


def cpu_baseline(coords, vals, reps: int = 3, frac_den: int = 32):
    """The oracle (single thread, pinned to one core) on a bounded sample of the same step.

    Runs before any GPU work: the oracle's permutation of the whole operand, then its
    std::map contraction of a seeded sample of 1/frac_den of the output rows (all of
    their products), each the median of `reps` runs; the step time is the
    permutation pro-rated to the sample's share of the operand plus the sampled
    contraction."""
    import numpy as np

    import oracle
    mask = os.sched_getaffinity(0)
    core = min(mask)
    os.sched_setaffinity(0, {core})
    try:
        dims = [SIDE] * 6
        o = oracle.create(dims, coords, vals)
        t_perm = []
        for _ in range(reps):
            t0 = time.perf_counter()
            p_full = oracle.permute(o, PERM)
            t_perm.append(time.perf_counter() - t0)
        rng = np.random.default_rng(1234)
        rows = np.unique(rng.integers(0, SIDE**3, SIDE**3 // frac_den)).astype(np.uint64)
        keep = np.isin(p_full.livs % np.uint64(SIDE**3), rows)
        sub = oracle.Tensor(p_full.dims, p_full.livs[keep], p_full.vals[keep])
        t_con = []
        for _ in range(reps):
            t0 = time.perf_counter()
            c_sub = oracle.contract(sub, LA, p_full, LB, LC)
            t_con.append(time.perf_counter() - t0)
    finally:
        os.sched_setaffinity(0, mask)
    tp, tc = statistics.median(t_perm), statistics.median(t_con)
    share = sub.nnz / p_full.nnz
    t_step = tp * share + tc
    cpu = host_cpu()
    return {
        "value": c_sub.nnz / t_step,
        "unit": "output nnz/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{rows.size} of {SIDE**3} output rows ({share:.4f} of the operand, seed 1234): oracle "
                   f"permutation of the full operand (median {tp:.2f} s of {reps}, pro-rated to the sample's "
                   f"share) + std::map contraction of the sampled rows (median {tc:.2f} s of {reps}, "
                   f"{c_sub.nnz} output nnz); one thread pinned to core {core}"),
        "seconds": sum(t_perm) + sum(t_con),
        "reps": reps,
        "pinned_core": core,
        "host_cpu": cpu["model"],
        "host_logical_cores": cpu["logical_cores"],
        "host_cores_available": cpu["cores_available"],
    }, (rows, c_sub)


def fd_compose_nnz(dim: int, s: int) -> int:
    """Non-zeros of the FD Laplacian composed with itself (Dirichlet), closed form."""
    from tests.fd_closed_form import fd_square_nnz
    return fd_square_nnz(dim, s)


def fd_labels(dim: int):
    return (list(range(2 * dim)), list(range(dim, 3 * dim)), list(range(dim)) + list(range(2 * dim, 3 * dim)))


def batched_leg(lco, ctx, torch, np, L, count: int, reps: int):
    """Batch of `count` uneven FD self-compositions: plain per-call loop vs one lco_contract_batch."""
    inst = L.batched_fd_instances(count)
    distinct = {}
    for dim, side in sorted(set(inst)):
        c, v = L.fd_laplacian(side, dim)
        idx_d = torch.from_numpy(c.view(np.int64).reshape(-1).copy()).to("cuda:0")
        val_d = torch.from_numpy(v).to("cuda:0")
        distinct[(dim, side)] = lco.lco_create(ctx, [side] * (2 * dim), idx_d, val_d, lco.LCO_COORDS)
    # every instance owns its operand (a device copy of the distinct operator)
    ops = []
    for dim, side in inst:
        src = distinct[(dim, side)]
        ops.append(lco.lco_create(ctx, src.dims, src.livs(), src.vals(), lco.LCO_SORTED))
    for t in distinct.values():
        t.destroy()
    items = []
    for a, (dim, _) in zip(ops, inst):
        la, lb, lc = fd_labels(dim)
        items.append((a, la, a, lb, lc))
    torch.cuda.synchronize()
    n_in = sum(a.nnz for a in ops)
    expect = [fd_compose_nnz(dim, side) for dim, side in inst]

    def plain():
        return [lco.lco_contract(ctx, *it) for it in items]

    def batched():
        return lco.lco_contract_batch(ctx, items)

    res = {}
    keep = {}
    for name, fn in (("plain", plain), ("batched", batched)):
        outs = fn()  # warm-up
        for o in outs:
            o.destroy()
        times = []
        for r in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            outs = fn()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            if r + 1 < reps:
                for o in outs:
                    o.destroy()
        keep[name] = outs
        res[name] = statistics.median(times)
    stats = lco.lco_batch_stats(ctx)
    ok_nnz = all(o.nnz == e for o, e in zip(keep["batched"], expect)) and \
        all(o.nnz == e for o, e in zip(keep["plain"], expect))
    rng = np.random.default_rng(11)
    sample = sorted(set(rng.integers(0, count, 16).tolist()) | {int(np.argmax(expect))})

    def same(x, y):
        return torch.equal(x.livs(), y.livs()) and torch.equal(x.vals().view(torch.int64), y.vals().view(torch.int64))

    ok_bits = all(same(keep["plain"][i], keep["batched"][i]) for i in sample)
    # every batched output, entry by entry, against the closed-form composed stencil (on the device)
    from tests.fd_closed_form import fd_square_matches
    t0 = time.perf_counter()
    bad_vals = [i for i, ((dim, side), o) in enumerate(zip(inst, keep["batched"]))
                if not fd_square_matches(torch, o.livs(), o.vals(), side, dim)]
    t_check = time.perf_counter() - t0
    for name, outs in keep.items():  # keep only the sampled plain outputs
        for i, o in enumerate(outs):
            if name == "batched" or i not in sample:
                o.destroy()
    ref = {i: keep["plain"][i] for i in sample}
    del keep
    torch.cuda.synchronize()
    # planned batch: host planning once, then the whole batch (setup, symbolic, offsets, numeric) as one
    # persistent launch, run directly and replayed as a HIP graph
    t0 = time.perf_counter()
    plan = lco.BatchPlan(ctx, items)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    planned = {"create_s": t_plan, "launches": plan.launches()}
    pouts = plan.outputs()
    ok_plan = all(same(ref[i], pouts[i]) for i in sample) and all(o.nnz == e for o, e in zip(pouts, expect))
    ok_plan = ok_plan and all(fd_square_matches(torch, o.livs(), o.vals(), side, dim)
                              for (dim, side), o in zip(inst, pouts))
    for mode in ("execute", "graph"):
        fn = plan.execute if mode == "execute" else plan.graph_launch
        fn()  # warm (the graph is captured on its first launch)
        torch.cuda.synchronize()
        tt = []
        for _ in range(max(3, reps)):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            tt.append(time.perf_counter() - t0)
        planned[mode + "_s"] = statistics.median(tt)
    ok_plan = ok_plan and all(same(ref[i], pouts[i]) for i in sample)
    plan.destroy()
    for o in ref.values():
        o.destroy()
    for a in ops:
        a.destroy()
    n_out = sum(expect)
    planned["graph_output_nnz_per_s"] = n_out / planned["graph_s"]
    planned["sampled_bit_identical"] = bool(ok_plan)
    return {
        "workload": f"{count} FD self-compositions (2-D 5-point / 3-D 7-point, 50/50, grid side U{{8..64}}, "
                    "seed 4096), one operand per instance, all resident in HBM",
        "instances": count, "input_nnz": n_in, "output_nnz": n_out,
        "plain_s": res["plain"], "batched_s": res["batched"],
        "plain_output_nnz_per_s": n_out / res["plain"], "batched_output_nnz_per_s": n_out / res["batched"],
        "speedup_batched_vs_plain": res["plain"] / res["batched"],
        "instances_batched": stats[0], "instances_per_call": stats[1], "instances_persistent": stats[2],
        "nnz_closed_form_ok": bool(ok_nnz), "sampled_bit_identical": bool(ok_bits), "sampled": len(sample),
        "values_closed_form_ok": not bad_vals, "values_checked": count, "values_closed_form_failures": bad_vals[:8],
        "values_check_s": t_check,
        "reps": reps, "planned": planned,
        "speedup_graph_vs_plain": res["plain"] / planned["graph_s"],
    }


def batch_profile_leg(lco, ctx, torch, np, L, count: int):
    """The batched work of the batched leg alone (for profilers): two lco_contract_batch calls over the
    same instances, then a planned batch executed once and replayed once as a graph."""
    inst = L.batched_fd_instances(count)
    distinct = {}
    for dim, side in sorted(set(inst)):
        c, v = L.fd_laplacian(side, dim)
        distinct[(dim, side)] = lco.lco_create(ctx, [side] * (2 * dim),
                                               torch.from_numpy(c.view(np.int64).reshape(-1).copy()).to("cuda:0"),
                                               torch.from_numpy(v).to("cuda:0"), lco.LCO_COORDS)
    ops = [lco.lco_create(ctx, distinct[k].dims, distinct[k].livs(), distinct[k].vals(), lco.LCO_SORTED)
           for k in inst]
    for t in distinct.values():
        t.destroy()
    items = [(a, *fd_labels(dim)[:1], a, *fd_labels(dim)[1:]) for a, (dim, _) in zip(ops, inst)]
    out = {}
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = lco.lco_contract_batch(ctx, items)
        torch.cuda.synchronize()
        out[f"batched_s_{rep}"] = time.perf_counter() - t0
        for o in outs:
            o.destroy()
    plan = lco.BatchPlan(ctx, items)
    plan.execute()
    plan.graph_launch()
    torch.cuda.synchronize()
    plan.destroy()
    for a in ops:
        a.destroy()
    return out


def serving_leg(lco, ctx, torch, np, L, seconds: float, workers: int, stress: float):
    """Replay a Poisson request trace in real time against the continuous-batching server, then
    the same trace against serial plain calls (one worker, one request at a time, FIFO).  With
    `stress` > 1 the same trace is replayed once more with arrival times divided by `stress`."""
    t_arr, cls, param = L.serving_trace(seconds)
    n = len(t_arr)
    dev = torch.device("cuda", 0)

    def make(coords, vals, dims, flags):
        return lco.lco_create(ctx, dims, coords.reshape(-1).contiguous(), vals, flags)

    pool = {}
    for c, p in sorted(set(zip(cls.tolist(), param.tolist()))):
        if c in (0, 1):
            dim = 2 + c
            co, va = L.fd_laplacian_torch(p, dim, dev)
            pool[(c, p)] = make(co, va, [p] * (2 * dim), lco.LCO_COORDS)
        else:
            pair = []
            for seed in (1, 2):
                co, va = L.kronecker_hypersparse_torch(p, 1 << (p + 8), seed, dev)
                pair.append(make(co, va, [1 << p] * 4, lco.LCO_COORDS | lco.LCO_SUM_DUPLICATES))
            pool[(c, p)] = tuple(pair)
        del co, va
    torch.cuda.synchronize()

    def request(i):
        c, p = int(cls[i]), int(param[i])
        if c == 2:
            a, b = pool[(c, p)]
            return (a, [0, 1, 2, 3], b, [2, 3, 4, 5], [0, 1, 4, 5])
        a = pool[(c, p)]
        la, lb, lc = fd_labels(2 + c)
        return (a, la, a, lb, lc)

    # the smallest request of each class is kept and compared with a plain call on its own
    probe = {}
    for i in range(n):
        k = int(cls[i])
        if k not in probe or param[i] < param[probe[k]]:
            probe[k] = i

    def replay(server, scale):
        lat = np.zeros(n)
        nnz = np.zeros(n, dtype=np.int64)
        bs = np.zeros(n, dtype=np.int64)
        kept = {}
        bad = []
        base = 0
        for k in probe.values():  # warm-up: one request per class, drained before the clock starts
            base = server.submit(*request(k)) + 1
        server.drain()
        for r in server.poll():
            if r["out"] is not None:
                r["out"].destroy()

        received = [0]

        def handle(results):
            for r in results:
                received[0] += 1
                i = r["ticket"] - base
                if r["status"] != 0 or r["out"] is None:
                    bad.append(i)
                    continue
                lat[i], bs[i] = r["latency_ms"], r["batch_size"]
                nnz[i] = r["out"].nnz
                if i in probe.values():
                    kept[i] = r["out"]  # read after the replay
                else:
                    r["out"].destroy()

        t0 = time.perf_counter()
        for i in range(n):
            target = t0 + t_arr[i] / scale
            while True:
                handle(server.poll())
                now = time.perf_counter()
                if now >= target:
                    break
                time.sleep(min(target - now, 2e-4))
            server.submit(*request(i))
        # drain while consuming results (completed outputs are the caller's memory)
        while received[0] < n:
            handle(server.poll())
            if received[0] < n:
                time.sleep(2e-4)
        wall = time.perf_counter() - t0
        for i, t in list(kept.items()):
            kept[i] = t.to_numpy()
            t.destroy()
        return lat, nnz, bs, kept, bad, wall

    out = {"workload": f"Poisson trace, 200 req/s for {seconds:g} s (seed 5): 70% 2-D 5-point FD compositions "
                       "(side 16..96), 25% 3-D 7-point (side 64..128), 5% hyper-sparse Kronecker pairs "
                       "(2^L per mode, L 12..16, 2^(L+8) draws); operands resident in HBM",
           "requests": n}

    def run_modes(scale):
        res = {}
        for name, kw in (("served", dict(workers=workers, max_batch=256, plain=False)),
                         ("serial_plain", dict(workers=1, max_batch=1, plain=True))):
            note(f"serving: {name} replay at x{scale:g} ({n} requests)")
            srv = lco.Server(0, **kw)
            try:
                lat, nnz, bs, kept, bad, wall = replay(srv, scale)
            finally:
                srv.destroy()
            ok = lat > 0
            per = {}
            for c, cname in enumerate(("fd2", "fd3", "kron")):
                m = ok & (cls == c)
                if m.any():
                    per[cname] = {"n": int(m.sum()), "p50_ms": float(np.percentile(lat[m], 50)),
                                  "p99_ms": float(np.percentile(lat[m], 99))}
            res[name] = {"p50_ms": float(np.percentile(lat[ok], 50)), "p99_ms": float(np.percentile(lat[ok], 99)),
                         "mean_ms": float(lat[ok].mean()), "req_per_s": float(ok.sum() / wall),
                         "output_nnz_per_s": float(nnz[ok].sum() / wall), "wall_s": wall, "errors": len(bad),
                         "mean_batch": float(bs[ok].mean()), "max_batch": int(bs[ok].max()), "per_class": per,
                         "config": kw}
            res[name + "_nnz"] = nnz
            res[name + "_kept"] = kept
        return res

    out.update(run_modes(1.0))
    # every request: identical output size in both modes; FD sizes equal the closed form
    same = bool(np.array_equal(out.pop("served_nnz"), out["serial_plain_nnz"]))
    fdn = out.pop("serial_plain_nnz")
    fd_ok = all(fdn[i] == fd_compose_nnz(2 + int(cls[i]), int(param[i])) for i in range(n) if cls[i] < 2)
    # probes: served result == serial plain result == a plain call on the main context
    ks, kp = out.pop("served_kept"), out.pop("serial_plain_kept")
    ident = True
    for i in probe.values():
        a = lco.lco_contract(ctx, *request(i))
        _, la_, va_ = a.to_numpy()
        a.destroy()
        for kept in (ks, kp):
            ident &= i in kept and np.array_equal(kept[i][1], la_) and \
                np.array_equal(kept[i][2].view(np.uint64), va_.view(np.uint64))
    if stress > 1:
        st = run_modes(stress)
        same &= bool(np.array_equal(st["served_nnz"], fdn)) and bool(np.array_equal(st["serial_plain_nnz"], fdn))
        out[f"stress_x{stress:g}"] = {"offered_req_per_s": 200.0 * stress, "served": st["served"],
                                      "serial_plain": st["serial_plain"],
                                      "p99_speedup_served_vs_plain":
                                          st["serial_plain"]["p99_ms"] / st["served"]["p99_ms"]}
    for t in pool.values():
        for x in (t if isinstance(t, tuple) else (t,)):
            x.destroy()
    out["nnz_same_served_vs_plain"] = same
    out["fd_nnz_closed_form_ok"] = bool(fd_ok)
    out["probes_bit_identical"] = bool(ident)
    out["p99_speedup_served_vs_plain"] = out["serial_plain"]["p99_ms"] / out["served"]["p99_ms"]
    return out


def small_leg(lco, ctx, torch, np, L, reps: int):
    """The 32x32 2-D FD operator (4,992 non-zeros): permutation (2,3,0,1) then the biharmonic
    self-contraction; latency-bound, so per-call p50/p99 over many repetitions."""
    c, v = L.fd_laplacian(32, 2)
    idx_d = torch.from_numpy(c.view(np.int64).reshape(-1).copy()).to("cuda:0")
    val_d = torch.from_numpy(v).to("cuda:0")
    A = lco.lco_create(ctx, [32] * 4, idx_d, val_d, lco.LCO_COORDS)
    la, lb, lc = fd_labels(2)
    res = {}
    for name in ("permute", "contract", "permute+contract"):
        t = []
        for k in range(reps + 20):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "permute":
                P = lco.lco_permute(ctx, A, [2, 3, 0, 1])
                ctx.synchronize()
                P.destroy()
            elif name == "contract":
                C = lco.lco_contract(ctx, A, la, A, lb, lc)
                ctx.synchronize()
                n_out = C.nnz
                C.destroy()
            else:
                P = lco.lco_permute(ctx, A, [2, 3, 0, 1])
                C = lco.lco_contract(ctx, P, la, P, lb, lc)
                ctx.synchronize()
                C.destroy()
                P.destroy()
            if k >= 20:
                t.append((time.perf_counter() - t0) * 1e6)
        res[name] = {"p50_us": float(np.percentile(t, 50)), "p99_us": float(np.percentile(t, 99))}
    A.destroy()
    return {"workload": "2-D 5-point FD Laplacian 32x32 (4,992 nnz): permute (2,3,0,1); self-contraction "
                        "over (2,3)x(0,1)", "nnz_out": n_out, "reps": reps, **res}


def hyper_leg(lco, ctx, torch, np, L, reps: int, forced: bool = True):
    """The order-4 hyper-sparse Kronecker pair (2^16 per mode, 2^24 draws each, duplicates summed),
    contracted over (2,3)x(0,1): index-sparse x index-sparse, where the selector measured on MI355X takes
    DCSC (no rearrangement) and the paper's table SOP (B permuted (2,3,0,1)); both are timed."""
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(2) as ex:  # the seeded PCG64 recipe on the host, both operands at once
        host = list(ex.map(lambda seed: L.kronecker_hypersparse(16, 1 << 24, seed), (1, 2)))
    ops = []
    for co, va in host:
        idx = torch.from_numpy(co.view(np.int64).reshape(-1)).to("cuda:0")
        ops.append(lco.lco_create(ctx, [1 << 16] * 4, idx, torch.from_numpy(va).to("cuda:0"),
                                  lco.LCO_COORDS | lco.LCO_SUM_DUPLICATES))
        del idx
    del host
    A, B = ops
    assert (A.nnz, B.nnz) == (16777201, 16777183), (A.nnz, B.nnz)
    la, lb, lc = [0, 1, 2, 3], [2, 3, 4, 5], [0, 1, 4, 5]
    plan = lco.lco_plan_info(ctx, A, la, B, lb, lc).as_dict()
    paper_ctx = lco.lco_ctx_create(0)
    lco.lco_ctx_use_paper_selector(paper_ctx)
    paper_algo = lco.lco_plan_info(paper_ctx, A, la, B, lb, lc).as_dict()["algo_name"]
    paper_ctx.destroy()
    C = lco.lco_contract(ctx, A, la, B, lb, lc)  # warm-up
    C.destroy()
    t = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        C = lco.lco_contract(ctx, A, la, B, lb, lc)
        ctx.synchronize()
        t.append(time.perf_counter() - t0)
        n_out = C.nnz
        C.destroy()
    # per-kernel breakdown from one more call with every launch bracketed by HIP events
    lco.lco_timing_reset(ctx)
    lco.lco_timing_enable(ctx, True)
    C = lco.lco_contract(ctx, A, la, B, lb, lc)
    ctx.synchronize()
    C.destroy()
    lco.lco_timing_enable(ctx, False)
    kernels = {}
    for name in lco.lco_timing_kernels(ctx):
        n_l, tot = lco.lco_timing_query(ctx, name)
        if n_l:
            kernels[name] = {"launches_per_rep": n_l, "ms_per_rep": tot}
    lco.lco_timing_reset(ctx)
    ms = statistics.median(t) * 1e3
    # the same product through the other algorithms of the cell (SOP: the paper's table's choice)
    ref = lco.lco_contract(ctx, A, la, B, lb, lc)
    alt = {}
    for name in [x for x in ("SOP", "DCSC", "DCSR") if x != plan["algo_name"] and forced]:
        f = lco.ALGO_IDS[name]
        C = lco.lco_contract(ctx, A, la, B, lb, lc, f)
        C.destroy()
        tt = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            C = lco.lco_contract(ctx, A, la, B, lb, lc, f)
            ctx.synchronize()
            tt.append(time.perf_counter() - t0)
            if len(tt) < reps:
                C.destroy()
        same = torch.equal(C.livs(), ref.livs()) and torch.equal(C.vals().view(torch.int64),
                                                                  ref.vals().view(torch.int64))
        C.destroy()
        alt[name] = {"ms": statistics.median(tt) * 1e3, "bit_identical_to_selected": bool(same)}
    ref.destroy()
    assert n_out == 118827201, n_out
    out = {"workload": "hyper-sparse Kronecker pair, order 4, 2^16 per mode, 2^24 draws each (PCG64 seeds 1/2, "
                       "duplicates summed), contracted over (2,3)x(0,1)",
           "nnz_a": A.nnz, "nnz_b": B.nnz, "nnz_out": n_out, "algo": plan["algo_name"],
           "permute_b": plan["permute_b"], "ms": ms, "output_nnz_per_s": n_out / (ms * 1e-3), "reps": reps,
           "paper_table_algo": paper_algo, "forced": alt,
           "kernels": dict(sorted(kernels.items(), key=lambda kv: -kv[1]["ms_per_rep"])[:12])}
    A.destroy()
    B.destroy()
    return out


def app_leg(lco, ctx, torch, np, L, n: int, reps: int):
    """The design tensor of the paper's Section 2 (combinatorial Laplacian) on an n x n image, n = 2^k - 1:
    a_ijlk = d_ii' delta_jl d_i'k + d_jj' delta_ik d_j'l, executed left to right as binary operations
    (two outer products with Kronecker deltas, the two hyper-sparse products of Section 6, one addition
    whose second term is re-sorted {1,0,3,2} first)."""
    I, J, K, LL, I2, J2 = 0, 1, 2, 3, 4, 5

    def up(c, v):
        return lco.lco_create(ctx, [n, n], torch.from_numpy(c.view(np.int64).reshape(-1).copy()).to("cuda:0"),
                              torch.from_numpy(v).to("cuda:0"), lco.LCO_COORDS)

    d = up(*L.fd_first_derivative(n))
    delta = up(*L.diagonal(2, n, np.ones(n)))

    def chain():
        by = lco.lco_contract(ctx, d, [I, I2], delta, [J, LL], [I, I2, J, LL])
        ty = lco.lco_contract(ctx, by, [I, I2, J, LL], d, [I2, K], [I, J, LL, K])
        bx = lco.lco_contract(ctx, d, [J, J2], delta, [I, K], [J, J2, I, K])
        tx = lco.lco_contract(ctx, bx, [J, J2, I, K], d, [J2, LL], [J, I, K, LL])
        a = lco.lco_add(ctx, ty, [I, J, LL, K], tx, [J, I, K, LL], [I, J, LL, K])
        return by, ty, bx, tx, a

    def timed(fn):
        fn()  # warm-up
        t = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            ctx.synchronize()
            t.append((time.perf_counter() - t0) * 1e3)
            for x in (r if isinstance(r, tuple) else (r,)):
                x.destroy()
        return statistics.median(t)

    ms_chain = timed(chain)
    by, ty, bx, tx, a = chain()
    plan = lco.lco_plan_info(ctx, by, [I, I2, J, LL], d, [I2, K], [I, J, LL, K]).as_dict()
    ms_prod = timed(lambda: lco.lco_contract(ctx, by, [I, I2, J, LL], d, [I2, K], [I, J, LL, K]))
    ms_prods = timed(lambda: (lco.lco_contract(ctx, by, [I, I2, J, LL], d, [I2, K], [I, J, LL, K]),
                              lco.lco_contract(ctx, bx, [J, J2, I, K], d, [J2, LL], [J, I, K, LL])))
    ms_add = timed(lambda: lco.lco_add(ctx, ty, [I, J, LL, K], tx, [J, I, K, LL], [I, J, LL, K]))
    # per-kernel breakdown of the addition from a second round with every launch bracketed by HIP events
    lco.lco_timing_reset(ctx)
    lco.lco_timing_enable(ctx, True)
    timed(lambda: lco.lco_add(ctx, ty, [I, J, LL, K], tx, [J, I, K, LL], [I, J, LL, K]))
    lco.lco_timing_enable(ctx, False)
    kernels = {}
    for name in lco.lco_timing_kernels(ctx):
        n_l, tot = lco.lco_timing_query(ctx, name)
        if n_l:
            kernels[name] = {"launches_per_add": n_l / (reps + 1), "avg_ms": tot / n_l}
    lco.lco_timing_reset(ctx)
    na, nb, nc = ty.nnz, tx.nnz, a.nnz
    add_bytes = 32 * nb + 16 * (na + nb) + 16 * nc  # permute b, read both, write the sum
    roof = None
    if "add_write" in kernels:
        wb = 16 * (na + nb) + 16 * nc
        ach = wb / (kernels["add_write"]["avg_ms"] * 1e-3) / 1e9
        kernels["add_write"]["algorithmic_GBps"] = ach
        roof = {"kernel": "add_write", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBPS, "traffic": measured_traffic("add_write", APP_WORKLOAD),
                "algorithmic_bytes_per_launch": wb, "avg_launch_ms": kernels["add_write"]["avg_ms"]}
    if "add_count" in kernels:
        kernels["add_count"]["algorithmic_GBps"] = 8 * (na + nb) / (kernels["add_count"]["avg_ms"] * 1e-3) / 1e9
    out = {"workload": f"combinatorial Laplacian (Section 2) on a {n}x{n} image: two outer products with "
                       "Kronecker deltas, two hyper-sparse products (Section 6), one addition with the "
                       "{1,0,3,2} re-sort",
           "n": n, "nnz_by": by.nnz, "nnz_term": ty.nnz, "nnz_design_tensor": nc,
           "hyper_sparse_product": {"algo": plan["algo_name"], "a_class": plan["a_class_name"],
                                    "b_class": plan["b_class_name"], "ms": ms_prod,
                                    "output_nnz_per_s": ty.nnz / (ms_prod * 1e-3)},
           "both_hyper_sparse_products_ms": ms_prods,
           "design_tensor_ms": ms_chain, "design_tensor_nnz_per_s": nc / (ms_chain * 1e-3),
           "add": {"ms": ms_add, "effective_GBps": add_bytes / (ms_add * 1e-3) / 1e9,
                   "bytes_algorithmic": add_bytes, "roofline": roof, "kernels": kernels},
           "paper_context": "E8400, 1 core, sequential: both hyper-sparse products at n = 2047 in 2.0 s "
                            "(poly-algorithm, operand rearrangement included); adding the two terms 2.7 s after a "
                            "4.9 s re-sort (largest n of that test)"}
    for t in (by, ty, bx, tx, a, d, delta):
        t.destroy()
    return out


def rp_leg(lco, ctx, torch, np, L, n: int, reps: int):
    """The paper's permutation experiment (Section 4.2, Table rp_timings): all 23 non-identity permutations
    of the fourth-order combinatorial Laplacian a_ijkl (Section 2) at n = 2^11.5 (rounded), built on the
    device by the library itself.  Each permutation is timed end to end (median); effective GB/s counts
    32 bytes per non-zero (read LIV + value, write LIV + value)."""
    import itertools
    I, J, K, LL, I2, J2 = 0, 1, 2, 3, 4, 5

    def up(c, v):
        return lco.lco_create(ctx, [n, n], torch.from_numpy(c.view(np.int64).reshape(-1).copy()).to("cuda:0"),
                              torch.from_numpy(v).to("cuda:0"), lco.LCO_COORDS)

    d = up(*L.fd_first_derivative(n))
    delta = up(*L.diagonal(2, n, np.ones(n)))
    by = lco.lco_contract(ctx, d, [I, I2], delta, [J, LL], [I, I2, J, LL])
    ty = lco.lco_contract(ctx, by, [I, I2, J, LL], d, [I2, K], [I, J, LL, K])
    by.destroy()
    bx = lco.lco_contract(ctx, d, [J, J2], delta, [I, K], [J, J2, I, K])
    tx = lco.lco_contract(ctx, bx, [J, J2, I, K], d, [J2, LL], [J, I, K, LL])
    bx.destroy()
    a = lco.lco_add(ctx, ty, [I, J, LL, K], tx, [J, I, K, LL], [I, J, K, LL])
    for t in (ty, tx, d, delta):
        t.destroy()
    nnz = a.nnz
    rows = []
    for perm in itertools.permutations(range(4)):
        if perm == (0, 1, 2, 3):
            continue
        plan = lco.lco_plan_permute([n] * 4, list(perm), nnz).as_dict()
        P = lco.lco_permute(ctx, a, list(perm))
        ctx.synchronize()
        P.destroy()
        t = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P = lco.lco_permute(ctx, a, list(perm))
            ctx.synchronize()
            t.append((time.perf_counter() - t0) * 1e3)
            P.destroy()
        ms = statistics.median(t)
        rows.append({"perm": "{" + ",".join(map(str, perm)) + "}", "ms": ms,
                     "effective_GBps": 32.0 * nnz / (ms * 1e-3) / 1e9, "method": plan["method"],
                     "key_bits": plan["key_bits"], "passes": plan["passes"]})
    a.destroy()
    by_perm = {r["perm"]: r for r in rows}
    ms_sorted = sorted(r["ms"] for r in rows)
    paper = {"{3,1,2,0}": 3.54, "{2,1,3,0}": 3.45, "{1,0,2,3}": 1.38}
    return {"workload": f"combinatorial Laplacian a_ijkl (Section 2), n = {n} (2^11.5 rounded), "
                        "all 23 non-identity permutations",
            "n": n, "nnz": nnz, "reps": reps,
            "min_ms": ms_sorted[0], "median_ms": ms_sorted[len(ms_sorted) // 2], "max_ms": ms_sorted[-1],
            "paper_rows": {p: {"ms": by_perm[p]["ms"], "effective_GBps": by_perm[p]["effective_GBps"],
                               "paper_RP_s_E8400": paper[p]} for p in paper},
            "perms": rows}


def calibrate_leg(lco, ctx, torch, np, L, reps: int):
    """The paper's hyper-sparsity sweeps (Sections 5.2.3-5.2.5) repeated on this GPU with R-TENSORs
    (Section 5.2.1): column-sparsity (a_ijk b_ljk, CSC vs DCSC), row-sparsity (a_ijk b_lmk, CSC vs CSCNA) and
    index-sparsity (M x N x N tensors with M = N^2, a_ijk b_ljk, CSC vs SOP, and DCSC beside both).  Each point
    times the forced algorithms end to end (median of `reps`); a crossover is where the alternative starts to win
    for good."""
    dev = torch.device("cuda", 0)

    def make(bits, draws, seed, extra=0):
        c, v = L.rtensor(bits, draws, seed, first_extra_bits=extra)
        dims = [1 << (bits + extra), 1 << bits, 1 << bits]
        t = lco.lco_create(ctx, dims, torch.from_numpy(c.view(np.int64).reshape(-1).copy()).to(dev),
                           torch.from_numpy(v).to(dev), lco.LCO_COORDS | lco.LCO_SUM_DUPLICATES)
        return t

    def timed(a, la, b, lb, lc, algo, on=None):
        on = on or ctx
        f = 0 if algo == "auto" else lco.ALGO_IDS[algo]
        lco.lco_contract(on, a, la, b, lb, lc, f).destroy()
        t = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c = lco.lco_contract(on, a, la, b, lb, lc, f)
            on.synchronize()
            t.append((time.perf_counter() - t0) * 1e3)
            c.destroy()
        return statistics.median(t)

    tuned_ctx = lco.lco_ctx_create(0)
    lco.lco_ctx_use_mi355x_selector(tuned_ctx)
    paper_ctx = lco.lco_ctx_create(0)
    lco.lco_ctx_use_paper_selector(paper_ctx)
    totals = {"paper_ms": 0.0, "mi355x_ms": 0.0, "changed_points": 0, "changed_paper_ms": 0.0,
              "changed_mi355x_ms": 0.0}

    def crossover(rows):
        rows = sorted(rows, key=lambda r: r["sparsity"])
        for i in range(len(rows)):
            if all(r["ratio"] > 1.0 for r in rows[i:]):
                if i == 0:
                    return rows[0]["sparsity"]
                return (rows[i - 1]["sparsity"] * rows[i]["sparsity"]) ** 0.5
        return None

    exps = {
        "column_sparsity": {"spec": "a_ijk b_ljk", "alt": "DCSC", "draws": (400_000, 700_000, 1_000_000),
                            "bits": range(9, 15), "extra": 0, "lab": ([0, 1, 2], [3, 1, 2], [0, 3]),
                            "paper_crossover": 10, "paper_threshold": 3},
        "row_sparsity": {"spec": "a_ijk b_lmk", "alt": "CSCNA", "draws": (100_000, 200_000, 300_000),
                         "bits": range(8, 14), "extra": 0, "lab": ([0, 1, 2], [3, 4, 2], [0, 1, 3, 4]),
                         "paper_crossover": 3, "paper_threshold": 3},
        "index_sparsity": {"spec": "a_ijk b_ljk, M x N x N with M = N^2", "alt": "SOP", "alt2": "DCSC",
                           "draws": (50_000, 100_000, 1_000_000),
                           "bits": range(7, 16), "extra": None, "lab": ([0, 1, 2], [3, 1, 2], [0, 3]),
                           "paper_crossover": 6, "paper_threshold": 3},
    }
    out = {}
    seed = 100
    for name, e in exps.items():
        rows = []
        la, lb, lc = e["lab"]
        for draws in e["draws"]:
            for bits in e["bits"]:
                extra = bits if e["extra"] is None else e["extra"]
                a = make(bits, draws, seed, extra)
                b = make(bits, draws, seed + 1, extra)
                seed += 2
                plan = lco.lco_plan_info(paper_ctx, a, la, b, lb, lc).as_dict()
                sp = (plan["k"] if name == "column_sparsity" else plan["m"]) / max(1, a.nnz)
                t_csc = timed(a, la, b, lb, lc, "CSC")
                t_alt = timed(a, la, b, lb, lc, e["alt"])
                t_alt2 = timed(a, la, b, lb, lc, e["alt2"]) if "alt2" in e else None
                t_paper = timed(a, la, b, lb, lc, "auto", paper_ctx)
                t_tuned = timed(a, la, b, lb, lc, "auto", tuned_ctx)
                totals["paper_ms"] += t_paper
                totals["mi355x_ms"] += t_tuned
                tuned = lco.lco_plan_info(tuned_ctx, a, la, b, lb, lc).as_dict()
                if tuned["algo_name"] != plan["algo_name"]:
                    totals["changed_points"] += 1
                    totals["changed_paper_ms"] += t_paper
                    totals["changed_mi355x_ms"] += t_tuned
                rows.append({"draws": draws, "bits": bits, "nnz_a": a.nnz, "sparsity": sp, "csc_ms": t_csc,
                             "alt_ms": t_alt, "ratio": t_csc / t_alt, "selected": plan["algo_name"],
                             "selected_mi355x": tuned["algo_name"], "auto_ms": t_paper, "auto_mi355x_ms": t_tuned})
                if t_alt2 is not None:
                    rows[-1].update({"alt2_ms": t_alt2, "ratio_alt_over_alt2": t_alt / t_alt2,
                                     "ratio_csc_over_alt2": t_csc / t_alt2})
                print(f"calibration {name} draws={draws} bits={bits} sparsity={sp:.2f} "
                      f"CSC {t_csc:.3f} ms {e['alt']} {t_alt:.3f} ms"
                      + (f" {e['alt2']} {t_alt2:.3f} ms" if t_alt2 is not None else "")
                      + f" auto {tuned['algo_name']} {t_tuned:.3f} ms", file=sys.stderr, flush=True)
                a.destroy()
                b.destroy()
        if "alt2" in e:
            out[name + "_" + e["alt2"].lower()] = {
                "product": e["spec"], "alternatives": [e["alt"], e["alt2"]],
                "crossover_vs_csc": crossover([{"sparsity": r["sparsity"], "ratio": r["ratio_csc_over_alt2"]}
                                               for r in rows]),
                "crossover_vs_sop": crossover([{"sparsity": r["sparsity"], "ratio": r["ratio_alt_over_alt2"]}
                                               for r in rows])}
        out[name] = {"product": e["spec"], "alternative": e["alt"], "crossover": crossover(rows),
                     "paper_crossover_E8400": e["paper_crossover"], "paper_threshold": e["paper_threshold"],
                     "points": rows}
    tuned_ctx.destroy()
    paper_ctx.destroy()
    out["selector_total"] = {**totals, "crossovers_paper": list(lco.PAPER_CROSSOVERS),
                             "crossovers_mi355x": list(lco.MI355X_CROSSOVERS),
                             "index_algorithm_mi355x": lco.MI355X_INDEX_ALGORITHM,
                             "note": "sums over every sweep point (and over the points whose choice differs) of the "
                                     "automatic choice's median time"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--small-reps", type=int, default=1000, help="repetitions of the 32x32 leg (0: skip)")
    ap.add_argument("--hyper-reps", type=int, default=5, help="repetitions of the hyper-sparse leg (0: skip)")
    ap.add_argument("--hyper-selected-only", action="store_true",
                    help="hyper-sparse leg: time the selected algorithm only (no forced alternatives)")
    ap.add_argument("--app-n", type=int, default=2047, help="image side of the combinatorial Laplacian leg")
    ap.add_argument("--app-reps", type=int, default=5, help="repetitions of the Laplacian leg (0: skip)")
    ap.add_argument("--rp-n", type=int, default=2896, help="side of the Laplacian in the permutation-table leg")
    ap.add_argument("--rp-reps", type=int, default=3, help="repetitions per permutation in that leg (0: skip)")
    ap.add_argument("--batch-count", type=int, default=4096, help="instances in the batched leg (0: skip)")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the replayed request trace (0: skip the serving leg)")
    ap.add_argument("--serve-workers", type=int, default=3)
    ap.add_argument("--serve-stress", type=float, default=4.0,
                    help="also replay the trace this many times faster (<= 1: skip)")
    ap.add_argument("--copy-probe-only", action="store_true",
                    help="run only the 1 GiB device copy (the reference kernel for HBM counter scaling)")
    ap.add_argument("--app-only", action="store_true", help="run only the combinatorial Laplacian leg")
    ap.add_argument("--rp-only", action="store_true", help="run only the permutation-table leg")
    ap.add_argument("--hyper-only", action="store_true", help="run only the hyper-sparse (SOP) leg")
    ap.add_argument("--batch-only", action="store_true", help="run only the batched leg")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving leg")
    ap.add_argument("--batch-profile", action="store_true",
                    help="run only the batched work of the batched leg, without the per-call loop and checks")
    ap.add_argument("--calibrate", action="store_true",
                    help="run only the selector calibration sweeps (R-TENSORs, Sections 5.2.3-5.2.5)")
    ap.add_argument("--calibrate-reps", type=int, default=3)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one MI355X only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU sharding of this path is described, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import lco_inputs as L
    import paper_1802_02619_amd as lco

    only = (args.copy_probe_only or args.app_only or args.calibrate or args.rp_only or args.hyper_only or
            args.batch_only or args.batch_profile or args.serve_only)
    coords = vals = cb = None
    if not only:
        coords, vals = L.fd_laplacian(SIDE, 3)
        if not args.no_cpu_baseline:
            # the oracle runs first, on one pinned core, before anything touches the GPU
            note("cpu baseline (oracle, one pinned core)")
            cb, (rows, c_sub) = cpu_baseline(coords, vals)
    torch.cuda.set_device(0)
    if args.copy_probe_only:
        print(json.dumps({"copy_GBps": copy_ceiling(torch), "bytes_each_way": 1 << 30}), flush=True)
        return
    ctx = lco.lco_ctx_create(0)
    if args.app_only:
        print(json.dumps({"laplacian": app_leg(lco, ctx, torch, np, L, args.app_n, max(1, args.app_reps))}),
              flush=True)
        return
    if args.calibrate:
        print(json.dumps({"calibration": calibrate_leg(lco, ctx, torch, np, L, args.calibrate_reps)}), flush=True)
        return
    if args.rp_only:
        print(json.dumps({"rp_table": rp_leg(lco, ctx, torch, np, L, args.rp_n, max(1, args.rp_reps))}), flush=True)
        return
    if args.hyper_only:
        print(json.dumps({"hyper_sparse": hyper_leg(lco, ctx, torch, np, L, max(1, args.hyper_reps),
                                                    not args.hyper_selected_only)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": serving_leg(lco, ctx, torch, np, L, args.serve_seconds, args.serve_workers,
                                                 args.serve_stress)}), flush=True)
        return
    if args.batch_profile:
        print(json.dumps({"batch_profile": batch_profile_leg(lco, ctx, torch, np, L, max(1, args.batch_count))}),
              flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batched": batched_leg(lco, ctx, torch, np, L, max(1, args.batch_count),
                                                 max(1, args.batch_reps))}), flush=True)
        return
    idx_d = torch.from_numpy(coords.view(np.int64).reshape(-1).copy()).to("cuda:0")
    val_d = torch.from_numpy(vals).to("cuda:0")
    A = lco.lco_create(ctx, [SIDE] * 6, idx_d, val_d, lco.LCO_COORDS)
    del idx_d, val_d
    nnz_in = A.nnz

    def step():
        P = lco.lco_permute(ctx, A, PERM)
        C = lco.lco_contract(ctx, P, LA, P, LB, LC)
        nc = C.nnz
        C.destroy()
        P.destroy()
        return nc

    nnz_c = 0
    for _ in range(args.warmup):
        nnz_c = step()
    torch.cuda.synchronize()
    plan = lco.lco_plan_info(ctx, A, LA, A, LB, LC).as_dict()

    # ---- per-kernel breakdown, from separate steps with every launch bracketed by HIP events on the
    # library stream (two event records per launch cost device time, so the timed region below brackets
    # only the dominant kernel)
    prof_steps = max(1, min(args.steps, 5))
    lco.lco_timing_reset(ctx)
    lco.lco_timing_only(ctx, None)
    lco.lco_timing_enable(ctx, True)
    for _ in range(prof_steps):
        step()
    torch.cuda.synchronize()
    lco.lco_timing_enable(ctx, False)
    kernels = {}
    for name in lco.lco_timing_kernels(ctx):
        n_l, tot = lco.lco_timing_query(ctx, name)
        if n_l:
            kernels[name] = {"launches_per_step": n_l / prof_steps, "avg_ms": tot / n_l,
                             "ms_per_step": tot / prof_steps}
    dom = max(kernels, key=lambda n: kernels[n]["ms_per_step"]) if kernels else None

    # ---- timed region: K steps; HIP events on the library stream around each launch of the dominant kernel
    lco.lco_timing_reset(ctx)
    lco.lco_timing_only(ctx, dom)
    lco.lco_timing_enable(ctx, dom is not None)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record()
        nnz_c = step()
        ends[k].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lco.lco_timing_enable(ctx, False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    step_ms = sorted(s.elapsed_time(e) for s, e in zip(starts, ends))
    dom_launches, dom_ms = lco.lco_timing_query(ctx, dom) if dom is not None else (0, 0.0)
    lco.lco_timing_only(ctx, None)
    lco.lco_timing_reset(ctx)

    # ---- permutation alone (effective GB/s: 32 bytes per non-zero moved)
    pe0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    pe1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    for k in range(args.steps):
        pe0[k].record()
        P = lco.lco_permute(ctx, A, PERM)
        pe1[k].record()
        P.destroy()
    torch.cuda.synchronize()
    perm_ms = statistics.median(a.elapsed_time(b) for a, b in zip(pe0, pe1))
    perm_gbps = 32.0 * nnz_in / (perm_ms * 1e-3) / 1e9
    # what the radix passes themselves move: per pass a digit count (8 B read per entry) and a
    # scatter (16 B read + 16 B written), by the model and by the committed counter summary
    rp = lco.lco_plan_permute([SIDE] * 6, PERM, nnz_in).as_dict()
    pass_bytes = rp["passes"] * 40.0 * nnz_in
    cnt_tr, sct_tr = measured_traffic("rx_count"), measured_traffic("rx_scatter")
    counter_bytes = rp["passes"] * (cnt_tr + sct_tr) if cnt_tr and sct_tr else None

    # ---- roofline of the dominant kernel, from its launches in the timed region
    sizes = {"n": nnz_in, "nnz_a": nnz_in, "nnz_b": nnz_in, "nnz_c": nnz_c, "k": SIDE**3, "rows": SIDE**3}
    roof = None
    if dom is not None and dom_launches:
        ab = algorithmic_bytes(dom, sizes)
        avg_ms = dom_ms / dom_launches
        ach = ab / (avg_ms * 1e-3) / 1e9 if ab else None
        tr = measured_traffic(dom, MAIN_WORKLOAD)
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": (ach / HBM_PEAK_GBPS) if ach else None, "traffic": tr,
                "algorithmic_bytes_per_launch": ab, "avg_launch_ms": avg_ms,
                "launches_timed": dom_launches}

    out = {
        "metric": "output nnz/s + permute GB/s (%HBM peak), batched/served vs plain; p50/p99 ms",
        "value": nnz_c / (ms_per_step * 1e-3),
        "unit": "output nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "p50_ms": step_ms[len(step_ms) // 2],
        "p99_ms": step_ms[min(len(step_ms) - 1, int(round(0.99 * (len(step_ms) - 1))))],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "order-6 FD Laplacian, 128^3 grid, Dirichlet: radix permutation (1..6)->(4,5,6,1,2,3) "
                        "then self-contraction over 3 modes",
            "dims": [SIDE] * 6, "nnz_in": nnz_in, "nnz_out": nnz_c, "algo": plan["algo_name"],
            "index": "u64 LIV", "parallelism": "single GPU",
        },
        "copy_ceiling_GBps": copy_ceiling(torch),
        "permute": {"ms": perm_ms, "effective_GBps": perm_gbps, "frac_hbm_peak": perm_gbps / HBM_PEAK_GBPS,
                    "bytes_algorithmic": 32 * nnz_in, "key_bits": rp["key_bits"], "passes": rp["passes"],
                    "pass_bytes_model": pass_bytes, "pass_GBps_model": pass_bytes / (perm_ms * 1e-3) / 1e9,
                    "pass_bytes_counters": counter_bytes,
                    "pass_GBps_counters": counter_bytes / (perm_ms * 1e-3) / 1e9 if counter_bytes else None},
        "roofline": roof,
        "kernels": kernels,
        "kernels_steps": prof_steps,
    }
    note(f"main step done: {ms_per_step:.3f} ms/step")
    if args.small_reps > 0:
        note("leg: small")
        out["small"] = small_leg(lco, ctx, torch, np, L, args.small_reps)
    if args.hyper_reps > 0:
        note("leg: hyper_sparse")
        out["hyper_sparse"] = hyper_leg(lco, ctx, torch, np, L, args.hyper_reps)
    if args.app_reps > 0:
        note("leg: laplacian")
        out["laplacian"] = app_leg(lco, ctx, torch, np, L, args.app_n, args.app_reps)
    if args.rp_reps > 0:
        note("leg: rp_table")
        out["rp_table"] = rp_leg(lco, ctx, torch, np, L, args.rp_n, args.rp_reps)
    if args.batch_count > 0:
        note("leg: batched")
        out["batched"] = batched_leg(lco, ctx, torch, np, L, args.batch_count, args.batch_reps)
    if args.serve_seconds > 0:
        note("leg: serving")
        out["serving"] = serving_leg(lco, ctx, torch, np, L, args.serve_seconds, args.serve_workers,
                                     args.serve_stress)
    if cb is not None:
        # the sampled rows of the GPU result must equal the oracle's
        P = lco.lco_permute(ctx, A, PERM)
        C = lco.lco_contract(ctx, P, LA, P, LB, LC)
        _, livs, cv = C.to_numpy()
        pick = np.isin(livs % np.uint64(SIDE**3), rows)
        cb["sample_matches_gpu"] = bool(np.array_equal(livs[pick], c_sub.livs) and
                                        np.array_equal(cv[pick], c_sub.vals))
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
