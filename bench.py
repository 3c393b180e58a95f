#!/usr/bin/env python3
"""Throughput of the fused efunc fit step on one MI355X.

A step is one efunc_fit_step over one minibatch of synthetic points:
moved-key binning, query binning into lattice cells, the tile kernel
(forward, MSE loss, dL/dO and backward with tile-level gradient flush), the
certificate fallback, the FP64 loss reduction and AdamW.  Inputs (a small
pool of pre-generated batches) are resident in HBM before timing starts.

Default workload "csg16_r32": 32^3 x 13 float32 parameters (paper
initialisation: rho = 7, mean-shift offsets from 16,384 surface samples),
target = smooth union (k = 0.05) of 16 seeded spheres/boxes, 2^21 points per
iteration (half uniform in [-1,1]^3, half surface samples + N(0, 0.01^2)).

Prints one JSON line.  Roofline: the dominant kernel (the tile kernel) is
bound by plain FP32 vector ALU work, so `achieved` is algorithmic FP32
operations per launch divided by its event-timed average duration, against
the non-packed FP32 lane-operation peak of the chip (see ROOFLINE_PEAK).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fit points·iters/sec (fused fwd+bwd)"

# Algorithmic FP32 operations per key-query pair (an FMA, add, mul, sub or
# exp2 is one operation).  Two counts are reported:
# * the method's per-pair work as the closed forms state it (the headline
#   fraction): forward 14 VALU + 1 exp (distance, logit, shifted exponent,
#   polynomial, the two running sums); backward 19 VALU + 1 exp per grid
#   pair (recomputed weight and polynomial, delta, r = f - O, the sums for o,
#   d and beta); moved pairs add the centre gradient
#   delta (-d + 2 beta x r), 8 more;
OPS_FWD = 15
OPS_BWD_GRID = 20
OPS_BWD_MOVED = 28
# * the operations this engine's factored form needs per pair:
#   forward:  x = q - c (3), |x|^2 (3), exponent fma (1), exp2 (1),
#             f = o + x.d (3), e += l (1), m += l f (1)                 = 13
#   backward: x (3), |x|^2 (3), exponent fma (1), exp2 (1), f (3),
#             delta = g w (1), u = delta (f - O) (2), sums for o, d, beta
#             (1 + 3 + 1)                                              = 19
#             moved keys add the centre sums u x (3); the -d sum(delta)
#             term is applied once per key, not per pair               = 22
ENG_FWD = 13
ENG_BWD_GRID = 19
ENG_BWD_MOVED = 22
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz: one FP32 lane-operation per lane
# per clock (packed FP32 is not used), 39.3 T lane-ops/s.
ROOFLINE_PEAK = 256 * 4 * 16 * 2.4e9


def alu_roofline(kernel, tile_avg_s, pairs, bwd_pairs, bwd_moved, traffic):
    """The tile kernel's roofline entry: algorithmic operations per launch
    over its event-timed average duration, against the FP32 lane peak."""
    ops = pairs * OPS_FWD + (bwd_pairs - bwd_moved) * OPS_BWD_GRID + bwd_moved * OPS_BWD_MOVED
    eng = pairs * ENG_FWD + (bwd_pairs - bwd_moved) * ENG_BWD_GRID + bwd_moved * ENG_BWD_MOVED
    return {
        "bound": "alu",
        "kernel": kernel,
        "achieved": ops / tile_avg_s / 1e12,
        "peak": ROOFLINE_PEAK / 1e12,
        "unit": "Tops/s",
        "frac": ops / tile_avg_s / ROOFLINE_PEAK,
        "traffic": traffic,
        "tile_kernel_ms": tile_avg_s * 1e3,
        "ops_per_pair": {"fwd": OPS_FWD, "bwd_grid": OPS_BWD_GRID, "bwd_moved": OPS_BWD_MOVED},
        "ops_per_launch": ops,
        "frac_engine_count": eng / tile_avg_s / ROOFLINE_PEAK,
        "engine_ops_per_pair": {"fwd": ENG_FWD, "bwd_grid": ENG_BWD_GRID, "bwd_moved": ENG_BWD_MOVED},
        "fwd_pairs_per_launch": pairs,
        "bwd_pairs_per_launch": bwd_pairs,
        "bwd_moved_pairs_per_launch": bwd_moved,
    }


def kernel_source_sha() -> str:
    src = os.path.join(ROOT, "paper_2505_21319_amd", "csrc", "efunc_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per tile-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source (its lines
    `kernel_source_sha: ...` and `hbm_bytes_per_launch: ...`)."""
    path = os.path.join(ROOT, "profiles", f"k_tile_fit_{workload}_pmc.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":", 1)[0].strip() in ("kernel_source_sha", "hbm_bytes_per_launch"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha") != kernel_source_sha():
        return None
    return int(float(fields["hbm_bytes_per_launch"]))


_ORACLE_CHILD = """
import sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle as orc
d = np.load(sys.argv[2])
th, q, o = d["theta"], d["q"], d["o"]
g = orc.Grid(R=th.shape[0])
n = th.size
t0 = time.perf_counter()
orc.fit_step(g, th, np.zeros(n), np.zeros(n), 1, q, o, mode=1, T=20.0)
print(time.perf_counter() - t0, orc.threads())
"""


def cpu_baseline(workload, q, o, R, theta, sample, sample_global=4096, reps=3):
    """The FP64 oracle's fit step timed on the host cores on a seeded
    subsample of the same batch (half uniform, half near-surface):
    * value: truncated mode (pairs within e^-20 of each query's largest
      weight, the result the engine reproduces) on `sample` points, all
      OpenMP threads, median of `reps`;
    * one_thread: the same on one thread (a child process with
      OMP_NUM_THREADS=1; it touches no GPU);
    * global_support: the paper's definition (every key for every point) on
      `sample_global` points, all threads."""
    import subprocess
    import tempfile
    import oracle as orc
    J = len(q)
    rng = np.random.default_rng(12345)
    h = sample // 2
    idx = np.concatenate([rng.choice(J // 2, h, replace=False),
                          J // 2 + rng.choice(J - J // 2, sample - h, replace=False)])
    qs, os_ = q[idx].astype(np.float64), o[idx].astype(np.float64)
    g = orc.Grid(R=R)
    n = theta.size
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        orc.fit_step(g, theta, np.zeros(n), np.zeros(n), 1, qs, os_, mode=1, T=20.0)
        ts.append(time.perf_counter() - t0)
    dt = float(np.median(ts))
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "sample.npz")
        np.savez(path, theta=theta, q=qs, o=os_)
        env = dict(os.environ, OMP_NUM_THREADS="1")
        res = subprocess.run([sys.executable, "-c", _ORACLE_CHILD, ROOT, path], env=env,
                             capture_output=True, text=True, check=True)
        dt1, thr1 = res.stdout.split()
        dt1 = float(dt1)
    hg = sample_global // 2
    gidx = np.concatenate([idx[:hg], idx[h:h + sample_global - hg]])
    t0 = time.perf_counter()
    orc.fit_step(g, theta, np.zeros(n), np.zeros(n), 1, q[gidx].astype(np.float64),
                 o[gidx].astype(np.float64), mode=0)
    dtg = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "points*iters/s", "cores": orc.threads(), "kind": "oracle",
            "sample": f"{sample} seeded points of iteration 0 ({h} uniform + {sample - h} near-surface), "
                      f"one FP64 fit step in truncated mode (e^-20, the result the engine reproduces), "
                      f"{orc.threads()} threads, median of {reps}: {dt:.2f} s",
            "one_thread": {"value": sample / dt1, "cores": int(thr1), "seconds": dt1},
            "global_support": {"value": sample_global / dtg, "cores": orc.threads(), "seconds": dtg,
                               "sample": f"{sample_global} of the same points, every one of the "
                                         f"{2 * R ** 3} keys per point (the paper's definition)"}}


def naive_efunc(theta, q):
    """Materialising autodiff baseline (plain PyTorch, float32): the global
    softmax over all keys with every key-query term held in memory, so that
    autograd can differentiate it (the construction the paper's fused kernels
    replace)."""
    import torch
    R = theta.shape[0]
    t = torch.linspace(-1, 1, R, device=q.device, dtype=torch.float64).to(torch.float32)
    K = torch.stack(torch.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    P = theta.reshape(-1, 13)
    centres = torch.cat([K, K + P[:, 5:8]])
    betas = torch.cat([P[:, 4].exp(), P[:, 12].exp()])
    vals = torch.cat([P[:, 0], P[:, 8]])
    slopes = torch.cat([P[:, 1:4], P[:, 9:12]])
    X = q[:, None, :] - centres[None]
    logits = -betas[None] * (X * X).sum(-1)
    F = vals[None] + (X * slopes[None]).sum(-1)
    return (torch.softmax(logits, dim=1) * F).sum(1)


def compare_autodiff(args):
    """Fused engine vs the materialising baseline at the paper's time/memory
    table shapes (16,384 queries, lattices 4^3 .. 64^3) and at the benchmark
    workload (2^21 queries, 32^3; the baseline chunked over queries)."""
    import torch
    import workloads as W
    from paper_2505_21319_amd import efunc as E
    dev = torch.device("cuda:0")
    w = W.get("csg16_r32")
    surf = torch.from_numpy(W.surface_points(w, 16384, seed=7, device=dev).astype(np.float32)).to(dev)

    def timed(fn, reps=10):
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    rows = []
    J = 16384
    q, o = W.make_batch(w, 0, J=J, device=dev)
    q, o = torch.from_numpy(q).to(dev), torch.from_numpy(o).to(dev)
    for R in (4, 8, 16, 32, 64):
        eng = E.Engine(R, J)
        th = torch.empty(R, R, R, 13, device=dev)
        eng.init_params(th, surf)
        g = torch.Generator(device="cpu").manual_seed(R)
        th[..., 0] += 0.1 * torch.randn(R, R, R, generator=g).to(dev)
        O = torch.empty(J, device=dev)
        lse = torch.empty(J, device=dev)
        dl = (2.0 / J) * torch.randn(J, generator=g).to(dev)
        G = torch.zeros_like(th)
        for _ in range(3):
            E.efunc_eval(eng.ctx, th, q, O, lse)
            E.efunc_grad(eng.ctx, th, q, O, lse, dl, G)
        fwd = timed(lambda: E.efunc_eval(eng.ctx, th, q, O, lse))
        bwd = timed(lambda: E.efunc_grad(eng.ctx, th, q, O, lse, dl, G))
        ws = eng.stats()["workspace_bytes"] + 2 * 4 * J
        eng.close()
        row = {"R": R, "keys": 2 * R ** 3, "J": J, "fused_fwd_ms": fwd, "fused_bwd_ms": bwd,
               "fused_extra_MB": ws / 2 ** 20}
        torch.cuda.empty_cache()
        try:
            T = th.clone().requires_grad_(True)
            base = torch.cuda.memory_allocated()
            torch.cuda.reset_peak_memory_stats()
            out = {}

            def f():
                out["O"] = naive_efunc(T, q)

            def b():
                T.grad = None
                naive_efunc(T, q).backward(dl)

            f()
            torch.cuda.synchronize()
            row["naive_fwd_ms"] = timed(f, 5)
            row["naive_bwd_ms"] = max(timed(b, 5) - row["naive_fwd_ms"], 0.0)
            row["naive_peak_GB"] = (torch.cuda.max_memory_allocated() - base) / 2 ** 30
            del out
        except torch.cuda.OutOfMemoryError:
            row["naive"] = "OOM"
        torch.cuda.empty_cache()
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    # the benchmark workload: fused fit step vs the baseline chunked over queries
    Jb = w.J
    qb, ob = W.make_batch(w, 0, device=dev)
    qb, ob = torch.from_numpy(qb).to(dev), torch.from_numpy(ob).to(dev)
    eng = E.Engine(w.R, Jb)
    th = torch.empty(w.R, w.R, w.R, 13, device=dev)
    eng.init_params(th, surf)
    m, v = torch.zeros_like(th), torch.zeros_like(th)
    for s_ in range(1, 4):
        eng.fit_step(th, m, v, s_, qb, ob)
    fit_ms = timed(lambda: eng.fit_step(th, m, v, 4, qb, ob), 10)
    eng.close()
    chunk, nchunks = 4096, 16
    T = th.clone().requires_grad_(True)

    def chunks():
        T.grad = None
        for c in range(nchunks):
            sl = slice(c * chunk, (c + 1) * chunk)
            r = naive_efunc(T, qb[sl]) - ob[sl]
            (r * r).sum().div(Jb).backward()

    chunks()
    torch.cuda.synchronize()
    naive_ms = timed(chunks, 3) * (Jb / (chunk * nchunks))
    cfg2 = {"workload": "csg16_r32", "J": Jb, "fused_fit_step_ms": fit_ms,
            "naive_fwd_bwd_ms_extrapolated": naive_ms,
            "naive_note": f"chunks of {chunk} queries; {nchunks} chunks timed and scaled to {Jb} "
                          "queries; no optimiser step"}
    print(json.dumps({"comparison": "fused engine vs materialising autodiff (global softmax)",
                      "table_shapes": rows, "benchmark_workload": cfg2}))


def bench_batch(args, torch):
    """Batched multi-shape fitting: 64 independent shapes (lattices 16^3 to
    64^3, 2^18 to 2^22 points per iteration, both log-uniform), one resident
    minibatch per shape, all shapes stepped together per iteration through
    one captured HIP graph."""
    import workloads as W
    from paper_2505_21319_amd import efunc as E

    dev = torch.device("cuda:0")
    ws = W.batch_set("batch64", 64, 300)
    t_gen = time.perf_counter()
    thetas, qs, os_ = [], [], []
    for i, w in enumerate(ws):
        q, o = W.make_batch(w, 0, device=dev)
        qs.append(torch.from_numpy(q).to(dev))
        os_.append(torch.from_numpy(o).to(dev))
        surf = W.surface_points(w, 16384, seed=W.seed_for(w, -2, "meanshift"), device=dev)
        th = torch.empty(w.R ** 3 * 13, device=dev, dtype=torch.float32)
        with E.Engine(w.R, 16) as e1:
            e1.init_params(th, torch.from_numpy(surf.astype(np.float32)).to(dev), 100.0, 7.0)
        thetas.append(th)
        if (i + 1) % 16 == 0:
            print(f"# generated {i + 1}/{len(ws)} shapes", file=sys.stderr, flush=True)
    t_gen = time.perf_counter() - t_gen
    ms_ = [torch.zeros_like(t) for t in thetas]
    vs_ = [torch.zeros_like(t) for t in thetas]
    loss = torch.zeros(len(ws), 2, device=dev, dtype=torch.float64)
    Jtot = sum(w.J for w in ws)

    B = E.BatchEngine([w.R for w in ws], [w.J for w in ws])
    B.bind(thetas, ms_, vs_, qs, os_, loss)
    tuned = None
    if args.tuning:
        B.set_tuning(*[int(x) for x in args.tuning.split(",")])
    if args.autotune:
        tuned = B.autotune(reps=2)
    step = 1
    B.fit(step, args.warmup, use_graph=True)
    step += args.warmup
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    B.fit(step, args.steps, use_graph=True)
    step += args.steps
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)

    # tile-kernel duration from directly launched iterations (events on the
    # stream the kernel runs on)
    n_eager = max(1, min(args.steps, 5))
    E.efunc_batch_set_timing(B.b, True)
    B.fit(step, n_eager, use_graph=False)
    tile_ms, launches = E.efunc_batch_read_timing(B.b)
    E.efunc_batch_set_timing(B.b, False)
    sts = [B.stats(i) for i in range(len(ws))]
    lossv = loss.cpu().numpy()
    pairs = sum(st["pairs"] for st in sts)
    bp = sum(st["bwd_pairs"] for st in sts)
    bpm = sum(st["bwd_pairs_moved"] for st in sts)
    tile_avg_s = tile_ms / max(launches, 1) * 1e-3
    Rs = [w.R for w in ws]
    out = {
        "metric": "batched fit points·iters/sec (64 shapes, fused fwd+bwd)",
        "value": Jtot * args.steps / (total_ms * 1e-3),
        "unit": "points*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "batch64",
            "shapes": len(ws),
            "R_min": min(Rs), "R_max": max(Rs),
            "points_per_iter": Jtot,
            "J_min": min(w.J for w in ws), "J_max": max(w.J for w in ws),
            "params": sum(R ** 3 * 13 for R in Rs),
            "target": "per shape a smooth union (k=0.05) of 4..64 seeded spheres/boxes",
            "init": "rho=7, zero values, mean-shift offsets (16384 surface samples, bandwidth 100)",
            "graph": True,
            "tuning": B.tuning(),
            "autotuned_ms": tuned[1] if tuned else None,
        },
        "roofline": alu_roofline("k_tile_batch", tile_avg_s, pairs, bp, bpm, None),
        "stats": {"uncertified": sum(st["n_uncertified"] for st in sts),
                  "tiles": sum(st["n_tiles"] for st in sts),
                  "loss_mse_mean": float(lossv[:, 0].mean()), "gen_seconds": t_gen,
                  "kernel_source_sha": kernel_source_sha()},
    }
    if not args.no_cpu_baseline:
        w = ws[0]
        th0 = W.plain_theta(w.R)
        out["cpu_baseline"] = cpu_baseline(w, qs[0].cpu().numpy(), os_[0].cpu().numpy(), w.R, th0,
                                           args.cpu_sample)
    B.close()
    print(json.dumps(out))


def bench_initnet(args, torch):
    """Learned initialiser: the matrix-core throughput of the network
    (forward + backward over a batch of 8 shapes on the 32^3 lattice) and
    the fitting experiment (train on synthetic shapes, fit held-out shapes
    from three initialisations)."""
    import workloads as W
    from paper_2505_21319_amd import efunc as E
    from paper_2505_21319_amd import initnet_train as T

    dev = torch.device("cuda:0")
    R = 32
    log = lambda m: print("# " + m, file=sys.stderr, flush=True)  # noqa: E731
    n_train, n_test = args.initnet_train, args.initnet_test
    if args.initnet_conv_only:
        n_train, n_test = 8, 0
    ws = W.batch_set("initnet", n_train + n_test, 400, R_range=(R, R), J_range=(1 << 16, 1 << 16),
                     prims_range=(8, 24))
    t_gen = time.perf_counter()
    data = []
    for i, w in enumerate(ws):
        q, o = W.make_batch(w, 0, device=dev)
        sdf = T.coarse_sdf(lambda g, w=w: W.target(w, g), R, dev)
        data.append((sdf, torch.from_numpy(q).to(dev), torch.from_numpy(o).to(dev), w))
        if (i + 1) % 64 == 0:
            log(f"generated {i + 1}/{len(ws)} shapes")
    train_set = []
    for sdf, q, o, w in data[:n_train]:
        qsets, osets = [q], [o]
        for k in range(1, args.initnet_train_sets):
            qk, ok_ = W.make_batch(w, k, device=dev)
            qsets.append(torch.from_numpy(qk).to(dev))
            osets.append(torch.from_numpy(ok_).to(dev))
        train_set.append((sdf, qsets, osets))
    t_gen = time.perf_counter() - t_gen
    test = data[n_train:]

    net = E.InitNet(R, 8, T.CHANNELS)
    params = torch.from_numpy(T.initial_params(1)).to(dev)
    # matrix-core throughput: forward + backward of 8 shapes, HIP events on the stream
    sdf8 = torch.stack([d[0] for d in data[:8]])
    dout = torch.randn(8, R ** 3, T.CHANNELS[-1], device=dev)
    g = torch.zeros_like(params)
    for _ in range(3):
        net.forward(params, sdf8)
        net.backward(dout, g)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    reps = 20
    torch.cuda.synchronize()
    ev[0].record(stream)
    for _ in range(reps):
        net.forward(params, sdf8)
    ev[1].record(stream)
    for _ in range(reps):
        net.backward(dout, g)
    ev[2].record(stream)
    torch.cuda.synchronize()
    fwd_ms = ev[0].elapsed_time(ev[1]) / reps
    bwd_ms = ev[1].elapsed_time(ev[2]) / reps
    conv_flop = sum(2 * 8 * R ** 3 * 27 * ci * co for ci, co in zip(T.CHANNELS[:-1], T.CHANNELS[1:]))
    # backward: weight gradient for every layer, data gradient for all but the first
    bwd_flop = conv_flop + sum(2 * 8 * R ** 3 * 27 * ci * co
                               for ci, co in list(zip(T.CHANNELS[:-1], T.CHANNELS[1:]))[1:])

    conv_res = {"metric": "learned-initialiser network fwd+bwd throughput (bf16 MFMA conv3d)",
                "value": (conv_flop + bwd_flop) / ((fwd_ms + bwd_ms) * 1e-3) / 1e12, "unit": "TFLOP/s",
                "fwd_ms": fwd_ms, "bwd_ms": bwd_ms}
    if args.initnet_conv_only:
        net.close()
        print(json.dumps(conv_res))
        return
    # train end to end, then fit held-out shapes from each initialisation
    t_train = time.perf_counter()
    params = torch.from_numpy(T.initial_params(1)).to(dev)
    losses = T.train(net, params, train_set, args.initnet_steps, 8, 1e-3, 2, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train
    inits = {"paper": [], "sdf": [], "newton": [], "learned": []}
    t_init = {"paper": 0.0, "sdf": 0.0, "newton": 0.0, "learned": 0.0}
    for sdf, q, o, w in test:
        surf = torch.from_numpy(W.surface_points(w, 16384, seed=W.seed_for(w, -2, "meanshift"),
                                                 device=dev).astype(np.float32)).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inits["paper"].append(T.paper_theta(R, surf, dev))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        inits["sdf"].append(T.sdf_theta(R, sdf, surf, dev))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        inits["newton"].append(T.newton_theta(sdf, R).reshape(-1).contiguous())
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        inits["learned"].append(T.learned_theta(net, params, sdf))
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        t_init["paper"] += t1 - t0
        t_init["sdf"] += t2 - t1
        t_init["newton"] += t3 - t2
        t_init["learned"] += t4 - t3
    # learned with the paper's initialisation as fallback, the fitting loss on
    # the shape's own training points deciding
    chosen = [T.choose_init(R, lt, pt, d[1], d[2]) for lt, pt, d in zip(inits["learned"], inits["paper"], test)]
    n_fallback = sum(fb for _, fb in chosen)
    if n_fallback:
        inits["learned_or_paper"] = [c for c, _ in chosen]
        t_init["learned_or_paper"] = t_init["learned"] + t_init["paper"]
    log(f"learned init kept for {len(test) - n_fallback}/{len(test)} shapes")
    # held-out scoring points: a seed of their own, half uniform, half near the surface
    heldout = []
    for i, (_, _, _, w) in enumerate(test):
        qh, oh = W.make_batch(w, 10 ** 6, J=args.initnet_heldout, device=dev)
        heldout.append((torch.from_numpy(qh).to(dev), torch.from_numpy(oh).to(dev)))
        if (i + 1) % 16 == 0:
            log(f"held-out points for {i + 1}/{len(test)} shapes")
    # training points of the fits: P point sets per held-out shape, cycled
    P = args.initnet_point_sets
    Jt = int(test[0][1].shape[0])
    qpool = torch.empty(P, len(test), Jt, 3, device=dev)
    opool = torch.empty(P, len(test), Jt, device=dev)
    for i, (_, q, o, w) in enumerate(test):
        qpool[0, i], opool[0, i] = q, o
        for k in range(1, P):
            qk, ok_ = W.make_batch(w, k, device=dev)
            qpool[k, i], opool[k, i] = torch.from_numpy(qk).to(dev), torch.from_numpy(ok_).to(dev)
    log(f"fit point pool: {P} sets x {len(test)} shapes x {Jt} points")
    thr = 1e-3
    results = {}
    marks = sorted({0, 10, 20, 50, 100, 250, 500, 1000, 2000, args.initnet_fit_steps})
    for name, ths in inits.items():
        curve, secs = T.fit_curves([R] * len(test), ths, qpool, opool, args.initnet_fit_steps, heldout, log=log)
        reach = T.steps_to(curve, thr)
        ok = [s for s in reach if s is not None]
        per_step = secs / args.initnet_fit_steps
        init_total = t_init[name]
        res = {
            "heldout_l1": {str(st): float(np.mean(a)) for st, a, *_ in curve if st in marks},
            "heldout_volume_l1": {str(st): float(np.mean(b)) for st, _, b, *_ in curve if st in marks},
            "heldout_near_l1": {str(st): float(np.mean(c)) for st, _, _, c, _ in curve if st in marks},
            "step_points_l1": {str(st): float(np.mean(t)) for st, *_, t in curve if st in marks and st > 0},
            "reached": len(ok),
            "median_steps_to_thr": float(np.median(ok)) if ok else None,
            "fit_seconds": secs,
            "seconds_per_batched_step": per_step,
            "init_seconds_total": init_total,
        }
        # wall time of the whole batch: initialisation + batched steps until the
        # half / all of the shapes reached the threshold
        srt = sorted(ok)
        half = (len(test) + 1) // 2
        res["wall_seconds_half_reached"] = init_total + srt[half - 1] * per_step if len(srt) >= half else None
        res["wall_seconds_all_reached"] = init_total + srt[-1] * per_step if len(srt) == len(test) else None
        results[name] = res
        log(f"{name}: {res}")
    net.close()
    out = {
        "metric": "learned-initialiser network fwd+bwd throughput (bf16 MFMA conv3d)",
        "value": (conv_flop + bwd_flop) / ((fwd_ms + bwd_ms) * 1e-3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": reps, "warmup": 3, "ms_per_step": fwd_ms + bwd_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16 x bf16 -> f32",
        "data": "synthetic",
        "config": {"workload": "initnet", "R": R, "channels": T.CHANNELS, "batch": 8,
                   "train_shapes": n_train, "test_shapes": n_test, "train_steps": args.initnet_steps,
                   "fit_steps": args.initnet_fit_steps, "points_per_shape": 1 << 16},
        "roofline": {"bound": "mfma", "achieved": (conv_flop + bwd_flop) / ((fwd_ms + bwd_ms) * 1e-3) / 1e12,
                     "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": (conv_flop + bwd_flop) / ((fwd_ms + bwd_ms) * 1e-3) / 2.5e15, "traffic": None,
                     "fwd_ms": fwd_ms, "bwd_ms": bwd_ms, "fwd_flop": conv_flop, "bwd_flop": bwd_flop},
        "experiment": {"train_loss": losses, "train_seconds": t_train, "gen_seconds": t_gen,
                       "l1_threshold": thr, "heldout_points_per_shape": args.initnet_heldout,
                       "fit_point_sets": P, "train_point_sets": args.initnet_train_sets,
                       "learned_kept": len(test) - n_fallback, "inits": results},
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="csg16_r32")
    ap.add_argument("--batches", type=int, default=4, help="distinct resident batches cycled")
    ap.add_argument("--cpu-sample", type=int, default=1 << 16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--deterministic", action="store_true",
                    help="run the fit step in the library's deterministic mode")
    ap.add_argument("--compare-autodiff", action="store_true",
                    help="print the fused vs materialising-autodiff comparison instead")
    ap.add_argument("--autotune", action="store_true",
                    help="batch64: run the autotuner before timing")
    ap.add_argument("--tuning", default="",
                    help="tile_cap,group_cells,blocks_per_cu for the tile kernel (default 512,2,8)")
    ap.add_argument("--initnet-train", type=int, default=256, help="initnet: training shapes")
    ap.add_argument("--initnet-test", type=int, default=64, help="initnet: held-out shapes")
    ap.add_argument("--initnet-steps", type=int, default=3000, help="initnet: network training steps")
    ap.add_argument("--initnet-train-sets", type=int, default=4, help="initnet: point sets per training shape")
    ap.add_argument("--initnet-fit-steps", type=int, default=2000, help="initnet: fit steps per init")
    ap.add_argument("--initnet-heldout", type=int, default=1 << 20, help="initnet: held-out scoring points per shape")
    ap.add_argument("--initnet-point-sets", type=int, default=8, help="initnet: point sets cycled by the fits")
    ap.add_argument("--initnet-conv-only", action="store_true",
                    help="initnet: time the network's forward and backward only")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark measures one GPU only: the fused fit step "
                                   "runs on a single device; run with --gpus 1"}))
        sys.exit(2)

    import torch
    if args.compare_autodiff:
        compare_autodiff(args)
        return
    if args.copy_calib_mib:
        n = args.copy_calib_mib * (1 << 20) // 4
        a = torch.ones(n, device="cuda", dtype=torch.float32)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))
        return

    if args.workload == "batch64":
        bench_batch(args, torch)
        return
    if args.workload == "initnet":
        bench_initnet(args, torch)
        return

    import workloads as W
    from paper_2505_21319_amd import efunc as E

    dev = torch.device("cuda:0")
    w = W.get(args.workload)
    R, J = w.R, w.J
    t_gen = time.perf_counter()
    batches = []
    for it in range(args.batches):
        q, o = W.make_batch(w, it, device=dev)
        batches.append((torch.from_numpy(q).to(dev), torch.from_numpy(o).to(dev)))
    surf = W.surface_points(w, 16384, seed=W.seed_for(w, -2, "meanshift"), device=dev)
    t_gen = time.perf_counter() - t_gen

    eng = E.Engine(R, J, deterministic=1 if args.deterministic else 0)
    if args.tuning:
        eng.set_tuning(*[int(x) for x in args.tuning.split(",")])
    theta = torch.empty(R, R, R, 13, device=dev, dtype=torch.float32)
    eng.init_params(theta, torch.from_numpy(surf.astype(np.float32)).to(dev), 100.0, 7.0)
    theta0 = theta.cpu().numpy()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    loss = torch.zeros(2, device=dev, dtype=torch.float64)

    step = 0
    for _ in range(args.warmup):
        step += 1
        q, o = batches[step % len(batches)]
        eng.fit_step(theta, m, v, step, q, o, loss)
    torch.cuda.synchronize()

    E.efunc_set_timing(eng.ctx, True)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step += 1
        q, o = batches[step % len(batches)]
        eng.fit_step(theta, m, v, step, q, o, loss)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    tile_ms, launches = E.efunc_read_timing(eng.ctx)
    st = eng.stats()
    lossv = loss.cpu().numpy()
    E.efunc_set_timing(eng.ctx, False)

    ms_step = total_ms / args.steps
    value = J * args.steps / (total_ms * 1e-3)
    tile_avg_s = tile_ms / max(launches, 1) * 1e-3
    pairs, pm = st["pairs"], st["pairs_moved"]
    bp, bpm = st["bwd_pairs"], st["bwd_pairs_moved"]
    traffic = measured_traffic(args.workload)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "R": R,
            "params": R ** 3 * 13,
            "points_per_iter": J,
            "target": (f"smooth union (k=0.05) of {w.n_prims} seeded spheres/boxes"
                       if w.shape == "csg" else "sphere r=0.5"),
            "mix": "50% uniform in [-1,1]^3, 50% surface + N(0, 0.01^2)",
            "init": "rho=7, zero values, mean-shift offsets (16384 surface samples, bandwidth 100)",
            "t_cut": 20.0,
            "resident_batches": args.batches,
            "tuning": eng.tuning(),
            "deterministic": bool(args.deterministic),
        },
        "roofline": dict(alu_roofline("k_tile<FIT>", tile_avg_s, pairs, bp, bpm, traffic),
                         fwd_moved_pairs_per_launch=pm),
        "stats": {"W": st["W"], "tiles": st["n_tiles"], "uncertified": st["n_uncertified"],
                  "queries_per_tile": J / max(st["n_tiles"], 1),
                  "window_keys_per_tile": st["window_keys"] / max(st["n_tiles"], 1),
                  "kept_keys_per_tile": st["kept_keys"] / max(st["n_tiles"], 1),
                  "beta_min": st["beta_min"], "loss_mse": float(lossv[0]), "loss_l1": float(lossv[1]),
                  "gen_seconds": t_gen, "kernel_source_sha": kernel_source_sha()},
    }
    if not args.no_cpu_baseline:
        q0, o0 = (x.cpu().numpy() for x in batches[0])
        out["cpu_baseline"] = cpu_baseline(w, q0, o0, R, theta0, args.cpu_sample)
    eng.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
