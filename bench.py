#!/usr/bin/env python3
"""Joined tuples per second of the relational layer on one MI355X.

Workload (the heterogeneous ER schema, hidden 128, two layers, FP32):
User 1M, Item 500k, Category 1k rows with N(0,1) embeddings of width 128;
Buys(user, item) 20M rows, item ~ Zipf(1.1), user uniform; BelongsTo gives
each item a uniform category.  Per layer two join rules run:

  Item'(i; sum(Lin_I(z_u (+) z_i (+) z_c)))  :- Buys(u,i), BelongsTo(i,c), ...   K = 384
  User'(u; mean(Lin_U(z_u (+) z_i)))          :- Buys(u,i), ...                   K = 256

with ReLU after each aggregate; layer 2 reads layer 1's outputs.  A step is
the four layer evaluations (80M joined tuples).  Inputs and indices are
resident in HBM before timing; the index build is timed separately.

Prints ONE JSON line.  ``value`` is the fused FP32 path; the same line
carries the FP32 plain (unfused) path and the fused BF16 path, the
roofline of the dominant kernel, and the FP64 oracle timed on host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "joined tuples/sec per layer (fwd, fwd+bwd) vs FP32 plain; serve p50/p99 ms"
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0}     # MI355X dense matrix peaks
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_workload(scale: float):
    import torch

    import relgen
    from paper_2605_24207_amd import Index

    t0 = time.perf_counter()
    n_user, n_item, n_buys = int(1_000_000 * scale), int(500_000 * scale), int(20_000_000 * scale)
    g = relgen.er_graph(n_user=n_user, n_item=n_item, n_buys=n_buys)
    log(f"generated ER graph in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    D = {"g": g, "U": t(g.user), "I": t(g.item), "C": t(g.cat), "bu": t(g.buys_u), "bi": t(g.buys_i),
         "bc": t(g.belongs_cat)}
    D["W_item"] = [t(w) for w in g.W_item]
    D["W_user"] = [t(w) for w in g.W_user]
    D["b_item"] = [t(b) for b in g.b_item]
    D["b_user"] = [t(b) for b in g.b_user]
    nu, ni, nc = g.user.shape[0], g.item.shape[0], g.cat.shape[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    D["ix_item1"] = Index([D["bu"], D["bi"]], [(nu, 0, None), (ni, 1, None), (nc, 2, None)], 1,
                          chains=[(1, D["bc"], None)])
    D["ix_user1"] = Index([D["bu"], D["bi"]], [(nu, 0, None), (ni, 1, None)], 0)
    ki = D["ix_item1"].export()["group_keys"]
    ku = D["ix_user1"].export()["group_keys"]
    Gi, Gu = D["ix_item1"].G, D["ix_user1"].G
    D["ix_item2"] = Index([D["bu"], D["bi"]], [(Gu, 0, ku), (Gi, 1, ki), (nc, 2, None)], 1,
                          chains=[(1, D["bc"], None)])
    D["ix_user2"] = Index([D["bu"], D["bi"]], [(Gu, 0, ku), (Gi, 1, ki)], 0)
    torch.cuda.synchronize()
    D["index_build_s"] = time.perf_counter() - t0
    D["keys"] = (ki, ku)
    log(f"built 4 indices in {D['index_build_s']:.2f}s: E_item={D['ix_item1'].E} G_item={Gi} "
        f"E_user={D['ix_user1'].E} G_user={Gu}")
    return D


class Net:
    """The two-layer ER network in one precision / path."""

    def __init__(self, D, dtype: str, plain: bool, pushdown: bool = False):
        import torch

        from paper_2605_24207_amd import Layer, workspace_size

        self.D = D
        tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
        self.dtype = dtype
        cv = lambda x: x.to(tdt).contiguous()
        self.U, self.I, self.C = cv(D["U"]), cv(D["I"]), cv(D["C"])
        self.W_item = [cv(w) for w in D["W_item"]]
        self.W_user = [cv(w) for w in D["W_user"]]
        od = "bf16" if dtype == "bf16" else "f32"
        self.L_item = Layer([128, 128, 128], 128, dtype, "sum", "none", "relu", plain=plain, out_dtype=od,
                            pushdown=pushdown)
        self.L_user = Layer([128, 128], 128, dtype, "mean", "none", "relu", plain=plain, out_dtype=od,
                            pushdown=pushdown)
        ix = [D["ix_item1"], D["ix_user1"], D["ix_item2"], D["ix_user2"]]
        ws = max(workspace_size(ix[q], [self.L_item, self.L_user][q % 2]) for q in range(4))
        self.ws = torch.empty(ws, dtype=torch.uint8, device="cuda")
        Gi, Gu = D["ix_item1"].G, D["ix_user1"].G
        self.out = [torch.empty(G, 128, dtype=tdt, device="cuda") for G in (Gi, Gu, Gi, Gu)]
        self.tuples = sum(x.E for x in ix)
        # algorithmic flops of one step: per tuple 2 K h (Linear) + h (bias) + h (aggregate)
        self.flops = sum(x.E * (2 * K * 128 + 2 * 128) for x, K in zip(ix, (384, 256, 384, 256)))
        self.bytes = step_bytes(ix, (384, 256, 384, 256), (3, 2, 3, 2), 128, 2 if dtype == "bf16" else 4)

    def step(self):
        from paper_2605_24207_amd import layer_fwd

        D, o = self.D, self.out
        layer_fwd(D["ix_item1"], self.L_item, [self.U, self.I, self.C], self.W_item[0], D["b_item"][0],
                  want_pre=False, ws=self.ws, out=o[0])
        layer_fwd(D["ix_user1"], self.L_user, [self.U, self.I], self.W_user[0], D["b_user"][0],
                  want_pre=False, ws=self.ws, out=o[1])
        layer_fwd(D["ix_item2"], self.L_item, [o[1], o[0], self.C], self.W_item[1], D["b_item"][1],
                  want_pre=False, ws=self.ws, out=o[2])
        layer_fwd(D["ix_user2"], self.L_user, [o[1], o[0]], self.W_user[1], D["b_user"][1],
                  want_pre=False, ws=self.ws, out=o[3])


def step_bytes(ix, Ks, ks, h, esz):
    """Algorithmic HBM bytes of one step, per kernel kind, summed over the
    step's layers (E tuples, G groups, K = Concat width, k atoms):
      fused   every joined row read once (E K esz), the k row numbers and the
              group number per tuple (4 (k + 1) E), out written (G h esz_out)
      gather  joined rows read and X written (2 E K esz) + row numbers (4 k E)
      gemm    X read (E K esz), Y written (4 E h), W (K h esz)
      reduce  Y and group numbers read (4 E (h + 1)), out written (4 G h),
              offsets (4 G)"""
    b = {"fused": 0, "gather": 0, "gemm": 0, "reduce": 0}
    for x, K, k in zip(ix, Ks, ks):
        E, G = x.E, x.G
        b["fused"] += E * K * esz + 4 * (k + 1) * E + G * h * esz
        b["gather"] += 2 * E * K * esz + 4 * k * E
        b["gemm"] += E * K * esz + 4 * E * h + K * h * esz
        b["reduce"] += 4 * E * (h + 1) + 4 * G * h + 4 * G
    return b


def measured_value(summary: str, sources, key: str):
    """A machine-readable figure of a committed profile summary, or None when
    a kernel source it was taken on has changed since (sha256 prefix of the
    sources' concatenated bytes)."""
    import hashlib
    import re

    try:
        text = open(os.path.join(ROOT, "profiles", summary)).read()
        h = hashlib.sha256()
        for src in sources:
            h.update(open(os.path.join(ROOT, "paper_2605_24207_amd", "csrc", src), "rb").read())
        want = re.search(r"source_sha256_prefix:\s*([0-9a-f]+)", text).group(1)
        val = float(re.search(key + r":\s*([0-9.e+]+)", text).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    return val if h.hexdigest()[:16] == want else None


def measured_traffic():
    """HBM bytes per launch of the fused FP32 forward from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated)."""
    return measured_value("fused_fwd_er_counters.md", ["layer_ws.hip"], "traffic_bytes_per_launch_fused_f32")


def gbs(nbytes_per_step, steps, kt):
    """Achieved GB/s of a kernel: its algorithmic bytes over its summed
    launch time (HIP events on the launch stream)."""
    ms = kt[0]
    return nbytes_per_step * steps / (ms * 1e-3) / 1e9 if ms > 0 else None


def time_net(net: Net, steps: int, warmup: int, kernels):
    import torch

    from paper_2605_24207_amd import api

    for _ in range(warmup):
        net.step()
    torch.cuda.synchronize()
    api.timing_reset()
    api.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        net.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    api.timing_enable(False)
    ktime = {k: api.timing_read(k) for k in kernels}
    api.timing_reset()
    return dt, ktime


def fwd_bwd_leg(steps: int, warmup: int, scale: float, dtype: str = "f32", pushdown: bool = False):
    """Differentiation form: Node [2M, 128], Edge 10M with s ~ Zipf(1.2), t
    uniform; layer 1 SUM + ReLU, layer 2 MAX, MSE against N(0,1) targets.  A
    step is forward and backward of both layers through RelLayerFn (20M
    joined tuples, each through fwd + bwd).  BF16: embeddings, weights and
    the layer-1 output in bf16, FP32 accumulation and FP32 gradients inside
    the library.  pushdown: both (affine) layers evaluate the transform once
    per node in the forward; the backward is the same."""
    import torch

    import relgen
    from paper_2605_24207_amd import Index, Layer, RelLayerFn, api

    p = relgen.power_graph(n_nodes=int(2_000_000 * scale), n_edges=int(10_000_000 * scale))
    dev = "cuda"
    s = torch.from_numpy(p.s).to(dev)
    t = torch.from_numpy(p.t).to(dev)
    n = p.z.shape[0]
    ix1 = Index([s, t], [(n, 0, None), (n, 1, None)], 1, bwd=True)
    k1 = ix1.export()["group_keys"]
    ix2 = Index([s, t], [(ix1.G, 0, k1), (ix1.G, 1, k1)], 1, bwd=True)
    L1 = Layer([128, 128], 128, dtype, "sum", "none", "relu", out_dtype=dtype, pushdown=pushdown)
    L2 = Layer([128, 128], 128, dtype, "max", "none", "none", pushdown=pushdown)
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
    z = torch.from_numpy(p.z).to(dev).to(tdt).requires_grad_(True)
    W1 = torch.from_numpy(p.W[0]).to(dev).to(tdt).requires_grad_(True)
    W2 = torch.from_numpy(p.W[1]).to(dev).to(tdt).requires_grad_(True)
    b1 = torch.from_numpy(p.b[0]).to(dev).requires_grad_(True)
    b2 = torch.from_numpy(p.b[1]).to(dev).requires_grad_(True)
    target = torch.from_numpy(p.target).to(dev)[ix2.export()["group_keys"].long()].contiguous()

    def step():
        for x in (z, W1, W2, b1, b2):
            x.grad = None
        h1 = RelLayerFn.apply(ix1, L1, W1, b1, z, z)
        h2 = RelLayerFn.apply(ix2, L2, W2, b2, h1, h1)
        torch.nn.functional.mse_loss(h2, target).backward()   # mean((h2 - target)^2), fused

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    api.timing_reset()
    api.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    api.timing_enable(False)
    kt = {k: api.timing_read(k) for k in ("fwd_fused", "fwd_push", "bwd_dw", "bwd_dx")}
    api.timing_reset()
    tuples = ix1.E + ix2.E
    return {"value": tuples * steps / dt, "unit": "tuples/s (fwd+bwd, per layer)", "ms_per_step": dt / steps * 1e3,
            "workload": "Node 2M x 128, Edge 10M (s ~ Zipf 1.2, t uniform); L1 SUM+ReLU, L2 MAX; MSE; "
                        + ("BF16" if dtype == "bf16" else "FP32") + ("; forward with pushdown" if pushdown else ""),
            "tuples_per_step": tuples, "steps": steps,
            "kernels_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in kt.items() if v[1]}}


def cobuy_leg(D, steps: int, warmup: int):
    """Precision form: CoBuy(u1; max(Lin(z_u1 (+) z_u2))) over the self-join
    of Buys on item, at most 50 paths per item (about 9.8M paths), User
    embeddings of width 256, h = 256, BF16 operands with FP32 accumulation.
    A step is one layer evaluation over all paths."""
    import torch

    import relgen
    from paper_2605_24207_amd import Index, Layer, api, layer_fwd, workspace_size

    rule = relgen.cobuy_rule(D["g"], d=256, h=256, cap=50, agg="max")
    nu = rule.atoms[0].n_rows
    t0 = time.perf_counter()
    ix = Index([D["bu"], D["bi"]], [(nu, 0, None), (nu, 2, None)], 0, two_hop=(1, 50))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    U = torch.from_numpy(rule.atoms[0].emb).to("cuda").to(torch.bfloat16).contiguous()
    W = torch.from_numpy(rule.W).to("cuda").to(torch.bfloat16).contiguous()
    b = torch.from_numpy(rule.b).to("cuda")
    L = Layer([256, 256], 256, "bf16", "max", "none", "none")
    ws = torch.empty(workspace_size(ix, L), dtype=torch.uint8, device="cuda")
    out = torch.empty(ix.G, 256, dtype=torch.float32, device="cuda")

    def step():
        layer_fwd(ix, L, [U, U], W, b, want_pre=False, want_argmax=False, ws=ws, out=out)

    D["cobuy_out"] = (out, ix.export()["group_keys"])

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    api.timing_reset()
    api.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    api.timing_enable(False)
    k_ms, k_n = api.timing_read("fwd_fused")
    api.timing_reset()
    flops = ix.E * (2 * 512 * 256 + 2 * 256)
    k_avg = k_ms / max(k_n, 1)
    return {"value": ix.E * steps / dt, "unit": "tuples/s", "ms_per_step": dt / steps * 1e3,
            "workload": "CoBuy(u1; max(Lin(z_u1 (+) z_u2))) :- Buys(u1,i), Buys(u2,i); <= 50 paths per item; "
                        "User 1M x 256; h 256; BF16 in, FP32 accumulate",
            "tuples_per_step": ix.E, "groups": ix.G, "steps": steps, "index_build_s": round(build_s, 3),
            "kernel_ms_per_launch": k_avg,
            "mfma_tflops": flops / (k_avg * 1e-3) / 1e12 if k_avg > 0 else None,
            "mfma_peak_tflops": PEAK_TFLOPS["bf16"]}


def serve_leg(D, dtype: str, rates, seconds: float):
    """Serving form: the resident ER graph, seed-item requests with sizes
    log-uniform over 1..4096, two hops with fanout 15 then 10, open-loop
    Poisson arrivals at each rate for ``seconds``; HBM budget 64 GiB.
    Latency = done - arrival, from the library's steady-clock stamps."""
    import threading

    import torch

    import relgen
    from paper_2605_24207_amd import Server

    tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
    cv = lambda x: x.to(tdt).contiguous()
    srv = Server(D["bu"], D["bi"], D["bc"], cv(D["U"]), cv(D["I"]), cv(D["C"]), cv(D["W_user"][0]),
                 cv(D["W_item"][0]), cv(D["W_item"][1]), dtype=dtype, max_seeds=4096, max_slots=64,
                 budget_bytes=64 << 30)
    n_items = D["I"].shape[0]
    warm = relgen.request_stream(n_items, 8, 1000.0, seed=1)
    for r in warm:
        srv.wait(srv.submit(r.seeds, r.req_seed), len(r.seeds))
    res = []
    for rate in rates:
        reqs = relgen.request_stream(n_items, max(1, int(rate * seconds)), rate, seed=int(rate))
        tickets = [None] * len(reqs)
        t0 = time.perf_counter()

        def submitter():
            for q, r in enumerate(reqs):
                dt = r.t_arrive - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                tickets[q] = srv.submit(r.seeds, r.req_seed)

        th = threading.Thread(target=submitter)
        th.start()
        n_done, lat, tuples, first, last = 0, [], 0, None, None
        seen = 0                                # tickets [0, seen) have been handed to the poller
        outstanding = []
        while n_done < len(reqs):
            while seen < len(reqs) and tickets[seen] is not None:
                outstanding.append(seen)
                seen += 1
            still = []
            for q in outstanding:
                r = srv.poll(tickets[q], len(reqs[q].seeds))
                if r is None:
                    still.append(q)
                    continue
                st = r[2]
                n_done += 1
                lat.append((st["t_done_ns"] - st["t_arrive_ns"]) * 1e-6)
                tuples += st["tuples"]
                first = st["t_arrive_ns"] if first is None else min(first, st["t_arrive_ns"])
                last = st["t_done_ns"] if last is None else max(last, st["t_done_ns"])
            outstanding = still
            time.sleep(0.0002)
        th.join()
        lat = np.array(lat)
        res.append({"rate_req_s": rate, "requests": len(reqs), "p50_ms": float(np.percentile(lat, 50)),
                    "p99_ms": float(np.percentile(lat, 99)), "tuples_per_s": tuples / ((last - first) * 1e-9),
                    "mean_seeds": float(np.mean([len(r.seeds) for r in reqs]))})
        log(f"serve {dtype} {rate} req/s: p50 {res[-1]['p50_ms']:.2f} ms, p99 {res[-1]['p99_ms']:.2f} ms, "
            f"{res[-1]['tuples_per_s'] / 1e6:.1f} M tuples/s")
    srv.close()
    return res


def copy_calibration(gib: float):
    """A plain device copy of known size, for scaling HBM byte counters."""
    import torch

    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}), flush=True)


def sample_groups(g, budget_tuples: int):
    """A seeded sample of output groups of both layer-1 rules (all tuples of
    the sampled groups), about budget_tuples / 2 tuples per rule."""
    rng = np.random.default_rng(42)
    out = {}
    for name, keys, n in (("item", g.buys_i, g.item.shape[0]), ("user", g.buys_u, g.user.shape[0])):
        cnt = np.bincount(keys, minlength=n)
        cand = rng.permutation(np.nonzero(cnt)[0])
        take, acc = [], 0
        for k in cand:
            if acc + cnt[k] > budget_tuples // 2:
                continue
            take.append(k)
            acc += cnt[k]
            if acc >= 0.9 * (budget_tuples // 2):
                break
        out[name] = np.sort(np.array(take, np.int64))
    return out


def gpu_rows(net, D, keys):
    """Layer-1 outputs of the sampled groups (FP32 on the host)."""
    import torch

    res = {}
    for name, q, gk in (("item", 0, D["keys"][0]), ("user", 1, D["keys"][1])):
        pos = torch.searchsorted(gk.long(), torch.from_numpy(keys[name]).to(gk.device))
        res[name] = net.out[q].index_select(0, pos).float().cpu().numpy()
    return res


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(g, keys):
    """The FP64 oracle, as it stands, on the sampled output groups of both
    layer-1 rules: once on one thread (BLAS limited to one) and once on all
    the host's cores.  Returns the line's field and the oracle's outputs
    (pre-activation aggregates and outputs per rule) for the error report."""
    import relgen
    from oracle import relnn_oracle as orc
    from threadpoolctl import threadpool_limits

    rules = {}
    for name in ("item", "user"):
        bk = g.buys_i if name == "item" else g.buys_u
        sel = np.isin(bk, keys[name])
        sub = relgen.ERGraph(g.user, g.item, g.cat, g.buys_u[sel], g.buys_i[sel], g.belongs_cat,
                             g.W_item, g.W_user, g.b_item, g.b_user)
        rules[name] = relgen.er_item_rule(sub) if name == "item" else relgen.er_user_rule(sub)

    def run_all():
        t0 = time.perf_counter()
        outs, tuples = {}, 0
        for name, rule in rules.items():
            idx = orc.build_index(rule)
            outs[name] = orc.layer_fwd(idx, [a.emb for a in rule.atoms], rule.W, rule.b, rule.agg, rule.act_pre,
                                       rule.act_post)[:2]
            tuples += idx.E
        return tuples, time.perf_counter() - t0, outs

    with threadpool_limits(limits=1):
        t1, s1, _ = run_all()
    tn, sn, outs = run_all()
    model, cores = cpu_info()
    field = {"value": tn / sn, "unit": "tuples/s", "cores": cores, "kind": "oracle",
             "single_thread_value": t1 / s1, "cpu_model": model,
             "sample": f"layer-1 forward of both ER rules over a seeded sample of output groups "
                       f"({len(keys['item'])} Item groups, {len(keys['user'])} User groups, {tn} tuples): "
                       f"{sn:.1f}s on all {cores} cores, {s1:.1f}s on one thread, FP64 numpy"}
    return field, outs


def row_errors(gpu, outs):
    """max and p99 over the sampled rows of |z - z_ref| / |pre_ref| (rows of
    both rules together)."""
    errs = []
    for name in ("item", "user"):
        o_out, o_pre = outs[name]
        den = np.maximum(np.linalg.norm(o_pre, axis=1), 1e-30)
        errs.append(np.linalg.norm(gpu[name].astype(np.float64) - o_out, axis=1) / den)
    e = np.concatenate(errs)
    return {"max": float(e.max()), "p99": float(np.percentile(e, 99)), "rows": int(e.size),
            "vs": "FP64 oracle on the FP32 master values, sampled output groups"}


def cfg1_leg(reps: int):
    """Workload 1: Node [1000, 32], Edge 5000 (s, t uniform), W [64, 32]
    ~ N(0, 0.1), SUM then ReLU, FP32; fused and plain.  Launch-latency bound
    (20 MFLOP, L2-resident): tuples/s over `reps` back-to-back layer calls,
    and the error of the whole output against the FP64 oracle."""
    import torch

    import relgen
    from oracle import relnn_oracle as orc
    from paper_2605_24207_amd import Index, Layer, layer_fwd, workspace

    rule = relgen.node_edge()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ix = Index([t(c) for c in rule.cols], [(1000, 0, None), (1000, 1, None)], 1)
    z, W, b = t(rule.atoms[0].emb), t(rule.W), t(rule.b)
    res = {"workload": "Node 1000 x 32, Edge 5000, W [64, 32], SUM, ReLU, FP32", "tuples": ix.E, "groups": ix.G}
    idx = orc.build_index(rule)
    o_out, o_pre, _ = orc.layer_fwd(idx, [rule.atoms[0].emb] * 2, rule.W, rule.b, "sum", "none", "relu")
    for name, plain in (("fused", False), ("plain", True)):
        L = Layer([32, 32], 32, "f32", "sum", "none", "relu", plain=plain)
        ws = workspace(ix, L)
        out = torch.empty(ix.G, 32, device="cuda")
        for _ in range(20):
            layer_fwd(ix, L, [z, z], W, b, want_pre=False, ws=ws, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            layer_fwd(ix, L, [z, z], W, b, want_pre=False, ws=ws, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        err = np.linalg.norm(out.cpu().numpy() - o_out, axis=1) / np.maximum(np.linalg.norm(o_pre, axis=1), 1e-30)
        res[name] = {"value": ix.E / dt, "unit": "tuples/s", "us_per_layer": dt * 1e6, "max_row_err": float(err.max())}
    return res


def time_calls(fn, reps: int, warmup: int = 2):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def next_legs(D, reps: int):
    """The rows built beyond the plain layer, each at a size of the ER
    workload's scale, with joined tuples/s and the bytes each path must move:
      attention  HGT-like head: 2M targets, 4M sources, 20M (target, source)
                 tuples with Zipf(1.1) targets, d = dv = 128, 8 heads, FP32
                 and BF16; forward and backward;
      union      Item(i) as the union of two bodies (the Item rule over the
                 first 10M Buys rows, the User rule's body grouped by item over
                 the other 10M), MEAN applied once, FP32; forward and backward;
      product    Item(i; mean(relu(z_u * z_i * z_c))) over Buys (20M), FP32;
                 forward and backward;
      triangle   the DHN triangle rule on 20k graphs of 40 nodes (index build
                 by sort-and-probe joins, then the layer), FP32."""
    import torch

    import relgen
    from paper_2605_24207_amd import (Index, Layer, Union, api, attn_bwd, attn_fwd, layer_bwd, layer_fwd,
                                      union_bwd, union_fwd, workspace)

    res = {}
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    # attention
    rng = np.random.default_rng(7)
    n_t, n_s, E, d = 2_000_000, 4_000_000, 20_000_000, 128
    tgt = relgen.zipf_ids(rng, E, n_t, 1.1).astype(np.int32)
    src = rng.integers(0, n_s, E).astype(np.int32)
    ix = Index([t(tgt), t(src)], [(n_t, 0, None), (n_s, 1, None), (n_s, 1, None)], 0, bwd=True)
    Qf = torch.randn(n_t, d, device="cuda")
    Kf = torch.randn(n_s, d, device="cuda")
    Vf = torch.randn(n_s, d, device="cuda")
    att = {"workload": "2M targets, 4M sources, 20M tuples (targets Zipf 1.1), d = dv = 128, 8 heads",
           "tuples": ix.E, "groups": ix.G}
    for dt in ("f32", "bf16"):
        cv = (lambda x: x.to(torch.bfloat16)) if dt == "bf16" else (lambda x: x)
        q, k, v = cv(Qf), cv(Kf), cv(Vf)
        esz = 2 if dt == "bf16" else 4
        ms = time_calls(lambda: attn_fwd(ix, q, k, v, 8, 0.25), reps) * 1e3
        out, lse = attn_fwd(ix, q, k, v, 8, 0.25)
        dout = torch.randn_like(out)
        dq, dk, dv = (torch.zeros(x.shape, device="cuda") for x in (q, k, v))
        msb = time_calls(lambda: attn_bwd(ix, q, k, v, 8, 0.25, out, lse, dout, dq, dk, dv), max(1, reps // 2)) * 1e3
        # Algorithmic bytes.  A row that is constant inside a group (here Q's,
        # keyed by the target) counts once per group: the tuples come sorted
        # by group, so it need not move more than once.  Forward: k and v
        # rows and three row numbers per tuple; the q row, the output and the
        # log-sum-exps per group.
        byt = ix.E * (2 * d * esz + 12) + ix.G * (d * esz + d * 4 + 8 * 4)
        # backward: the weights pass reads k and v rows and writes two
        # weights per head per tuple, and per group the q and dout rows, D
        # and lse, and writes dQ; the dK and dV gather-sums read a q or dout
        # row, the head weights and three numbers per tuple, and add into
        # each source row once
        byt_b = (ix.E * (2 * d * esz + 2 * 8 * 4 + 12) + ix.G * (d * esz + 2 * d * 4 + 2 * 8 * 4)
                 + ix.E * (d * esz + 8 * 4 + 12) + ix.E * (d * 4 + 8 * 4 + 12) + 2 * n_s * d * 4 * 2)
        att[dt] = {"fwd_ms": ms, "fwd_tuples_per_s": ix.E / (ms * 1e-3), "fwd_hbm_gbs_algorithmic": byt / (ms * 1e-3) / 1e9,
                   "bwd_ms": msb, "fwd_bwd_tuples_per_s": ix.E / ((ms + msb) * 1e-3),
                   "roofline": {"bound": "hbm", "unit": "GB/s", "peak": PEAK_HBM_GBS,
                                "fwd_achieved": byt / (ms * 1e-3) / 1e9, "fwd_frac": byt / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                "bwd_achieved": byt_b / (msb * 1e-3) / 1e9,
                                "bwd_frac": byt_b / (msb * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                "fwd_bytes": byt, "bwd_bytes": byt_b}}
        log(f"attention {dt}: fwd {ms:.2f} ms, bwd {msb:.2f} ms")
    res["attention"] = att
    del ix, Qf, Kf, Vf, q, k, v, out, lse, dout, dq, dk, dv
    torch.cuda.empty_cache()
    # union of two bodies of Item(i)
    g = D["g"]
    half = len(g.buys_u) // 2
    nu, ni, nc = g.user.shape[0], g.item.shape[0], g.cat.shape[0]
    b1 = Index([D["bu"][:half].contiguous(), D["bi"][:half].contiguous()], [(nu, 0, None), (ni, 1, None),
                                                                            (nc, 2, None)], 1,
               chains=[(1, D["bc"], None)], bwd=True)
    b2 = Index([D["bu"][half:].contiguous(), D["bi"][half:].contiguous()], [(nu, 0, None), (ni, 1, None)], 1,
               bwd=True)
    U = Union([b1, b2])
    L1 = Layer([128, 128, 128], 128, "f32", "mean")
    L2 = Layer([128, 128], 128, "f32", "mean")
    fn = lambda: union_fwd(U, [L1, L2], "mean", "relu", [[D["U"], D["I"], D["C"]], [D["U"], D["I"]]],
                           [D["W_item"][0], D["W_user"][0]], [D["b_item"][0], D["b_user"][0]], want_pre=False)
    ms = time_calls(fn, reps) * 1e3
    ufl = b1.E * (2 * 384 * 128 + 2 * 128) + b2.E * (2 * 256 * 128 + 2 * 128)
    # backward of affine MEAN branches: per tuple the joined row is gathered
    # again (FP32, for the per-group sums that dW needs) and, for every atom
    # not keyed by the group, the routed gradient row and its row numbers are
    # read in that atom's transpose order; every joined row's gradient is
    # read and written once per branch.  The products themselves are per
    # group and per joined row, not per tuple.
    ub_bytes = (b1.E * (384 * 4 + 2 * (128 * 4 + 8) + 12) + b2.E * (256 * 4 + (128 * 4 + 8) + 8)
                + 2 * (nu + ni) * 128 * 8 + nc * 128 * 8)
    uembs = [[D["U"], D["I"], D["C"]], [D["U"], D["I"]]]
    uW = [D["W_item"][0], D["W_user"][0]]
    ub = [D["b_item"][0], D["b_user"][0]]
    uout, upre, _ = union_fwd(U, [L1, L2], "mean", "relu", uembs, uW, ub)
    udout = torch.randn_like(uout)
    ug = {k: torch.zeros(D[k].shape, device="cuda") for k in ("U", "I", "C")}
    udemb = [[ug["U"], ug["I"], ug["C"]], [ug["U"], ug["I"]]]
    udW = [torch.empty(384, 128, device="cuda"), torch.empty(256, 128, device="cuda")]
    udb = [torch.empty(128, device="cuda"), torch.empty(128, device="cuda")]
    msb = time_calls(lambda: union_bwd(U, [L1, L2], "mean", "relu", uembs, uW, ub, None, None, upre, None, udout,
                                       udemb, udW, udb), max(1, reps // 2)) * 1e3
    res["union"] = {"workload": "Item(i) over two bodies: Item rule on Buys rows 0..10M (K = 384), User body "
                                "grouped by item on rows 10M..20M (K = 256); MEAN once; FP32",
                    "ms": ms, "tuples_per_s": (b1.E + b2.E) / (ms * 1e-3), "groups": U.G,
                    "bwd_ms": msb, "fwd_bwd_tuples_per_s": (b1.E + b2.E) / ((ms + msb) * 1e-3),
                    "roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": PEAK_TFLOPS["f32"],
                                 "achieved": ufl / (ms * 1e-3) / 1e12,
                                 "frac": ufl / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["f32"], "flop": ufl},
                    "bwd_roofline": {"bound": "hbm", "unit": "GB/s", "peak": PEAK_HBM_GBS,
                                     "achieved": ub_bytes / (msb * 1e-3) / 1e9,
                                     "frac": ub_bytes / (msb * 1e-3) / 1e9 / PEAK_HBM_GBS, "bytes": ub_bytes}}
    log(f"union: fwd {ms:.2f} ms, bwd {msb:.2f} ms")
    del U, b1, b2, uout, upre, udout, ug, udemb, udW, udb
    torch.cuda.empty_cache()
    # product transform
    ixp = D["ix_item1"]
    Lp = Layer([128, 128, 128], 128, "f32", "mean", "relu", "none", transform="product")
    wsp = workspace(ixp, Lp)
    outp = torch.empty(ixp.G, 128, device="cuda")
    ms = time_calls(lambda: layer_fwd(ixp, Lp, [D["U"], D["I"], D["C"]], None, want_pre=False, ws=wsp, out=outp),
                    reps) * 1e3
    # forward: the User row and four numbers per tuple; the Item and
    # Category rows, constant inside a group, once per group, and the output
    byt = ixp.E * (128 * 4 + 16) + ixp.G * (2 * 128 * 4 + 128 * 4)
    # backward (on an index with the transpose orders).  Item and Category
    # are constant inside a group, so their product Q_g is formed once per
    # group: the User pass reads, per tuple, the group's R_g = dA_g * Q_g row,
    # its sign bits and three row numbers; the per-group sum pass reads the
    # User row and two numbers; the Category pass two numbers; per group the
    # Item, Category, dA, R, S and V rows move once; every joined row's
    # gradient is read and written once
    ixpb = Index([D["bu"], D["bi"]], [(nu, 0, None), (ni, 1, None), (nc, 2, None)], 1,
                 chains=[(1, D["bc"], None)], bwd=True)
    pembs = [D["U"], D["I"], D["C"]]
    pout, _, _ = layer_fwd(ixpb, Lp, pembs, None)
    pdout = torch.randn_like(pout)
    pg = [torch.zeros(x.shape, device="cuda") for x in pembs]
    msb = time_calls(lambda: layer_bwd(ixpb, Lp, pembs, None, None, None, None, pdout, pg, None),
                     max(1, reps // 2)) * 1e3
    byt_b = (ixpb.E * (128 * 4 + 32 + 12) + ixpb.E * (128 * 4 + 8) + ixpb.E * 8 + ixpb.G * (7 * 128 * 4 + 32)
             + sum(x.shape[0] * 128 * 8 for x in pembs))
    res["product"] = {"workload": "Item(i; mean(relu(z_u * z_i * z_c))) over Buys 20M, FP32", "ms": ms,
                      "tuples_per_s": ixp.E / (ms * 1e-3), "hbm_gbs_algorithmic": byt / (ms * 1e-3) / 1e9,
                      "bwd_ms": msb, "fwd_bwd_tuples_per_s": ixp.E / ((ms + msb) * 1e-3),
                      "roofline": {"bound": "hbm", "unit": "GB/s", "peak": PEAK_HBM_GBS,
                                   "achieved": byt / (ms * 1e-3) / 1e9,
                                   "frac": byt / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, "bytes": byt,
                                   "bwd_achieved": byt_b / (msb * 1e-3) / 1e9,
                                   "bwd_frac": byt_b / (msb * 1e-3) / 1e9 / PEAK_HBM_GBS, "bwd_bytes": byt_b}}
    log(f"product: fwd {ms:.2f} ms, bwd {msb:.2f} ms")
    del ixpb, pout, pdout, pg
    torch.cuda.empty_cache()
    # triangle rule
    rule = relgen.triangle_rule(n_graphs=20_000, n_nodes=40, avg_degree=6, d=64, h=64)
    tc = lambda cols: [t(c) for c in cols]
    mk = lambda: Index(tc(rule.cols), [(a.n_rows, a.col, None) for a in rule.atoms], rule.group_col,
                       steps=[(tc(st.cols), st.on, st.key) for st in rule.steps])
    t0 = time.perf_counter()
    ixt = mk()
    torch.cuda.synchronize()
    build = time.perf_counter() - t0
    Lt = Layer([64, 64, 64], 64, "f32", "sum", "none", "relu")
    z = t(rule.atoms[0].emb)
    Wt, bt = t(rule.W), t(rule.b)
    wst = workspace(ixt, Lt)
    outt = torch.empty(ixt.G, 64, device="cuda")
    ms = time_calls(lambda: layer_fwd(ixt, Lt, [z, z, z], Wt, bt, want_pre=False, ws=wst, out=outt), reps) * 1e3
    tfl = ixt.E * (2 * 192 * 64 + 2 * 64)
    res["triangle"] = {"workload": "C3(n; sum(Lin(h_n (+) h_v (+) h_w))) on 20k graphs x 40 nodes, 4.8M directed "
                                   "edges, d = h = 64, FP32", "matches": ixt.E, "index_build_s": build,
                       "layer_ms": ms, "tuples_per_s": ixt.E / (ms * 1e-3),
                       "roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": PEAK_TFLOPS["f32"],
                                    "achieved": tfl / (ms * 1e-3) / 1e12,
                                    "frac": tfl / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["f32"], "flop": tfl}}
    log(f"triangle: {ixt.E} matches, build {build:.2f} s, layer {ms:.2f} ms")
    return res


def cobuy_error(g, gpu_out, gpu_keys, frac=0.01):
    """gpu_out / gpu_keys: the co-buy leg's output [G, 256] and group keys
    (device tensors)."""
    import torch

    """Error of the precision form (co-buy MAX, BF16) against the FP64 oracle
    on a seeded sample of its output groups: the oracle's two-hop paths are
    built for every item the sampled users bought (a path list depends only
    on its item's rows), and the sampled groups evaluated."""
    import relgen
    from oracle import relnn_oracle as orc

    rule = relgen.cobuy_rule(g, d=256, h=256, cap=50, agg="max")
    users = np.unique(g.buys_u)
    rng = np.random.default_rng(29)
    samp = np.sort(rng.choice(users, max(1, int(frac * len(users))), replace=False))
    items = np.unique(g.buys_i[np.isin(g.buys_u, samp)])
    sel = np.isin(g.buys_i, items)
    sub = relgen.Rule(cols=[c[sel] for c in rule.cols], atoms=rule.atoms, group_col=rule.group_col, W=rule.W,
                      b=rule.b, agg="max", two_hop_mid=rule.two_hop_mid, two_hop_cap=rule.two_hop_cap)
    idx = orc.build_index(sub)
    groups = np.nonzero(np.isin(idx.group_keys, samp))[0]
    _, pre, _ = orc.layer_fwd(idx, [a.emb for a in rule.atoms], rule.W, rule.b, "max", groups=groups)
    pos = torch.searchsorted(gpu_keys.long(), torch.from_numpy(idx.group_keys[groups]).to(gpu_keys.device))
    z = gpu_out.index_select(0, pos).cpu().numpy().astype(np.float64)
    e = np.linalg.norm(z - pre, axis=1) / np.maximum(np.linalg.norm(pre, axis=1), 1e-30)
    return {"max": float(e.max()), "p99": float(np.percentile(e, 99)), "rows": int(len(groups)),
            "vs": "FP64 oracle on the FP32 master values, 1% of the output groups"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the workload (testing only)")
    ap.add_argument("--cpu-budget", type=int, default=4_000_000, help="oracle sample size in tuples")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="f32,plain,bf16,push_f32,push_bf16,cobuy_bf16,serve,fwdbwd,fwdbwd_bf16,"
                                      "fwdbwd_push,cfg1,next",
                    help="comma list of f32,plain,bf16,push_f32,push_bf16,cobuy_bf16,serve,fwdbwd,fwdbwd_bf16,"
                         "fwdbwd_push,cfg1,next")
    ap.add_argument("--serve-seconds", type=float, default=15.0, help="arrival window per serving rate")
    ap.add_argument("--serve-rates", default="200,1000,2000", help="Poisson arrival rates (req/s)")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="only run a plain copy of this many GiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_gib > 0:
        copy_calibration(args.copy_gib)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(it would shard the tuple list by group ranges; not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    legs = set(args.legs.split(","))
    D = build_workload(args.scale)
    keys = sample_groups(D["g"], args.cpu_budget)
    gpu_sample = {}
    res = {}
    for leg in ("f32", "plain", "bf16", "push_f32", "push_bf16"):
        if leg not in legs:
            continue
        dtype = "bf16" if leg.endswith("bf16") else "f32"
        net = Net(D, dtype, plain=(leg == "plain"), pushdown=leg.startswith("push"))
        kern = (["fwd_gather", "fwd_gemm", "fwd_reduce"] if leg == "plain" else
                ["fwd_push"] if leg.startswith("push") else ["fwd_fused"])
        steps = args.steps if leg != "plain" else max(1, args.steps // 2)
        dt, kt = time_net(net, steps, args.warmup, kern)
        res[leg] = {"dt": dt, "steps": steps, "kt": kt, "tuples": net.tuples, "flops": net.flops,
                    "bytes": net.bytes}
        gpu_sample[leg] = gpu_rows(net, D, keys)
        log(f"{leg}: {dt / steps * 1e3:.2f} ms/step, {net.tuples * steps / dt / 1e9:.3f} G tuples/s; "
            + ", ".join(f"{k} {v[0] / max(v[1], 1):.3f} ms x{v[1]}" for k, v in kt.items()))
        del net
        torch.cuda.empty_cache()

    line = {"metric": METRIC, "value": None, "unit": "tuples/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "ER schema User 1M / Item 500k / Category 1k, Buys 20M (item Zipf 1.1), "
                                   "hidden 128, 2 layers x (Item SUM K=384, User MEAN K=256), ReLU, FP32 forward",
                       "scale": args.scale, "layers_per_step": 4, "index_build_s": round(D["index_build_s"], 3)}}
    value = None
    if "f32" in res:
        main_leg = res["f32"]
        value = main_leg["tuples"] * main_leg["steps"] / main_leg["dt"]
        k_ms, k_n = main_leg["kt"]["fwd_fused"]
        launches_per_step = k_n / main_leg["steps"]
        flops_per_launch = main_leg["flops"] / launches_per_step
        achieved = flops_per_launch / (k_ms / k_n * 1e-3) / 1e12
        line.update({"value": value, "steps": main_leg["steps"],
                     "ms_per_step": main_leg["dt"] / main_leg["steps"] * 1e3})
        line["config"]["tuples_per_step"] = main_leg["tuples"]
        line["roofline"] = {"bound": "mfma", "kernel": "k_fwd_dma<float> (fused FP32 forward)",
                            "achieved": achieved, "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                            "frac": achieved / PEAK_TFLOPS["f32"], "traffic": measured_traffic(),
                            "avg_launch_ms": k_ms / k_n,
                            "flop_per_launch": flops_per_launch,
                            "hbm_gbs_algorithmic": gbs(main_leg["bytes"]["fused"], main_leg["steps"],
                                                       main_leg["kt"]["fwd_fused"])}
    for leg, key in (("plain", "plain_f32"), ("bf16", "fused_bf16"), ("push_f32", "pushdown_f32"),
                     ("push_bf16", "pushdown_bf16")):
        if leg in res:
            r = res[leg]
            line[key] = {"value": r["tuples"] * r["steps"] / r["dt"], "unit": "tuples/s",
                         "ms_per_step": r["dt"] / r["steps"] * 1e3,
                         "kernels_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in r["kt"].items()}}
    if "plain" in res:
        r = res["plain"]
        if value is not None:
            line["speedup_vs_plain_f32"] = value / line["plain_f32"]["value"]
        line["plain_f32"]["hbm_gbs"] = {k: gbs(r["bytes"][k], r["steps"], r["kt"]["fwd_" + k])
                                        for k in ("gather", "reduce")}
        line["plain_f32"]["gemm_tflops"] = (r["flops"] * r["steps"] / (r["kt"]["fwd_gemm"][0] * 1e-3) / 1e12
                                            if r["kt"]["fwd_gemm"][0] > 0 else None)
        line["plain_f32"]["hbm_peak_gbs"] = PEAK_HBM_GBS
        # DRAM bytes by rocprof counters (copy-calibrated FETCH_SIZE + WRITE_SIZE per launch)
        cnt = {k: measured_value("plain_er_counters.md", ["layer_fwd.hip", "plain.hip"], f"{k}_hbm_bytes_per_launch")
               for k in ("gather", "reduce")}
        line["plain_f32"]["hbm_gbs_counters"] = {
            k: (cnt[k] / (r["kt"]["fwd_" + k][0] / r["kt"]["fwd_" + k][1] * 1e-3) / 1e9 if cnt[k] else None)
            for k in ("gather", "reduce")}
    if "bf16" in res:
        r = res["bf16"]
        bk_ms, bk_n = r["kt"]["fwd_fused"]
        line["fused_bf16"]["speedup_vs_plain_f32"] = (line["fused_bf16"]["value"] / line["plain_f32"]["value"]
                                                      if "plain" in res else None)
        line["fused_bf16"]["mfma_tflops"] = r["flops"] / (bk_n / r["steps"]) / (bk_ms / bk_n * 1e-3) / 1e12
        line["fused_bf16"]["hbm_gbs_algorithmic"] = gbs(r["bytes"]["fused"], r["steps"], r["kt"]["fwd_fused"])
    if "cobuy_bf16" in legs:
        cb = cobuy_leg(D, args.steps, args.warmup)
        line["cobuy_bf16"] = cb
        log(f"cobuy bf16: {cb['ms_per_step']:.2f} ms/step, {cb['value'] / 1e9:.3f} G tuples/s, "
            f"{cb['kernel_ms_per_launch']:.3f} ms/launch")
        if not args.no_cpu_baseline:
            t0 = time.perf_counter()
            cb["error"] = cobuy_error(D["g"], *D.pop("cobuy_out"))
            log(f"cobuy error against the oracle in {time.perf_counter() - t0:.1f}s: {cb['error']}")
        D.pop("cobuy_out", None)
        torch.cuda.empty_cache()
    if "cfg1" in legs:
        line["workload1_f32"] = cfg1_leg(2000)
        log(f"workload 1: {line['workload1_f32']}")
    if "next" in legs:
        line["next_rows"] = next_legs(D, args.steps)
        torch.cuda.empty_cache()
    if "serve" in legs:
        rates = [float(x) for x in args.serve_rates.split(",")]
        line["serve"] = {"workload": "resident ER graph (Buys 20M); requests of log-uniform 1..4096 seed items, "
                                     "fanout 15 then 10, Poisson arrivals; budget 64 GiB",
                         "fused_f32": serve_leg(D, "f32", rates, args.serve_seconds),
                         "fused_bf16": serve_leg(D, "bf16", rates, args.serve_seconds)}
    g_host = D["g"]
    if legs & {"fwdbwd", "fwdbwd_bf16", "fwdbwd_push"}:
        del D
        torch.cuda.empty_cache()
    for leg, dt, key in (("fwdbwd", "f32", "fwd_bwd_f32"), ("fwdbwd_bf16", "bf16", "fwd_bwd_bf16"),
                         ("fwdbwd_push", "f32", "fwd_bwd_f32_pushdown")):
        if leg not in legs:
            continue
        fb = fwd_bwd_leg(max(1, args.steps // 2), args.warmup, args.scale, dt, pushdown=leg == "fwdbwd_push")
        line[key] = fb
        log(f"fwd+bwd {leg}: {fb['ms_per_step']:.2f} ms/step, {fb['value'] / 1e9:.3f} G tuples/s; " +
            ", ".join(f"{k} {v:.3f} ms" for k, v in fb["kernels_ms_per_launch"].items()))
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        line["cpu_baseline"], outs = cpu_baseline(g_host, keys)
        log(f"cpu baseline in {time.perf_counter() - t0:.1f}s")
        # accuracy of the fused legs on the same sampled groups (layer 1)
        line["accuracy"] = {leg: row_errors(gpu_sample[leg], outs) for leg in ("f32", "bf16", "plain",
                                                                                 "push_f32", "push_bf16")
                            if leg in gpu_sample}
        if "cobuy_bf16" in line and "error" in line["cobuy_bf16"]:
            line["accuracy"]["cobuy_bf16"] = line["cobuy_bf16"]["error"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
