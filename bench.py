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


def measured_traffic():
    """HBM bytes per launch of the fused FP32 forward from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when
    the kernel source has changed since the counters were taken."""
    import hashlib
    import re

    summ = os.path.join(ROOT, "profiles", "fused_fwd_er_counters.md")
    src = os.path.join(ROOT, "paper_2605_24207_amd", "csrc", "layer_ws.hip")
    try:
        text = open(summ).read()
        have = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        want = re.search(r"source_sha256_prefix:\s*([0-9a-f]+)", text).group(1)
        val = float(re.search(r"traffic_bytes_per_launch_fused_f32:\s*([0-9.e+]+)", text).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    return val if have == want else None


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
        done, lat, tuples, first, last = set(), [], 0, None, None
        while len(done) < len(reqs):
            for q, t in enumerate(tickets):
                if t is None or q in done:
                    continue
                r = srv.poll(t, len(reqs[q].seeds))
                if r is None:
                    continue
                st = r[2]
                done.add(q)
                lat.append((st["t_done_ns"] - st["t_arrive_ns"]) * 1e-6)
                tuples += st["tuples"]
                first = st["t_arrive_ns"] if first is None else min(first, st["t_arrive_ns"])
                last = st["t_done_ns"] if last is None else max(last, st["t_done_ns"])
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


def cpu_baseline(D, budget_tuples: int):
    """The FP64 oracle, as it stands, on a seeded sample of output groups of
    both rules (all tuples of the sampled groups)."""
    import relgen
    from oracle import relnn_oracle as orc

    g = D["g"]
    rng = np.random.default_rng(42)
    total_t, total_s, desc = 0, 0.0, []
    for name, gcol in (("item", 1), ("user", 0)):
        keys = g.buys_i if gcol == 1 else g.buys_u
        cnt = np.bincount(keys, minlength=(g.item if gcol == 1 else g.user).shape[0])
        cand = rng.permutation(np.nonzero(cnt)[0])
        take, acc = [], 0
        for k in cand:
            if acc + cnt[k] > budget_tuples // 2:
                continue
            take.append(k)
            acc += cnt[k]
            if acc >= 0.9 * (budget_tuples // 2):
                break
        sel = np.isin(keys, np.array(take))
        sub = relgen.ERGraph(g.user, g.item, g.cat, g.buys_u[sel], g.buys_i[sel], g.belongs_cat,
                             g.W_item, g.W_user, g.b_item, g.b_user)
        rule = relgen.er_item_rule(sub) if gcol == 1 else relgen.er_user_rule(sub)
        t0 = time.perf_counter()
        idx = orc.build_index(rule)
        orc.layer_fwd(idx, [a.emb for a in rule.atoms], rule.W, rule.b, rule.agg, rule.act_pre,
                      rule.act_post)
        total_s += time.perf_counter() - t0
        total_t += idx.E
        desc.append(f"{len(take)} {name} groups ({idx.E} tuples)")
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = 1
    return {"value": total_t / total_s, "unit": "tuples/s", "cores": int(cores), "kind": "oracle",
            "sample": "layer-1 forward of both rules over a seeded sample of output groups: "
                      + ", ".join(desc) + f"; {total_s:.1f}s of FP64 numpy"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the workload (testing only)")
    ap.add_argument("--cpu-budget", type=int, default=9_000_000, help="oracle sample size in tuples")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="f32,plain,bf16,push_f32,push_bf16,cobuy_bf16,serve,fwdbwd,fwdbwd_bf16,"
                                      "fwdbwd_push",
                    help="comma list of f32,plain,bf16,push_f32,push_bf16,cobuy_bf16,serve,fwdbwd,fwdbwd_bf16,"
                         "fwdbwd_push")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="arrival window per serving rate")
    ap.add_argument("--serve-rates", default="200,500,1000,2000", help="Poisson arrival rates (req/s)")
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
        line["cpu_baseline"] = cpu_baseline({"g": g_host}, args.cpu_budget)
        log(f"cpu baseline in {time.perf_counter() - t0:.1f}s")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
