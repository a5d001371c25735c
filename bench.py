#!/usr/bin/env python3
"""Throughput of exact Expected Force on one MI355X.

Workload: R-MAT scale 22, edge factor 10 (a=.57 b=.19 c=.19 d=.05),
symmetrised, self-loops and duplicates removed, ids shuffled (seed 1,
permutation seed 3): 4,194,304 nodes, ~40.6M undirected edges, synthetic.

One step = the whole exact hot path on that graph, all nodes, inputs resident
in device memory: degree binning and work lists, cluster generation and
scoring (pair loops), super-tile reduction, triangle pass, per-node sums and
Eq. 1, FP32 recomputation of cancellation-prone seeds. Cluster-centric
formulation (Algorithm 1), FP32 terms with compensated sums.

Prints one JSON line. value = clusters/s where clusters = sum_v k_v(k_v-1)/2
(Algorithm 1's cluster set) per step. Two further workloads are reported
beside it in the same line (they are not the headline value):
  batch     - 512 small graphs (half Watts-Strogatz, half configuration model
              with power-law degrees, n uniform in 1e3..1e5) computed as one
              disjoint union by a replayed HIP graph, against 512 separate calls;
  surrogate - the MLP surrogate trained on exact EF of generator graphs and
              evaluated on a held-out Barabasi-Albert graph (n = 4M, m = 8):
              rank agreement with exact EF, and its speed against the exact path;
  three_events - EF with three transmission events on Barabasi-Albert n = 1e6;
  sir       - 300 SIR outbreaks (about 100 global) on the same Barabasi-Albert
              graph at the paper's calibration, and the correlation of exp(EF)
              with the measured spreading power of orders 1-4.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "clusters/s & EF nodes/s (R-MAT 42M edges), % HBM peak; surrogate vs exact"

# MI355X published FP32 vector peak: 157.3 TFLOP/s = 256 CUs x 2.4 GHz x 256
# flops per CU and clock: 64 lanes, packed FP32 (two values per lane) and an
# FMA counted as two flops.
FP32_VECTOR_PEAK_FLOPS = 157.3e12
# VALU issue peak without packed FP32 (the library is built without it): one
# wave64 instruction per CU and clock, 256 x 2.4 GHz x 64 = 3.93e13 lane
# operations per second for an add, a multiply, an FMA or a DPP add alike.
# On the device, loops of the pair kernel's table step (integer DPP add, add,
# DPP add) issue 1.005 and chains of FMAs 0.98 wave64 instructions per CU and
# clock; the pair kernel issues 1.0 counting each v_log_f32 once.
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9
# Algorithmic VALU instructions per cluster of the super-tile pair loop as
# built: a table-scored cluster takes the table index step, the row credit
# and the column credit (3); a cluster scored with the log takes the degree
# step, the log, the multiply and the two credits (5).
VALU_OPS_TABLE_CLUSTER = 3
VALU_OPS_LOG_CLUSTER = 5
# The scope table's estimate of the cost of one cluster with a log per
# cluster: about 16 FP32 VALU operations (the degree, d log d, the two
# credits, the triangle test's share). Reported beside the roofline: the
# score table removes most of them.
OPS_PER_CLUSTER = 16
# the kernel's rule: a full off-diagonal 64 x 64 tile of a big centre (rows in
# an earlier super-block of 1024 than its columns) whose largest degrees
# satisfy k_p + k_q - 2 < TABLE_ENTRIES reads the table
TABLE_ENTRIES = 8192
# HBM bytes per launch of k_pairs_big<float> at this workload (R-MAT scale 22,
# edge factor 10): FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 from two rocprofv3
# counter runs, each counter scaled by its reading on a 1 GiB copy; mostly the
# super-tile records the kernel writes (one float per entry). Taken on the current kernel (the
# counter summaries sit with the other rocprofv3 summaries); set to None
# whenever the kernel changes.
PAIRS_BIG_TRAFFIC_BYTES = 1.821e9
# Hardware counters of k_pairs_big<float> at the same workload, per launch
# (rocprofv3 --pmc, the counter summaries sit with the other rocprofv3
# summaries): SQ_INSTS_VALU (wave64 VALU instructions), of which
# SQ_INSTS_VALU_TRANS_F32 transcendentals (v_log_f32) and SQ_INSTS_LDS.
# None whenever the kernel changes.
PAIRS_BIG_VALU_INSTS = 5.904e9
PAIRS_BIG_TRANS_INSTS = 1.330e8
PAIRS_BIG_LDS_INSTS = 1.612e9
# VALU cost of one SIR attempt along an arc, in FP32-FMA-equivalent lane slots:
# the counter (2e) K and SplitMix64's two multiplications are three 64-bit
# products of three 32-bit multiplies each, at a quarter of the FMA rate
# (36); three 64-bit xor-shifts (9), the 64-bit additions and xors of the
# counter (4), the threshold compare (2) and the arc's index (3).
SIR_OPS_PER_ARC = 54
# HBM bytes of the attempt kernels per call on the SIR workload below (BA
# n = 1e6, m = 5, 300 outbreaks, seed 2306): FETCH_SIZE x 2.0 + WRITE_SIZE x
# 1.0 summed over the call's launches, from two rocprofv3 counter runs (the
# counter summaries sit with the other rocprofv3 summaries); None whenever
# the kernel changes. Mostly whole lines fetched for the row bounds of each
# frontier node and the column entry of each successful draw.
SIR_ATTEMPT_TRAFFIC_BYTES = 25.1e9


def table_clusters(rp, ci):
    """Clusters of big centres (degree > 1024) that the FP32 super-tile loop
    scores from its LDS table, by the kernel's rule on the degree-sorted rows:
    full 64 x 64 tiles off the diagonal whose largest row and column degrees
    fit, in the off-diagonal super-tiles and inside the diagonal ones."""
    import numpy as np

    deg = np.diff(rp).astype(np.int64)
    total = 0
    for v in np.flatnonzero(deg > 1024):
        k = int(deg[v])
        nbr = np.sort(deg[ci[rp[v]:rp[v + 1]]])
        nb = (k + 63) // 64
        m = nbr[np.minimum(np.arange(nb) * 64 + 63, k - 1)]  # largest degree per block
        full = (np.arange(nb) + 1) * 64 <= k
        # for a full column block j: the row blocks i < j (all full) with
        # m[i] + m[j] - 2 < TABLE_ENTRIES, a prefix since the rows ascend
        fit = np.minimum(np.searchsorted(m, TABLE_ENTRIES + 2 - m, side="left"), np.arange(nb))
        total += int(fit[full].sum()) * 64 * 64
    return total


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def host_cpu():
    """CPU model name and the number of host cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def oracle_sample(rp, ci, order, Ns, threads, budget_s, start_chunk=256):
    """Runs the oracle on seeds order[0..m) in growing chunks until budget_s of
    oracle time is spent; returns (m, event sequences, seconds, N, D, EF)."""
    import numpy as np

    import oracle

    done, seqs, t_used, chunk = 0, 0, 0.0, start_chunk
    outs = []
    while t_used < budget_s and done < order.size:
        seeds = order[done:done + chunk]
        t0 = time.perf_counter()
        outs.append(oracle.ef(rp, ci, seeds=seeds, threads=threads))
        t_used += time.perf_counter() - t0
        seqs += int(Ns[seeds].sum())
        done += seeds.size
        chunk = min(chunk * 2, 65536)
    N, D, E = (np.concatenate([o[i] for o in outs]) for i in range(3))
    return done, seqs, t_used, N, D, E


def cpu_baseline(rp, ci, gpu_out, prec, budget_s=15.0, budget_1t_s=8.0):
    """The CPU oracle (single pass, as it stands) on a bounded random sample of
    seeds of the same graph, on this host's cores (up to 16 threads, OpenMP
    dynamic schedule with chunk 2) and on one thread. Returns Algorithm-1
    clusters per second (each cluster is 4 event sequences across its seeds).
    The oracle's N, D and EF of the sampled seeds are compared with the timed
    GPU step's outputs gpu_out = (EF, D, N): integers bit-exact, EF within the
    precision's relative tolerance."""
    import numpy as np

    import oracle

    model, nproc, usable = host_cpu()
    threads = max(1, min(usable, 16))
    n = rp.size - 1
    deg = np.diff(rp).astype(np.int64)
    src = np.repeat(np.arange(n), deg)
    A = np.bincount(src, weights=deg[ci], minlength=n).astype(np.int64)
    Ns = deg * deg - 2 * deg + A
    order = np.random.default_rng(123).permutation(np.flatnonzero(deg > 0)).astype(np.int32)
    oracle.ef(rp, ci, seeds=order[:64], threads=threads)  # warm caches
    done, seqs, t_used, oN, oD, oE = oracle_sample(rp, ci, order, Ns, threads, budget_s)
    rate = seqs / t_used
    # single thread, on a prefix of the same sample
    d1, s1, t1, _, _, _ = oracle_sample(rp, ci, order, Ns, 1, budget_1t_s, start_chunk=64)
    # parity of the benched step on the sampled seeds
    ef, D, N = gpu_out
    seeds = order[:done]
    tol = 1e-5 if prec == "fp32c" else 1e-9
    int_ok = bool(np.array_equal(N[seeds], oN) and np.array_equal(D[seeds], oD))
    pos = oE > 0
    rel = np.abs(ef[seeds] - oE)
    max_rel = float((rel[pos] / oE[pos]).max()) if pos.any() else 0.0
    ef_ok = bool(np.all(rel <= tol * np.abs(oE)))
    return {"value": rate / 4.0, "unit": "clusters/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} seeds drawn uniformly from the non-isolated nodes of the same "
                      f"graph, {seqs} event sequences in {t_used:.1f} s on {threads} threads; "
                      f"clusters/s = sequences/s / 4",
            "single_thread": {"value": s1 / t1 / 4.0, "unit": "clusters/s", "cores": 1,
                              "sample": f"the first {d1} of the same seeds, {s1} event "
                                        f"sequences in {t1:.1f} s on one thread"},
            "cpu_model": model, "nproc": nproc, "usable_cores": usable,
            "parity": {"seeds": int(done), "integers_bit_exact": int_ok,
                       "ef_max_rel_err": max_rel, "ef_tolerance": tol,
                       "ok": bool(int_ok and ef_ok)}}


def bench_j3(steps, with_cpu):
    """Expected Force with three transmission events (ef_compute_j3) on the
    Barabasi-Albert graph n = 10^6, m = 5, all nodes, FP32C. The unit of work
    is one event sequence (a cluster instance of Sec. 3.3 with j = 3); their
    count is sum N."""
    import numpy as np
    import torch

    from paper_2306_00606_amd import efgpu, gen

    dev = torch.device("cuda:0")
    log("three events: generating BA n = 1e6, m = 5")
    rp, ci = gen.ba_1m()
    n = rp.size - 1
    g = efgpu.Graph(rp, ci, validate=False)
    out = (torch.empty(n, dtype=torch.float64, device=dev),
           torch.empty(n, dtype=torch.int64, device=dev),
           torch.empty(n, dtype=torch.int64, device=dev))
    g.compute(prec="fp32c", out=out, j=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.compute(prec="fp32c", out=out, j=3)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    g.compute(prec="fp32c", out=out, j=3, profile=True)
    st = g.stats()
    seqs = float(out[2].sum().item())
    log(f"three events: {ms:.1f} ms/step, {seqs:.3e} sequences")
    # sequences are accounted for, not scored one by one (the M part of a
    # first event is scored once per distinct d_T): an equivalent rate
    rec = {"workload": "ba_1m_m5", "nodes": n, "arcs": int(ci.size), "precision": "fp32c",
           "steps": steps, "ms_per_step": ms, "sequences": seqs,
           "equivalent_sequences_per_s": seqs / (ms * 1e-3),
           "phases_ms": {"items": st["t_stream_ms"], "finalize": st["t_finalize_ms"],
                         "fp64_recompute": st["t_pass2_ms"]},
           "fp64_recomputed_seeds": int(st["promoted"])}
    g.close()
    if with_cpu:
        import oracle
        threads = max(1, min(os.cpu_count() or 1, 16))
        N3 = out[2].cpu().numpy()
        order = np.random.default_rng(7).permutation(np.flatnonzero(N3 > 0)).astype(np.int32)
        done, total, t_used, chunk = 0, 0.0, 0.0, 64
        while t_used < 10.0 and done < order.size:
            seeds = order[done:done + chunk]
            t1 = time.perf_counter()
            oracle.ef(rp, ci, seeds=seeds, threads=threads, j=3)
            dt = time.perf_counter() - t1
            t_used += dt
            total += float(N3[seeds].sum())
            done += seeds.size
            # size the next chunk to about half of the budget left
            rate = seeds.size / max(dt, 1e-3)
            chunk = int(max(16, min(4096, 0.5 * rate * max(10.0 - t_used, 0.0))))
        rec["cpu_baseline"] = {
            "value": total / t_used, "unit": "sequences/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} seeds drawn uniformly from the nodes with sequences, "
                      f"{total:.3e} sequences in {t_used:.1f} s on {threads} threads"}
    return rec


def bench_sir(runs, with_cpu):
    """SIR outbreaks (ef_sir) on the Barabasi-Albert graph n = 10^6, m = 5 at
    the paper's calibration (beta = 1.3 / (3 <k>), mu = 1/3): 300 outbreaks from
    uniform index cases, of which about 100 are global, the number the paper's
    spreading-power comparison rests on (Sec. 5.4). The
    empirical spreading power of order d of a node is its mean number of
    descendants within d generations of the infection tree over the global
    outbreaks (size >= n / 4) that infected it; reported with its Pearson
    correlation with exp(EF) and with degree over the nodes that have one.
    Roofline of the attempt kernel: VALU slots of the per-arc draws."""
    import numpy as np
    import torch

    from paper_2306_00606_amd import efgpu, gen

    sims, seed = 300, 2306
    log("SIR: generating BA n = 1e6, m = 5")
    rp, ci = gen.ba_1m()
    n = rp.size - 1
    kbar = ci.size / n
    beta, mu = 1.3 / (3.0 * kbar), 1.0 / 3.0
    g = efgpu.Graph(rp, ci, validate=False)
    ef, _, _ = g.compute(prec="fp32c")
    g.sir(beta, mu, seed, sims)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(runs):
        o = g.sir(beta, mu, seed, sims)
    ms = 1e3 * (time.perf_counter() - t0) / runs
    prof = g.sir(beta, mu, seed, sims, profile=True)
    g.close()
    ph = prof["phase_ms"]
    arcs, fsteps = int(o["work"][0]), int(o["work"][1])
    glob = o["size"] >= (n + 3) // 4
    have = o["inf_count"] > 0
    deg = np.diff(rp).astype(np.float64)
    x = np.exp(ef[have])
    pe, pd = [], []
    for d in range(4):
        sp = o["sp_sum"][d][have] / o["inf_count"][have]
        pe.append(float(np.corrcoef(x, sp)[0, 1]))
        pd.append(float(np.corrcoef(deg[have], sp)[0, 1]))
    idx_ef = ef[o["index"]]
    achieved = arcs * SIR_OPS_PER_ARC / (ph["attempts"] * 1e-3)
    rec = {"workload": "ba_1m_m5", "nodes": n, "arcs": int(ci.size), "beta": beta, "mu": mu,
           "outbreaks": sims, "runs": runs, "ms_per_run": ms,
           "outbreaks_per_s": sims / (ms * 1e-3), "arc_visits": arcs,
           "frontier_node_steps": fsteps, "arc_visits_per_s": arcs / (ms * 1e-3),
           "phases_ms": {k: round(v, 4) for k, v in ph.items()},
           "roofline": {"bound": "alu", "kernel": "k_sir_attempt",
                        "achieved": achieved / 1e12, "peak": VALU_LANE_OPS_PEAK / 1e12,
                        "unit": "TOP/s", "frac": achieved / VALU_LANE_OPS_PEAK,
                        "traffic": SIR_ATTEMPT_TRAFFIC_BYTES,
                        "ops_per_arc": SIR_OPS_PER_ARC, "arcs_per_run": arcs,
                        "kernel_ms_per_run": ph["attempts"]},
           "global_outbreaks": int(glob.sum()), "mean_global_size": float(o["size"][glob].mean())
           if glob.any() else None, "nodes_with_spreading_power": int(have.sum()),
           "pearson_expEF_vs_sp_d1_4": pe, "pearson_degree_vs_sp_d1_4": pd,
           "index_case_ef_mean_global": float(idx_ef[glob].mean()) if glob.any() else None,
           "index_case_ef_mean_local": float(idx_ef[~glob].mean()) if (~glob).any() else None}
    log(f"SIR: {ms:.1f} ms per {sims} outbreaks, {int(glob.sum())} global, {arcs:.3e} arcs; "
        f"phases {ph}; Pearson exp(EF) {[round(v, 3) for v in pe]}, "
        f"degree {[round(v, 3) for v in pd]}")
    if with_cpu:
        import oracle
        done, t_used, oc = 0, 0.0, None
        while t_used < 5.0 and done < sims:  # the last call takes 5-10 s
            k = min(sims, max(done + 4, 2 * done))
            t1 = time.perf_counter()
            oc = oracle.sir(rp, ci, beta, mu, seed, k)
            t_used = time.perf_counter() - t1
            done = k
        rec["cpu_baseline"] = {
            "value": done / t_used, "unit": "outbreaks/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {done} of the same outbreaks "
                      f"({int((oc['size'] >= (n + 3) // 4).sum())} global) in {t_used:.1f} s "
                      f"on one thread"}
    return rec


def bench_batch(steps):
    """Config of 512 uneven graphs in one replayed HIP graph vs separate calls."""
    import numpy as np
    import torch

    from paper_2306_00606_amd import efgpu, gen

    dev = torch.device("cuda:0")
    log("batch: generating 512 graphs")
    graphs = gen.batch_512()
    b = efgpu.Batch(graphs)
    n = b.n
    out = (torch.empty(n, dtype=torch.float64, device=dev),
           torch.empty(n, dtype=torch.int64, device=dev),
           torch.empty(n, dtype=torch.int64, device=dev))
    b.autotune("fp32c")
    designs = {}
    for design in ("phased", "persistent"):
        b.compute(out=out, design=design)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            b.compute(out=out, design=design)
        torch.cuda.synchronize()
        designs[design] = 1e3 * (time.perf_counter() - t0) / steps
        b.compute(out=out, design=design, profile=True)
        designs[design + "_kernel_ms"] = b.stats()["replay_ms"]
    bst = b.stats()
    tuned = "persistent" if bst["design"] == 1 else "phased"
    replay_ms = designs[tuned]
    b.close()
    # the same work as 512 separate calls (graphs loaded beforehand, device outputs)
    gs = [efgpu.Graph(rp, ci, validate=False) for rp, ci in graphs]
    outs = [(torch.empty(g.n, dtype=torch.float64, device=dev),
             torch.empty(g.n, dtype=torch.int64, device=dev),
             torch.empty(g.n, dtype=torch.int64, device=dev)) for g in gs]
    for g, o in zip(gs, outs):
        g.compute(out=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, o in zip(gs, outs):
        g.compute(out=o)
    torch.cuda.synchronize()
    sep_ms = 1e3 * (time.perf_counter() - t0)
    for g in gs:
        g.close()
    W = int(bst["clusters"])
    log(f"batch: replay {replay_ms:.2f} ms ({tuned}; phased {designs['phased']:.2f}, "
        f"persistent {designs['persistent']:.2f}), separate calls {sep_ms:.1f} ms")
    return {"workload": "batch512_ws_cm", "graphs": len(graphs), "nodes": n,
            "arcs": int(bst["nnz"]), "clusters": W, "ms_per_batch": replay_ms,
            "tuned_design": tuned, "graphs_per_s": len(graphs) / (replay_ms * 1e-3),
            "clusters_per_s": W / (replay_ms * 1e-3),
            "designs_ms": {k: round(v, 4) for k, v in designs.items()},
            "persistent_items": int(bst["items"]),
            "separate_calls_ms": sep_ms, "speedup_vs_separate": sep_ms / replay_ms,
            "tuned_thresholds": [int(bst["thr8"]), int(bst["thr16"]), int(bst["thr32"])],
            "tune_ms": {"phased": [round(x, 3) for x in bst["tune_ms"]],
                        "persistent": [round(x, 3) for x in bst["persist_tune_ms"]]}}


def bench_surrogate():
    """Train the MLP surrogate on exact EF of generator graphs; evaluate it on a
    held-out Barabasi-Albert graph (n = 4,000,000, m = 8, seed 99)."""
    from paper_2306_00606_amd import efgpu, gen, surrogate

    log("surrogate: labelling training graphs with the exact kernel")
    t0 = time.perf_counter()
    graphs = surrogate.training_graphs(seed=0, count=18)
    X, y = surrogate.labelled_rows(graphs)
    t_label = time.perf_counter() - t0
    sur = efgpu.Surrogate(seed=0)
    rep = sur.train(X, y, lr=3e-3, epochs=20, batch=8192, seed=0, val_fraction=0.05,
                    patience=4)
    log(f"surrogate: trained on {len(y)} rows: {rep}")
    rp, ci = gen.barabasi_albert(4_000_000, 8, 99)
    with efgpu.Graph(rp, ci, validate=False) as g:
        res = surrogate.evaluate(sur, g)
    sur.close()
    log(f"surrogate: {res}")
    res.update({"workload": "ba4m_m8_heldout", "train_rows": int(len(y)),
                "train_graphs": len(graphs), "label_s": t_label, "train": rep})
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--algo", default="cluster", choices=["cluster", "per_seed"])
    ap.add_argument("--prec", default="fp32c", choices=["fp32c", "fp64"])
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--edge-factor", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--per-seed-steps", type=int, default=2,
                    help="also time the per-seed formulation (0 = skip)")
    ap.add_argument("--profile-only", action="store_true",
                    help="only the profiled steps (every phase alone on the stream); for "
                         "kernel-trace runs whose per-kernel averages the roofline uses")
    ap.add_argument("--agg-steps", type=int, default=5,
                    help="also time the degree-class aggregated variant (0 = skip)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-graph batch")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate")
    ap.add_argument("--j3-steps", type=int, default=2,
                    help="also time EF with three transmission events (0 = skip)")
    ap.add_argument("--only", choices=["batch", "surrogate", "three_events", "sir"],
                    help="run only this section and print its record (profiling runs)")
    ap.add_argument("--sir-runs", type=int, default=2,
                    help="also time 300 SIR outbreaks with spreading power (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the exact path runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    if args.only:
        run = {"batch": lambda: bench_batch(max(3, args.steps)), "surrogate": bench_surrogate,
               "three_events": lambda: bench_j3(max(1, args.j3_steps), False),
               "sir": lambda: bench_sir(max(1, args.sir_runs), False)}[args.only]
        print(json.dumps({"section": args.only, "record": run()}))
        return

    import numpy as np
    import torch

    from paper_2306_00606_amd import efgpu, gen

    log(f"generating R-MAT scale {args.scale}, edge factor {args.edge_factor}")
    rp, ci = gen.rmat(args.scale, args.edge_factor, 1, 0.57, 0.19, 0.19, perm_seed=3)
    n = rp.size - 1
    dev = torch.device("cuda:0")
    log("loading graph")
    g = efgpu.Graph(rp, ci, validate=False)
    info = g.info()
    W = info["clusters"]
    ef = torch.empty(n, dtype=torch.float64, device=dev)
    D = torch.empty(n, dtype=torch.int64, device=dev)
    N = torch.empty(n, dtype=torch.int64, device=dev)
    out = (ef, D, N)
    log(f"n={n} nnz={info['nnz']} W={W} max_degree={info['max_degree']}; warmup {args.warmup}")
    ms = None
    if not args.profile_only:
        for _ in range(args.warmup):
            g.compute(algo=args.algo, prec=args.prec, out=out)
        torch.cuda.synchronize()
        log(f"timing {args.steps} steps")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.compute(algo=args.algo, prec=args.prec, out=out)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ms = 1e3 * t / args.steps
        log(f"{ms:.2f} ms/step")

    # per-kernel HIP-event timings on the call's stream (separate profiled steps)
    prof = []
    for _ in range(max(3, min(args.steps, 5))):
        g.compute(algo=args.algo, prec=args.prec, out=out, profile=True)
        prof.append(g.stats())
    st = {k: float(np.mean([p[k] for p in prof])) for k in prof[0]}
    log("phases (ms): " + ", ".join(f"{k[2:-3]}={st[k]:.2f}" for k in st if k.startswith("t_")))
    if ms is None:
        ms = st["t_total_ms"]  # profile-only: phases run one after another

    # dominant kernel: the super-tile pair loop (clusters of centres with k > 1024)
    headline = (args.scale, args.edge_factor) == (22, 10)
    if args.algo == "cluster" and args.prec == "fp32c" and st["t_pairs_big_ms"] > 0:
        t_launch = st["t_pairs_big_ms"] * 1e-3
        w_launch = st["pairs_big"]
        w_table = table_clusters(rp, ci)
        ops = VALU_OPS_TABLE_CLUSTER * w_table + VALU_OPS_LOG_CLUSTER * (w_launch - w_table)
        achieved = ops / t_launch
        counters = None
        if headline and PAIRS_BIG_VALU_INSTS:
            lane_insts = PAIRS_BIG_VALU_INSTS * 64 / t_launch
            counters = {"valu_insts_per_launch": PAIRS_BIG_VALU_INSTS,
                        "trans_insts_per_launch": PAIRS_BIG_TRANS_INSTS,
                        "lds_insts_per_launch": PAIRS_BIG_LDS_INSTS,
                        "valu_insts_per_cluster": PAIRS_BIG_VALU_INSTS * 64 / w_launch,
                        "valu_lane_insts_per_s": lane_insts,
                        "frac_of_issue_peak": lane_insts / VALU_LANE_OPS_PEAK}
        roofline = {"bound": "alu", "kernel": "k_pairs_big<float>",
                    "achieved": achieved / 1e12, "peak": VALU_LANE_OPS_PEAK / 1e12,
                    "unit": "T VALU lane-ops/s", "frac": achieved / VALU_LANE_OPS_PEAK,
                    "traffic": PAIRS_BIG_TRAFFIC_BYTES if headline else None,
                    "valu_ops_per_cluster": {"table": VALU_OPS_TABLE_CLUSTER,
                                             "log": VALU_OPS_LOG_CLUSTER},
                    "clusters_per_launch": w_launch, "table_clusters": w_table,
                    "avg_launch_ms": st["t_pairs_big_ms"], "counters": counters,
                    "scope_ops": {"ops_per_cluster": OPS_PER_CLUSTER,
                                  "achieved_tops": w_launch * OPS_PER_CLUSTER / t_launch / 1e12,
                                  "fp32_vector_peak_tflops": FP32_VECTOR_PEAK_FLOPS / 1e12,
                                  "frac": w_launch * OPS_PER_CLUSTER / t_launch
                                  / FP32_VECTOR_PEAK_FLOPS}}
    else:
        roofline = None
    # the headline step's outputs, before any other section reuses the device
    ef_h, D_h, N_h = ef.cpu().numpy(), D.cpu().numpy(), N.cpu().numpy()

    # the other formulations write their own buffers
    out = tuple(torch.empty_like(x) for x in out)
    per_seed = None
    if args.algo == "cluster" and args.per_seed_steps > 0:
        log(f"per-seed formulation: {args.per_seed_steps} steps")
        g.compute(algo="per_seed", prec=args.prec, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.per_seed_steps):
            g.compute(algo="per_seed", prec=args.prec, out=out)
        torch.cuda.synchronize()
        ps_ms = 1e3 * (time.perf_counter() - t0) / args.per_seed_steps
        g.compute(algo="per_seed", prec=args.prec, out=out, profile=True)
        pst = g.stats()
        # algorithmic bytes of the 2-hop stream: one (id, degree) pair of 8 B per
        # entry of every neighbour's row, sum_a k_a^2 entries in total
        b_stream = 8.0 * info["sum_sq_degree"]
        per_seed = {"ms_per_step": ps_ms, "clusters_per_s": W / (ps_ms * 1e-3),
                    "phases_ms": {k[2:-3]: round(pst[k], 4) for k in pst if k.startswith("t_")},
                    "stream_bytes": b_stream,
                    "stream_GBps": b_stream / (pst["t_stream_ms"] * 1e-3) / 1e9
                    if pst["t_stream_ms"] > 0 else None,
                    "stream_frac_hbm_peak": b_stream / (pst["t_stream_ms"] * 1e-3) / 8.0e12
                    if pst["t_stream_ms"] > 0 else None}
        log(f"per-seed {ps_ms:.1f} ms/step; stream {pst['t_stream_ms']:.1f} ms")

    # degree-class aggregated variant: the same results with the pair sums of
    # centres of degree > 1024 formed per class of equal neighbour degree;
    # clusters are accounted, not enumerated, so its rate is "equivalent"
    agg = None
    if args.algo == "cluster" and args.agg_steps > 0:
        log(f"aggregated variant: {args.agg_steps} steps")
        g.compute(algo="cluster_agg", prec=args.prec, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.agg_steps):
            g.compute(algo="cluster_agg", prec=args.prec, out=out)
        torch.cuda.synchronize()
        agg_ms = 1e3 * (time.perf_counter() - t0) / args.agg_steps
        g.compute(algo="cluster_agg", prec=args.prec, out=out, profile=True)
        ast = g.stats()
        agg = {"algo": "cluster_agg", "ms_per_step": agg_ms,
               "equivalent_clusters_per_s": W / (agg_ms * 1e-3),
               "phases_ms": {k[2:-3]: round(ast[k], 4) for k in ast if k.startswith("t_")}}
        log(f"aggregated variant {agg_ms:.2f} ms/step")

    # whole-step algorithmic HBM bytes: CSR in (row_ptr, col_idx), the triangle
    # pass's walk over up(w) lists (4 B per wedge check), outputs (EF, D, N)
    step_bytes = (4.0 * (n + 1) + 4.0 * info["nnz"] + 4.0 * info["wedge_checks"] + 24.0 * n)
    hbm = {"algorithmic_bytes_per_step": step_bytes,
           "GBps": step_bytes / (ms * 1e-3) / 1e9,
           "frac_hbm_peak": step_bytes / (ms * 1e-3) / 8.0e12}

    batch = None if args.no_batch else bench_batch(max(3, args.steps))
    sur = None if args.no_surrogate else bench_surrogate()
    j3 = None if args.j3_steps <= 0 else bench_j3(args.j3_steps, not args.no_cpu_baseline)
    sir = None if args.sir_runs <= 0 else bench_sir(args.sir_runs, not args.no_cpu_baseline)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        cpu = cpu_baseline(rp, ci, (ef_h, D_h, N_h), args.prec)
        log(f"oracle parity of the benched step on the sample: {cpu['parity']}")

    rec = {
        "metric": METRIC,
        "value": W / (ms * 1e-3),
        "unit": "clusters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32c" else "f64",
        "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}_ef{args.edge_factor}", "nodes": n,
                   "arcs": int(info["nnz"]), "clusters": int(W), "algo": args.algo,
                   "precision": args.prec, "global_batch": 1, "parallelism": "single-gpu"},
        "nodes_per_s": n / (ms * 1e-3),
        "phases_ms": {k[2:-3]: round(st[k], 4) for k in st if k.startswith("t_")},
        "promoted_seeds": int(st["promoted"]),
        "fp64_finalized_seeds": int(st["fp64_finalized"]),
        "ef_checksum": float(np.sum(ef_h)),
        "roofline": roofline,
        "per_seed": per_seed,
        "aggregated": agg,
        "hbm": hbm,
        "batch": batch,
        "surrogate": sur,
        "three_events": j3,
        "sir": sir,
        "cpu_baseline": cpu,
    }
    g.close()
    print(json.dumps(rec))
    if cpu is not None and not cpu["parity"]["ok"]:
        log("the benched step disagrees with the oracle on the sampled seeds")
        sys.exit(1)


if __name__ == "__main__":
    main()
