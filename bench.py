#!/usr/bin/env python3
"""Throughput of one deep-potential MD step (neighbour lists -> E, F, virial) on one MI355X.

A step is one dp_compute_device call on a synthetic protein-in-water-shaped
box with coordinates already resident in HBM: cell-list neighbour search,
environment matrix, type-embedded embedding net, two gated self-attention
layers, descriptor contraction, fitting net, energy reduction, hand-written
backward, force gather and virial.  `value` is atoms evaluated (E and F) per
second of wall clock over the timed steps.

The JSON line also carries the roofline of the dominant kernel (its average
duration from HIP events recorded on the launch stream inside the library),
the same path at the other precision, the force error of the run on sampled
atoms against the FP64 oracle, and the oracle's own throughput on the host
cores (a bounded sample of the same workload).

The GNN-variant model (message passing over edges and angles) is timed on the 40k-atom
chain in both precisions as well, under "gnn", and the repformer-style model (float32)
under "repformer".

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--precision bf16|fp32]
                       [--workload chain25k] [--serve-requests 2000] [--no-cpu-baseline]
                       [--gnn-steps 5]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2.5e15, "fp32": 157.3e12}     # MI355X dense MFMA peaks, FLOP/s
HBM_PEAK = 8.0e12
METRIC = "atom-evals/s (E+F), BF16 vs FP32 path at fixed force RMSE; p50/p99 latency"

# Algorithmic multiply-accumulates per atom-eval with n neighbours, split by kernel.
# Model sizes: embedding 1->25->50->100 (6,275 MAC per neighbour with the type part of
# the first layer folded into a bias), attention M = 100, d = 128, two layers (forward
# 4nMd + 2n^2 d, backward 4nMd + 4n^2 d; input gradients only), contraction T = G^T Rt
# (400 n) and D = T T<^T (6,400), fitting 1600-240-240-240-1 (499,440 each way).
# Sum: 218,550 n + 1,536 n^2 + 1,018,080 MAC.
M_EMB, M_ATT, D_ATT, N_LAYERS = 6275, 100, 128, 2
FIT_MAC = 1600 * 240 + 2 * 240 * 240 + 240


def mac_desc_fwd(n):
    return M_EMB * n + N_LAYERS * (4 * n * M_ATT * D_ATT + 2 * n * n * D_ATT) + 400 * n + 6400


def mac_desc_bwd_alg(n):
    """Backward proper (attention, embedding and contraction backward), no recompute credited."""
    return M_EMB * n + N_LAYERS * (4 * n * M_ATT * D_ATT + 4 * n * n * D_ATT) + 800 * n + 12800


def flop_per_atom_eval(n):
    return 2.0 * (mac_desc_fwd(n) + mac_desc_bwd_alg(n) + 2 * FIT_MAC)


# GNN variant (message passing over edges and angles): algorithmic FLOP of its products
# as the kernels evaluate them, with the terms an angle takes from its two edges formed
# once per angle-list edge (e_x[:32] times Waa[32:96] and Wea[32:64], 2*32*128 per edge)
# and the centre's part of every edge update once per atom (n_i Wee[0:64], 2*64*64).
# Forward, per layer: an angle 2 (32*32 + 32*64), an edge 2 (128*64), an atom 2 (64*64 +
# 128*64); the fitting net and its gradient per atom 2 (64*128 + 128*128 + 128) +
# 2 (128*128 + 64*128).  Backward, per layer: an angle 2 (32*64 + 32*32 + 64*32 + 32*32 +
# 96*32) (recomputed activations, the two transposed products and the terms of edge q),
# an angle-list edge 2*32*128 (recomputed), an edge 2 (128*64 + 2*64*64) (2 (128*64 +
# 64*64) in layer 0, which needs no neighbour part), an atom 2 (64*64 + 128*64 + 2*64*64).
GNN_F = dict(fwd_angle=2 * (32 * 32 + 32 * 64), fwd_aedge=2 * 32 * 128, fwd_edge=2 * 128 * 64,
             fwd_node=2 * (64 * 64 + 128 * 64), fit=2 * (64 * 128 + 128 * 128 + 128) + 2 * (128 * 128 + 64 * 128),
             bwd_angle=2 * (32 * 64 + 32 * 32 + 64 * 32 + 32 * 32 + 96 * 32), bwd_aedge=2 * 32 * 128,
             bwd_edge=2 * (128 * 64 + 2 * 64 * 64), bwd_edge0=2 * (128 * 64 + 64 * 64),
             bwd_node=2 * (64 * 64 + 128 * 64 + 2 * 64 * 64))


def gnn_flop(N, E, C, A):
    """(forward, backward) algorithmic FLOP of one GNN step: N atoms, E edges, C angle-list
    edges, A angles."""
    f = GNN_F
    fwd = 3 * (A * f["fwd_angle"] + C * f["fwd_aedge"] + E * f["fwd_edge"] + N * f["fwd_node"]) + N * f["fit"]
    bwd = 3 * (A * f["bwd_angle"] + C * f["bwd_aedge"] + N * f["bwd_node"]) + E * (2 * f["bwd_edge"] + f["bwd_edge0"])
    return float(fwd), float(bwd)


def gnn_bench(steps, warmup):
    """The GNN-variant model on the 40k-atom chain, both precisions: throughput, phase
    times (HIP events on the launch stream) and the roofline of the backward layer kernel."""
    import torch
    from paper_2602_02234_amd import GnnModel
    from synth import config_system
    from synth.gnn_weights import default_gnn_file
    s = config_system("chain40k")
    dev = torch.device("cuda:0")
    X = torch.tensor(s.coords, device=dev)
    T = torch.tensor(s.types, device=dev)
    F = torch.empty((s.natoms, 3), dtype=torch.float64, device=dev)
    V = torch.empty(9, dtype=torch.float64, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    out = {"workload": f"chain40k: seeded solvated chain, {s.natoms} atoms, periodic cubic {s.box[0, 0]:.2f} A box",
           "model": "GNN variant: 3 layers over edges (rc 6 A, width 64) and angles (rca 4 A, width 32), "
                    "node width 64, fitting 64-128-128-1, seeded random weights", "natoms": s.natoms}
    for prec in ("bf16", "fp32"):
        m = GnnModel(default_gnn_file(), precision=prec)
        for _ in range(warmup):
            m.compute_device(X, T, s.box, forces=F, virial=V, energy=E)
        torch.cuda.synchronize()
        m.profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            m.compute_device(X, T, s.box, forces=F, virial=V, energy=E)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = m.profile_read()
        m.profile(False)
        ne, nce, na = m.graph_size()
        m.close()
        fwd, bwd = gnn_flop(s.natoms, ne, nce, na)
        ph = {k: (ms / c if c else 0.0) for k, (ms, c) in prof.items()}
        per_launch_ms = ph["layers_bwd"] / 3.0
        achieved = (bwd / 3.0) / (per_launch_ms * 1e-3)
        out.update(edges=ne, angle_edges=nce, angles=na)
        out[prec] = {
            "value": s.natoms * steps / dt, "unit": "atom-evals/s", "ms_per_step": 1e3 * dt / steps, "steps": steps,
            "phase_ms": ph,
            "roofline": {"bound": "mfma", "kernel": "k_layer_bwd (three launches per step, one per layer)",
                         "achieved": achieved / 1e12, "peak": PEAK[prec] / 1e12, "unit": "TFLOP/s",
                         "frac": achieved / PEAK[prec], "avg_ms": per_launch_ms, "alg_flop_per_launch": bwd / 3.0,
                         "traffic": measured_traffic("layers_bwd", prec, "chain40k_gnn"),
                         "executed_flop_per_launch": measured_traffic("layers_bwd", prec, "chain40k_gnn",
                                                                      "mfma_flop_per_launch") if prec == "bf16" else None},
            "step_roofline": {"alg_flop_per_step": fwd + bwd, "frac": (fwd + bwd) / (dt / steps) / PEAK[prec]},
        }
        print(f"[bench] GNN chain40k {prec}: {1e3 * dt / steps:.1f} ms/step -> {s.natoms * steps / dt:.4g} "
              f"atom-evals/s; backward layer {per_launch_ms:.2f} ms = {achieved / 1e12:.1f} TFLOP/s",
              file=sys.stderr, flush=True)
    return out


# Repformer-style model: algorithmic FLOP of its products (float32 VALU).  Forward, per
# layer: an edge 2 (96*32 + 3*32*32 + 32*4 + 32) (pair update, projections, contraction,
# convolution), an ordered neighbour pair (j, k) of one centre 2 (32 + 32) (score, A V),
# an atom 2 (32*4*4 + 224*64) (D and the node update); the fitting net and its gradient
# 98,560 per atom.  Backward, per layer: an edge 2 (96*32 + 3*32*32 + 3*32*4 + 2*32), a
# pair 2 (4*32) (dA, dQ, dV, dK), an atom 2 (224*64 + 2*32*4*4).
REP_F = dict(fwd_edge=2 * (96 * 32 + 3 * 32 * 32 + 32 * 4 + 32), fwd_pair=2 * 64, fwd_atom=2 * (32 * 16 + 224 * 64),
             fit=GNN_F["fit"], bwd_edge=2 * (96 * 32 + 3 * 32 * 32 + 3 * 32 * 4 + 2 * 32), bwd_pair=2 * 4 * 32,
             bwd_atom=2 * (224 * 64 + 2 * 32 * 16))
FP32_PEAK = 157.3e12  # MI355X FP32, FLOP/s: dense MFMA and vector ALU have the same peak


def rep_flop(N, E, P):
    """(forward, backward) algorithmic FLOP of one repformer step: N atoms, E edges, P ordered pairs."""
    f = REP_F
    fwd = 3 * (E * f["fwd_edge"] + P * f["fwd_pair"] + N * f["fwd_atom"]) + N * f["fit"]
    bwd = 3 * (E * f["bwd_edge"] + P * f["bwd_pair"] + N * f["bwd_atom"])
    return float(fwd), float(bwd)


def rep_bench(steps, warmup):
    """The repformer-style model on the 40k-atom chain (float32): throughput, phase times
    and the roofline of the backward layer kernel against the FP32 peak (its attention
    products run on MFMA, the rest on the vector ALU; both peak at 157.3 TFLOP/s)."""
    import torch
    from paper_2602_02234_amd import Model, RepModel
    from synth import config_system, default_model_file
    from synth.rep_weights import default_rep_file
    s = config_system("chain40k")
    lm = Model(default_model_file(), precision="fp32")
    _, nnei, _ = lm.neighbors(s.coords, s.box)
    lm.close()
    pairs = float(np.sum(nnei.astype(np.float64) ** 2))
    dev = torch.device("cuda:0")
    X = torch.tensor(s.coords, device=dev)
    T = torch.tensor(s.types, device=dev)
    F = torch.empty((s.natoms, 3), dtype=torch.float64, device=dev)
    V = torch.empty(9, dtype=torch.float64, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    m = RepModel(default_rep_file())
    for _ in range(warmup):
        m.compute_device(X, T, s.box, forces=F, virial=V, energy=E)
    torch.cuda.synchronize()
    m.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        m.compute_device(X, T, s.box, forces=F, virial=V, energy=E)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = m.profile_read()
    m.profile(False)
    ne = m.edges()
    m.close()
    fwd, bwd = rep_flop(s.natoms, ne, pairs)
    ph = {k: (ms / c if c else 0.0) for k, (ms, c) in prof.items()}
    per_launch_ms = ph["layers_bwd"] / 3.0
    achieved = (bwd / 3.0) / (per_launch_ms * 1e-3)
    print(f"[bench] repformer chain40k fp32: {1e3 * dt / steps:.1f} ms/step -> {s.natoms * steps / dt:.4g} "
          f"atom-evals/s; backward layer {per_launch_ms:.2f} ms = {achieved / 1e12:.2f} TFLOP/s",
          file=sys.stderr, flush=True)
    return {
        "workload": f"chain40k: seeded solvated chain, {s.natoms} atoms, periodic cubic {s.box[0, 0]:.2f} A box",
        "model": "repformer-style: 3 layers, node width 64, pair width 32, gated self-attention over neighbours, "
                 "fitting 64-128-128-1, seeded random weights",
        "natoms": s.natoms, "edges": ne, "neighbor_pairs": pairs,
        "fp32": {"value": s.natoms * steps / dt, "unit": "atom-evals/s", "ms_per_step": 1e3 * dt / steps,
                 "steps": steps, "phase_ms": ph,
                 "roofline": {"bound": "mfma", "kernel": "k_rep_bwd (three launches per step, one per layer)",
                              "achieved": achieved / 1e12, "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s",
                              "frac": achieved / FP32_PEAK, "avg_ms": per_launch_ms,
                              "alg_flop_per_launch": bwd / 3.0,
                              "traffic": measured_traffic("layers_bwd", "fp32", "chain40k_rep")},
                 "step_roofline": {"alg_flop_per_step": fwd + bwd,
                                   "frac": (fwd + bwd) / (dt / steps) / FP32_PEAK}},
    }


def _cpu_worker(args):
    """Oracle E_i and dE_i/dDelta_ij for consecutive chunks of 16 centre atoms of one
    worker's share, until the time budget is spent (one BLAS thread per process)."""
    from threadpoolctl import threadpool_limits
    from oracle.dp import evaluate_subset
    m, system, nl, nn, atoms, budget_s = args
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s and done < len(atoms):
            evaluate_subset(m, system.coords, system.types, system.box, atoms[done:done + 16], nl, nn)
            done += 16
        dt = time.perf_counter() - t0
    return done, dt


def cpu_baseline(system, workload, budget_s=10.0):
    """The FP64 oracle on the host cores, on random centre atoms of the benchmark system:
    once in one process with one BLAS thread, once in one process per host core (each with
    one BLAS thread).  Runs before anything touches the GPU (it forks)."""
    import multiprocessing as mp
    import platform
    from threadpoolctl import threadpool_info
    from synth import default_model_file
    from oracle import load_model
    from oracle.neighbors import neighbor_list_cells
    m = load_model(default_model_file())
    nl, nn, _ = neighbor_list_cells(system.coords, system.box, m.rc, m.sel)
    order = np.random.default_rng(0).permutation(system.natoms)
    one, dt1 = _cpu_worker((m, system, nl, nn, order, budget_s))
    cores = max(1, min(len(os.sched_getaffinity(0)), 64))
    shares = np.array_split(order, cores)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_cpu_worker, [(m, system, nl, nn, sh, budget_s) for sh in shares], chunksize=1)
    wall = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    cpu_model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next(ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name"))
    except (OSError, StopIteration):
        pass
    blas = [f"{d.get('internal_api')} {d.get('version')}" for d in threadpool_info() if d.get("user_api") == "blas"]
    return {"value": done / wall, "unit": "atom-evals/s", "cores": cores, "kind": "oracle",
            "sample": f"random centre atoms of the {system.natoms:,}-atom {workload} box: E_i and dE_i/dDelta_ij "
                      f"in float64 NumPy, {cores} processes x 1 BLAS thread, each on its share of the atoms for "
                      f"up to {budget_s:.0f} s ({done} atoms in {wall:.1f} s wall); neighbour search excluded",
            "single_thread": {"value": one / dt1, "cores": 1, "atoms": one, "seconds": dt1},
            "cpu_model": cpu_model, "blas": blas, "host_cores_visible": len(os.sched_getaffinity(0))}


def sampled_force_error(model_path, system, F, k=6, seed=1):
    """Force RMSE / max of the GPU forces on k random atoms against the oracle (local evaluation)."""
    from oracle import load_model
    from oracle.dp import evaluate_subset
    from oracle.neighbors import neighbor_list_cells
    m = load_model(model_path)
    nl, nn, _ = neighbor_list_cells(system.coords, system.box, m.rc, m.sel)
    atoms = np.random.default_rng(seed).choice(system.natoms, size=k, replace=False)
    errs = []
    for i in atoms:
        centres = [int(i)] + nl[i, :nn[i]].tolist()
        _, nbrs, gs, _ = evaluate_subset(m, system.coords, system.types, system.box, centres, nl, nn)
        f = gs[0].sum(0)
        for c, js, g in zip(centres[1:], nbrs[1:], gs[1:]):
            f -= g[np.nonzero(js == i)[0][0]]
        errs.append(F[i] - f)
    e = np.array(errs)
    return float(np.sqrt(np.mean(e ** 2))), float(np.max(np.abs(e)))


def _make_request(r):
    from synth import request_system
    s = request_system(r["natoms"], r["kind"], r["seed"])
    return s.coords, s.types, s.box


def _pct(v, p):
    """Nearest-rank percentile."""
    v = np.sort(np.asarray(v))
    k = min(max(int(np.ceil(p * len(v))), 1), len(v))
    return float(v[k - 1])


def make_trace(n_req, workers):
    """The first n_req requests of the serving trace, generated on host worker processes
    (called before anything touches the GPU)."""
    import multiprocessing as mp
    from synth import serving_trace
    trace = serving_trace(n_req)
    with mp.get_context("fork").Pool(workers) as pool:
        systems = pool.map(_make_request, trace, chunksize=1)
    return trace, systems


def serving_bench(model_path, trace_all, systems_all, legs, budget_bytes, max_inflight=3):
    """The Poisson request trace (sizes log-uniform 192..40,000 atoms, water boxes or solvated
    chains) replayed in real time against the BF16 continuous-batching server and against the
    FP32 path evaluating one request at a time (host API).  legs: (arrival rate, number of
    requests from the start of the trace); the trace's arrival times are scaled to the rate."""
    import time as _t
    from paper_2602_02234_amd import Model, Server
    out = {"hbm_budget_GB": budget_bytes / 2**30, "max_inflight": max_inflight, "rates": {}}
    for rate, n_req in legs:
        trace, systems = trace_all[:n_req], systems_all[:n_req]
        atoms = np.array([len(t) for _, t, _ in systems])
        base_t = np.array([r["t"] for r in trace])
        arr = base_t * (200.0 / rate)
        row = {"requests": len(trace), "atoms_total": int(atoms.sum()), "atoms_median": float(np.median(atoms)),
               "trace_seconds": float(arr[-1])}
        # BF16 server, continuous batching
        m = Model(model_path, "bf16")
        srv = Server(m, budget_bytes, max_inflight)
        srv.wait(srv.submit(*systems[0]), 120.0)
        srv.close()
        srv = Server(m, budget_bytes, max_inflight)
        t0 = _t.perf_counter()
        ids = []
        for a, sysk in zip(arr, systems):
            d = t0 + a - _t.perf_counter()
            if d > 0:
                _t.sleep(d)
            ids.append(srv.submit(*sysk))
        lat = [srv.wait(i, 600.0)["latency"] for i in ids]
        st = srv.stats()
        srv.close()
        m.close()
        row["bf16_server"] = {"p50_ms": 1e3 * _pct(lat, 0.5), "p99_ms": 1e3 * _pct(lat, 0.99),
                              "atom_evals_per_s": st["atom_evals_per_s"], "batches": st["batches"],
                              "max_batch_atoms": st["max_batch_atoms"]}
        # FP32, one request at a time in arrival order
        m = Model(model_path, "fp32")
        m.compute(*systems[0])
        t0 = _t.perf_counter()
        lat, last = [], 0.0
        for a, sysk in zip(arr, systems):
            d = t0 + a - _t.perf_counter()
            if d > 0:
                _t.sleep(d)
            m.compute(*sysk)
            last = _t.perf_counter() - t0
            lat.append(last - a)
        m.close()
        row["fp32_one_at_a_time"] = {"p50_ms": 1e3 * _pct(lat, 0.5), "p99_ms": 1e3 * _pct(lat, 0.99),
                                     "atom_evals_per_s": float(atoms.sum() / (last - arr[0]))}
        out["rates"][f"{rate:g}_req_per_s"] = row
        print(f"[bench] serving at {rate:g} req/s: bf16 server p50 {row['bf16_server']['p50_ms']:.1f} ms, "
              f"p99 {row['bf16_server']['p99_ms']:.1f} ms; fp32 one-at-a-time p50 "
              f"{row['fp32_one_at_a_time']['p50_ms']:.1f} ms, p99 {row['fp32_one_at_a_time']['p99_ms']:.1f} ms",
              file=sys.stderr, flush=True)
    return out


def measured_traffic(phase, precision, workload, key="hbm_bytes_per_launch"):
    """HBM bytes per launch of a phase from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's reading), or None when there
    is none for this phase and workload or a kernel source changed since it was taken.
    key = "mfma_flop_per_launch": the executed MFMA FLOP from the same summary instead."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get("phases", {}).get(phase)
    if rec is None:
        return None
    csrc = os.path.join(ROOT, "paper_2602_02234_amd", "csrc")
    if not isinstance(rec.get("sources"), dict) or key not in rec:
        return None
    for name, digest in rec["sources"].items():
        if not os.path.exists(os.path.join(csrc, name)):
            return None
        with open(os.path.join(csrc, name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return rec[key]


def time_path(model, X, T, box, F, V, E, steps, warmup):
    import torch
    for _ in range(warmup):
        model.compute_device(X, T, box, forces=F, virial=V, energy=E)
    torch.cuda.synchronize()
    model.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        model.compute_device(X, T, box, forces=F, virial=V, energy=E)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = model.profile_read()
    model.profile(False)
    return dt, prof


def time_graph_replays(model, X, T, box, F, V, E, replays=20):
    """Warm replays of the step's HIP graph: device time of each replay (HIP events on the
    stream the graph runs on) and host wall-clock per call (launch, status read-back)."""
    import torch
    model.set_graph(True)
    st = torch.cuda.current_stream()
    for _ in range(3):
        model.compute_device(X, T, box, forces=F, virial=V, energy=E)
    torch.cuda.synchronize()
    dev_ms, host_ms = [], []
    for _ in range(replays):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        a.record(st)
        model.compute_device(X, T, box, forces=F, virial=V, energy=E)
        b.record(st)
        b.synchronize()
        host_ms.append(1e3 * (time.perf_counter() - t0))
        dev_ms.append(a.elapsed_time(b))
    model.set_graph(False)
    return {"replays": replays, "median_device_ms": float(np.median(dev_ms)),
            "median_host_ms": float(np.median(host_ms)), "min_device_ms": float(np.min(dev_ms))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32"])
    ap.add_argument("--workload", default="chain25k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the other-precision run")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the serving trace replayed at 200 req/s (0 = skip the serving run); "
                         "the first quarter of them is also replayed at 20 req/s")
    ap.add_argument("--gnn-steps", type=int, default=5,
                    help="steps of the GNN-variant model (per precision) and of the repformer-style model on the "
                         "40k-atom chain (0 = skip both)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 512 MiB device-to-device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    from synth import config_system, default_model_file
    system = None if args.copy_probe else config_system(args.workload)
    # host-side work that forks (the oracle baseline, the serving trace) runs before anything
    # touches the GPU
    cpu = None
    if not args.no_cpu_baseline and not args.copy_probe:
        t0 = time.perf_counter()
        cpu = cpu_baseline(system, args.workload)
        print(f"[bench] oracle on {cpu['cores']} host cores: {cpu['value']:.4g} atom-evals/s "
              f"(1 thread: {cpu['single_thread']['value']:.4g}) in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    trace = systems_trace = None
    if args.serve_requests > 0 and not args.copy_probe:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
        t0 = time.perf_counter()
        trace, systems_trace = make_trace(args.serve_requests, workers)
        print(f"[bench] generated {len(trace)} serving requests in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    import torch
    from paper_2602_02234_amd import Model

    dev = torch.device("cuda:0")
    if args.copy_probe:
        src = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": src.numel() * 4, "copy_probe_bytes_written": dst.numel() * 4}))
        return
    N = system.natoms
    path = default_model_file()
    X = torch.tensor(system.coords, dtype=torch.float64, device=dev).contiguous()
    T = torch.tensor(system.types, dtype=torch.int32, device=dev).contiguous()
    F = torch.empty((N, 3), dtype=torch.float64, device=dev)
    V = torch.empty(9, dtype=torch.float64, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    box = system.box

    results = {}
    precs = [args.precision] + ([] if args.no_compare else [p for p in ("bf16", "fp32") if p != args.precision])
    nnei = None
    for prec in precs:
        model = Model(path, precision=prec)
        if nnei is None:
            _, nnei, _ = model.neighbors(system.coords, box)
        steps = args.steps if prec == args.precision else max(3, args.steps // 4)
        dt, prof = time_path(model, X, T, box, F, V, E, steps, args.warmup)
        f_rmse, f_max = sampled_force_error(path, system, F.cpu().numpy())
        graph = time_graph_replays(model, X, T, box, F, V, E) if prec == args.precision else None
        results[prec] = dict(dt=dt, steps=steps, prof=prof, f_rmse=f_rmse, f_max=f_max, E=float(E.item()),
                             graph=graph)
        print(f"[bench] {prec}: {steps} steps in {dt:.3f} s -> {N * steps / dt:.4g} atom-evals/s; "
              f"sampled force RMSE {f_rmse:.2e}" + (f"; graph replay median {graph['median_device_ms']:.3f} ms"
                                                     if graph else ""), file=sys.stderr, flush=True)
        model.close()

    r = results[args.precision]
    value = N * r["steps"] / r["dt"]
    n = nnei.astype(np.float64)
    alg = {
        "descriptor_fwd": 2.0 * float(np.sum(mac_desc_fwd(n))),
        "fitting": 2.0 * N * 2 * FIT_MAC,
        "descriptor_bwd": 2.0 * float(np.sum(mac_desc_bwd_alg(n))),
    }
    prof = r["prof"]
    avg = {k: (ms / c if c else 0.0) for k, (ms, c) in prof.items()}
    dom = max(("descriptor_fwd", "fitting", "descriptor_bwd"), key=lambda k: avg[k])
    achieved = alg[dom] / (avg[dom] * 1e-3)
    step_alg = sum(alg.values())
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-evals/s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r["dt"] / r["steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: seeded solvated chain, {N} atoms, periodic cubic "
                               f"{system.box[0, 0]:.2f} A box, rc 6 A, sel 120; energy+forces+virial per step",
                   "precision_path": args.precision, "natoms": N, "mean_neighbors": float(n.mean())},
        "roofline": {"bound": "mfma", "kernel": dom, "achieved": achieved / 1e12, "peak": PEAK[args.precision] / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK[args.precision],
                     "traffic": measured_traffic(dom, args.precision, args.workload),
                     "avg_ms": avg[dom], "alg_flop_per_launch": alg[dom],
                     "executed_flop_per_launch": measured_traffic(dom, args.precision, args.workload,
                                                                  "mfma_flop_per_launch")},
        "step_roofline": {"alg_flop_per_step": step_alg,
                          "frac": step_alg / (r["dt"] / r["steps"]) / PEAK[args.precision]},
        "phase_ms": avg,
        "graph_replay": r["graph"],
        "accuracy": {"force_rmse_sampled": r["f_rmse"], "force_max_sampled": r["f_max"], "unit": "eV/A"},
    }
    for prec in precs[1:]:
        o = results[prec]
        out[f"{prec}_value"] = N * o["steps"] / o["dt"]
        out[f"{prec}_ms_per_step"] = 1e3 * o["dt"] / o["steps"]
        out[f"{prec}_force_rmse_sampled"] = o["f_rmse"]
        out[f"{prec}_phase_ms"] = {k: (ms / c if c else 0.0) for k, (ms, c) in o["prof"].items()}
    if trace is not None:
        legs = [(200.0, len(trace)), (20.0, max(1, len(trace) // 4))]
        out["serving"] = serving_bench(path, trace, systems_trace, legs, 16 << 30)
        r200 = out["serving"]["rates"]["200_req_per_s"]["bf16_server"]
        out["latency_p50_ms"], out["latency_p99_ms"] = r200["p50_ms"], r200["p99_ms"]
    if args.gnn_steps > 0:
        out["gnn"] = gnn_bench(args.gnn_steps, 1)
        out["repformer"] = rep_bench(args.gnn_steps, 1)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
