"""Benchmark of the mortar coupling hot path on one MI355X.

One step = the whole path on one synthetic interface with inputs resident in
HBM: contact search and clipping (mt_build_pairs), CSR pattern
(mt_csr_pattern), segment-based integration and assembly of D, M and the
weighted gap (mt_integrate), and the backward pass for keyed N(0,1) upstream
weights (mt_backward).  Workload: the wavy interface z = 0.05 sin(2 pi x)
sin(2 pi y), slave 1024x1024 / master 777x777 quad4, master nodes offset
along the normal by U[-1e-3, 1e-3], delta = 1.25e-3.

Prints one JSON line: value = pairs / (wall time of one step), plus the
roofline of the dominant kernel (from the library's HIP events around that
kernel in the timed steps; the per-phase breakdown comes from a separate
instrumented pass of the same number of steps) and the CPU oracle timed on
a bounded sample.  Extra
objects: the same step with the dual basis, element-based integration of the
same interface (n x n Gauss points per slave element, for several n: time
and difference from the segment-based values), the same step with auxiliary
planes from the continuous nodal normal field, and 64 batched interfaces.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0
# Adjoint of one inverse bilinear map by the implicit-function theorem:
# Jacobian at the solution (8), transposed 2x2 solve (12), node adjoints (16),
# point adjoint (2).
IFT_FLOPS = 38
# Gauss points per direction of the element-based integration variants
ELEM_RULES = (2, 4, 8)

# Library phase timer of a single-kernel phase -> (kernel, source files whose
# hash identifies the kernel version, committed traffic summary).
KERNELS = {
    "pair_poly": ("k_pair_poly", ["mt_pairs.hip", "mt_pair_eval.h", "mt_geometry.h"],
                  "profiles/k_pair_poly_wavy1024_traffic.md"),
    "pair_fwd": ("k_pair_fwd", ["mt_pairs.hip", "mt_pair_eval.h", "mt_geometry.h"],
                 "profiles/k_pair_fwd_wavy1024_traffic.md"),
    "pair_bwd": ("k_pair_bwd", ["mt_backward.hip", "mt_dual.h", "mt_pair_eval.h", "mt_geometry.h"],
                 "profiles/k_pair_bwd_wavy1024_traffic.md"),
}


def kernel_source_hash(files):
    """Hash of the sources that make a kernel: whole files, or (file, marker)
    for the part of a file before the line that starts with marker (the
    device code of a file whose host code follows it)."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        name, marker = f if isinstance(f, tuple) else (f, None)
        with open(os.path.join(ROOT, "paper_2202_03933_amd", "csrc", name), "rb") as fh:
            text = fh.read()
        if marker is not None:
            at = text.find(b"\n" + marker.encode())
            if at < 0:
                raise RuntimeError(f"{name}: no line starting with {marker!r}")
            text = text[:at + 1]
        h.update(text)
    return h.hexdigest()[:16]


def recorded_traffic(kernel):
    """HBM bytes per launch recorded by a committed rocprofv3 --pmc summary,
    or None when the summary is missing or the kernel sources changed since."""
    _, files, path = KERNELS[kernel]
    full = os.path.join(ROOT, path)
    if not os.path.exists(full):
        return None
    rec = {}
    with open(full) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                rec[k.strip()] = v.strip().strip("`")
    if rec.get("source_hash") != kernel_source_hash(files):
        return None
    try:
        return float(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


_SHARD_ITF = None  # the workload, inherited by the forked oracle workers


def _oracle_shard(rows):
    """The oracle (serial C++, one core) on the slave elements of grid rows
    [r0, r1) against the whole master side: search, clip, integration,
    assembly and forward-mode gradients.  Returns (pairs, fwd s, all s)."""
    import numpy as np

    import oracle
    import synth
    from synth.weights import keyed_normal, TAG_D, TAG_M, TAG_G

    r0, r1, seed = rows
    itf = _SHARD_ITF
    nx = int(round(itf.slave.n_el ** 0.5))
    sub = synth.Mesh(itf.slave.X, itf.slave.conn[r0 * nx:r1 * nx].copy())
    prm = oracle.params(delta=itf.delta)
    oracle._lib()  # load outside the timed region
    t0 = time.perf_counter()
    cs, cm = oracle.search(sub, itf.master, itf.delta)
    nv, blocks, _ = oracle.eval_candidates(sub, itf.master, prm, cs, cm, integrate=True)
    keep = nv >= 3
    ps, pm = cs[keep], cm[keep]
    oracle.assemble(sub, itf.master, ps, pm, blocks[keep])
    t_fwd = time.perf_counter() - t0
    fD = lambda r, c: keyed_normal(seed, TAG_D, r, c)  # noqa: E731
    fM = lambda r, c: keyed_normal(seed, TAG_M, r, c)  # noqa: E731
    fg = lambda r: keyed_normal(seed, TAG_G, r, np.zeros_like(r))  # noqa: E731
    w = oracle.pair_weights(sub, itf.master, ps, pm, fD, fM, fg)
    g24, _ = oracle.pair_grads(sub, itf.master, prm, ps, pm, w)
    oracle.scatter_grads(sub, itf.master, ps, pm, g24)
    return int(ps.size), t_fwd, time.perf_counter() - t0


def host_cores():
    """Host threads the oracle legs use: the CPUs this process may run on,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(itf, rows=16, seed=3000):
    """Oracle timings on the host, run before the GPU is touched: one core
    on grid rows [0, rows), and all host cores (forked worker processes, one
    contiguous block of `rows` slave-element rows each, rows [0, cores x
    rows)) -- the embarrassingly sharded oracle.  Pairs/s over the wall time
    of each leg."""
    import multiprocessing as mp

    global _SHARD_ITF
    _SHARD_ITF = itf
    p1, f1, a1 = _oracle_shard((0, rows, seed))
    n = host_cores()
    with mp.get_context("fork").Pool(n) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_shard, [(k * rows, (k + 1) * rows, seed) for k in range(n)], chunksize=1)
        wall = time.perf_counter() - t0
    pn = sum(r[0] for r in res)
    return {"one_core": {"pairs": p1, "t_fwd": f1, "t_all": a1, "rows": rows},
            "all_cores": {"pairs": pn, "wall": wall, "cores": n, "rows": n * rows,
                          "worker_fwd_s_max": max(r[1] for r in res), "worker_all_s_max": max(r[2] for r in res)}}


def oracle_flop_model(itf, n_slave_el_sample=16384):
    """The oracle's operation counts per unit (its flop-counting scalar on
    every 16th pair of the first rows of the workload): the algorithmic-work
    model, reported beside the executed FP64 instruction counts."""
    import numpy as np

    import oracle
    import synth

    sub = synth.Mesh(itf.slave.X, itf.slave.conn[:n_slave_el_sample].copy())
    prm = oracle.params(delta=itf.delta)
    cs, cm = oracle.search(sub, itf.master, itf.delta)
    nv, _, _ = oracle.eval_candidates(sub, itf.master, prm, cs, cm, integrate=False)
    keep = nv >= 3
    ps, pm = cs[keep], cm[keep]
    #   k_pair_poly:  the candidate pass of every pair;
    #   k_pair_fwd:   the pair evaluation minus its candidate pass;
    #   k_pair_bwd:   that forward recompute + the reverse-mode adjoint of the
    #     pair evaluation minus that of its candidate pass (cost model: adjoint
    #     of add/sub 2, mul 4, div 4, sqrt 3) + IFT_FLOPS per inverse map.
    f_cp, f_pair, f_adj, n_inv, f_cadj = oracle.count_flops(sub, itf.master, prm, ps[::16], pm[::16], detail=True)
    npp = max(1, ps[::16].size)
    esel = ps < 2048
    n_e = max(1, np.unique(ps[esel]).size)
    elem_flops = {ng: oracle.count_flops_elements(sub, itf.master, prm, ps[esel], pm[esel], ng) / n_e
                  for ng in ELEM_RULES}
    return {"pair_poly": f_cp / npp, "pair_fwd": (f_pair - f_cp) / npp,
            "pair_bwd": (f_pair - f_cp + f_adj - f_cadj + IFT_FLOPS * n_inv) / npp,
            "elem_flops_per_element": elem_flops}


def bench_batched(reps=5):
    """64 interfaces of uneven size (log-uniform 16^2..512^2 slave quads,
    master/slave resolution ratio U[0.7, 1.3], flat / cylinder / wavy):
    one persistent graph-launched forward (and backward) over all of them
    versus one mt_integrate (mt_backward) call per interface on one stream."""
    import numpy as np
    import torch

    import synth
    from paper_2202_03933_amd import MortarBatch, MortarInterface, default_params
    from synth.weights import keyed_normal, TAG_D, TAG_M, TAG_G

    dev = torch.device("cuda", 0)
    ifaces, W = [], []
    insts = synth.batched_instances(64)
    for itf in insts:
        it = MortarInterface(torch.from_numpy(itf.slave.X), torch.from_numpy(itf.slave.conn),
                             torch.from_numpy(itf.master.X), torch.from_numpy(itf.master.conn),
                             params=default_params(delta=itf.delta), device=dev).setup()
        ns = it.n_slave_nodes
        Dr = np.repeat(np.arange(ns), np.diff(it.D_rowptr.cpu().numpy()))
        Mr = np.repeat(np.arange(ns), np.diff(it.M_rowptr.cpu().numpy()))
        W.append((torch.from_numpy(keyed_normal(3000, TAG_D, Dr, it.D_col.cpu().numpy())).to(dev),
                  torch.from_numpy(keyed_normal(3000, TAG_M, Mr, it.M_col.cpu().numpy())).to(dev),
                  torch.from_numpy(keyed_normal(3000, TAG_G, np.arange(ns), np.zeros(ns, np.int64))).to(dev)))
        ifaces.append(it)
    pairs = sum(it.n_pairs for it in ifaces)
    b = MortarBatch(ifaces)
    tuning = b.autotune()
    outs = b.alloc_outputs()
    gouts = [(torch.empty(3, it.n_slave_nodes, dtype=torch.float64, device=dev),
              torch.empty(3, it.n_master_nodes, dtype=torch.float64, device=dev)) for it in ifaces]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    def per_fwd():
        for it, o in zip(ifaces, outs):
            it.integrate(o)

    def per_bwd():
        for it, w, g in zip(ifaces, W, gouts):
            it.backward(*w, out=g)

    res = {"n_interfaces": len(ifaces), "pairs": pairs, "tuning": tuning,
           "pairs_by_geometry": {g: sum(it.n_pairs for it, itf in zip(ifaces, insts) if itf.meta["geometry"] == g)
                                 for g in ("flat", "cylinder", "wavy")},
           "fwd_ms_batched_graph": timed(lambda: b.forward(outs, use_graph=True)),
           "fwd_ms_per_interface": timed(per_fwd),
           "bwd_ms_batched_graph": timed(lambda: b.backward(W, outs=gouts, use_graph=True)),
           "bwd_ms_per_interface": timed(per_bwd)}
    # the search and pattern of every interface: one mt_build_pairs +
    # mt_csr_pattern per interface (with and without the count read-backs)
    # versus one mt_batch_search (the instances on four internal streams)

    def per_search_sync():
        for it in ifaces:
            it.build_pairs()
            it.csr_pattern()

    def per_search_nowait():
        for it in ifaces:
            it.build_pairs(sync=False)
            it.csr_pattern(sync=False)

    res["search_ms_per_interface_sync"] = timed(per_search_sync)
    res["search_ms_per_interface_nowait"] = timed(per_search_nowait)
    res["search_ms_batched"] = timed(lambda: b.search(rebuild=False))
    # the same call captured into a HIP graph once (in the warm-up call) and
    # replayed
    res["search_ms_batched_graph"] = timed(lambda: b.search(use_graph=True, rebuild=False))
    b.search(rebuild=True)  # counts read back, batch built again for them
    assert sum(it.n_pairs for it in ifaces) == pairs
    res["search_speedup_vs_per_interface_sync"] = res["search_ms_per_interface_sync"] / res["search_ms_batched"]
    res["search_speedup_graph_vs_per_interface_sync"] = (res["search_ms_per_interface_sync"]
                                                         / res["search_ms_batched_graph"])
    res["search_pairs_per_s_batched"] = pairs / (res["search_ms_batched"] * 1e-3)
    res["search_pairs_per_s_batched_graph"] = pairs / (res["search_ms_batched_graph"] * 1e-3)
    ab = {"forward": 0, "backward": 0, "search": 0}
    for it, itf in zip(ifaces, insts):
        a = algorithmic_bytes(itf.slave.n_nodes, itf.master.n_nodes, itf.slave.n_el, itf.master.n_el, it.n_cand,
                              it.n_pairs, it.nnz_D, it.nnz_M)
        ab["forward"] += a["forward"]
        ab["backward"] += a["backward"]
        ab["search"] += a["search"] + a["pattern"]
    counters = recorded_counters(FP64_SUMMARY)
    res["hbm"] = {}
    for k, phase, kern in (("fwd", "forward", "k_batch_fwd"), ("bwd", "backward", "k_batch_bwd")):
        res[f"{k}_pairs_per_s_batched"] = pairs / (res[f"{k}_ms_batched_graph"] * 1e-3)
        res[f"{k}_pairs_per_s_per_interface"] = pairs / (res[f"{k}_ms_per_interface"] * 1e-3)
        res[f"{k}_speedup"] = res[f"{k}_ms_per_interface"] / res[f"{k}_ms_batched_graph"]
        for mode in ("batched_graph", "per_interface"):
            res["hbm"][f"{k}_{mode}"] = hbm_entry(ab[phase], res[f"{k}_ms_{mode}"])
            fl = counters.get(f"{kern}.fp64_flops_per_launch") if counters else None
            # executed FP64 flops of the batched launch (the same pair arithmetic
            # as the per-interface kernels) over each mode's wall time
            res[f"{k}_fp64_frac_{mode}"] = (fl / (res[f"{k}_ms_{mode}"] * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS
                                            if fl else None)
    for mode in ("batched", "batched_graph", "per_interface_sync"):
        res["hbm"][f"search_{mode}"] = hbm_entry(ab["search"], res[f"search_ms_{mode}"])
    return res


def bench_elements(itf, seg_outs, steps, warmup):
    """Element-based integration (an n x n Gauss rule on each slave element,
    no clipping) on the same interface for the rules in ELEM_RULES: time of
    the forward integration and assembly, and the relative Frobenius
    difference of D, M and the gap from the segment-based values."""
    import numpy as np
    import torch
    from paper_2202_03933_amd import MortarInterface, default_params
    dev = torch.device("cuda", 0)
    out = {}
    for ng in ELEM_RULES:
        it = MortarInterface(torch.from_numpy(itf.slave.X), torch.from_numpy(itf.slave.conn),
                             torch.from_numpy(itf.master.X), torch.from_numpy(itf.master.conn),
                             params=default_params(delta=itf.delta, element_rule=ng), device=dev)
        it.setup()
        outs = it.alloc_outputs()
        for _ in range(warmup):
            it.integrate(outs)
        torch.cuda.synchronize()
        it.timings(reset=True)
        it.set_timing(True)
        for _ in range(steps):
            it.integrate(outs)
        torch.cuda.synchronize()
        it.set_timing(False)
        tim = it.timings(reset=True)
        t0 = time.perf_counter()  # wall time without events
        for _ in range(steps):
            it.integrate(outs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        n_pairs = it.n_pairs
        n_el = int(np.unique(it.pairs()[0].cpu().numpy()).size)
        err = {}
        for name, a, b in zip(("D", "M", "g"), outs, seg_outs):
            assert a.shape == b.shape
            err[name] = (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item()
        it.close()
        ms = (t1 - t0) * 1e3 / steps
        out[str(ng)] = {"integrate_ms": ms, "pairs_per_s": n_pairs / (ms * 1e-3), "slave_elements": n_el,
                        "n_pairs": n_pairs,
                        "k_elem_fwd_ms": tim["pair_fwd"][0] / max(1, tim["pair_fwd"][1]),
                        "assemble_ms": tim["assemble"][0] / max(1, tim["assemble"][1]),
                        "rel_diff_vs_segment": err}
    return out


def bench_variant(itf, weights, steps, warmup, sync=True, **params):
    """The same step with other parameters: the dual Lagrange multiplier basis
    (dual-basis forward and backward, the backward including the adjoint of
    the dual coefficients), auxiliary planes from the continuous nodal
    normal field (its normals computed in every search, its gradient chain in
    every backward), or every kernel on the caller's stream (single_stream:
    no phase runs beside another, so the phase times are those of each phase
    alone).  sync=False: no count read-backs in the step."""
    import torch
    from paper_2202_03933_amd import MortarInterface, default_params
    dev = torch.device("cuda", 0)
    it = MortarInterface(torch.from_numpy(itf.slave.X), torch.from_numpy(itf.slave.conn),
                         torch.from_numpy(itf.master.X), torch.from_numpy(itf.master.conn),
                         params=default_params(delta=itf.delta, **params), device=dev)
    it.setup()
    outs = it.alloc_outputs()
    grads = (torch.empty(3, itf.slave.n_nodes, dtype=torch.float64, device=dev),
             torch.empty(3, itf.master.n_nodes, dtype=torch.float64, device=dev))

    def step():
        it.build_pairs(sync=sync)
        it.csr_pattern(sync=sync)
        it.integrate(outs)
        it.backward(*weights, grads)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    it.timings(reset=True)
    it.set_timing(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    it.set_timing(False)
    tim = it.timings(reset=True)
    t0 = time.perf_counter()  # wall time without events
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_pairs = it.stats()["n_pairs"]  # (read back: the no-wait step leaves the host counts unset)
    it.close()
    ms = (t1 - t0) * 1e3 / steps
    return {"ms_per_step": ms, "pairs_per_s": n_pairs / (ms * 1e-3), "n_pairs": n_pairs,
            "phase_ms_per_step": {k: v[0] / steps for k, v in tim.items()}}


def recorded_counters(name):
    """Executed-instruction counts recorded by a committed rocprofv3 --pmc
    summary (profiles/<name>): entries `<kernel>.<quantity>`, each kernel's
    valid only while the hash of its source files equals the recorded
    `<kernel>.source_hash` (else the kernel changed since the counters were
    taken and its entries are dropped).  None when the summary is missing."""
    full = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(full):
        return None
    rec = {}
    with open(full) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                rec[k.strip()] = v.strip().strip("`")
    out = {}
    for k, v in rec.items():
        kern, _, q = k.rpartition(".")
        if q == "source_hash" or kern not in COUNTER_SOURCES:
            continue
        if rec.get(f"{kern}.source_hash") != kernel_source_hash(COUNTER_SOURCES[kern]):
            continue
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


ALL_SOURCES = ["mt_prims.hip", "mt_search.hip", "mt_pairs.hip", "mt_assemble.hip", "mt_backward.hip",
               "mt_elements.hip", "mt_normals.hip", "mt_batch.hip", "mt_api.hip", "mt_geometry.h",
               "mt_pair_eval.h", "mt_dual.h", "mt_rows.h", "mt_internal.h"]
FP64_SUMMARY = "wavy1024_fp64_counters.md"  # executed FP64 VALU instructions of every kernel of the step
# mt_batch.hip holds its kernels first and the host code that drives them after
# this line; the batched kernels are identified by the part before it
BATCH_HOST = "struct mt_batch {"
# source files whose hash identifies each counted kernel ("step": the whole library)
COUNTER_SOURCES = {
    "k_pair_fwd": ["mt_pairs.hip", "mt_pair_eval.h", "mt_geometry.h"],
    "k_pair_bwd": ["mt_backward.hip", "mt_dual.h", "mt_pair_eval.h", "mt_geometry.h"],
    "k_batch_fwd": [("mt_batch.hip", BATCH_HOST), "mt_dual.h", "mt_rows.h", "mt_pair_eval.h", "mt_geometry.h"],
    "k_batch_bwd": [("mt_batch.hip", BATCH_HOST), "mt_dual.h", "mt_rows.h", "mt_pair_eval.h", "mt_geometry.h"],
    "step": ALL_SOURCES,
}


def algorithmic_bytes(n_sn, n_mn, n_se, n_me, n_cand, n_pairs, nnz_D, nnz_M):
    """Algorithmic HBM bytes of each phase: what the method must move, not
    what the kernels' staging adds.
      search:   nodes once (24 B/node), connectivity once (16 B/element), the
                master bin sort (4 passes, key+value read and written, 16 B
                per master per pass), candidate list written and read
                (2 x 8 B per candidate), pair list written (8 B per pair);
      pattern:  pair list (8 B) and each pair's master connectivity (16 B)
                read, slave connectivity (16 B/element) read, CSR column
                indices (4 B/nonzero) and row pointers (2 x 4 B/row) written;
      forward:  nodes, connectivity and pair list read, CSR indices read, D, M
                and gap values written (8 B each);
      backward: nodes, connectivity, pair list and CSR indices read, the
                upstream weights read (8 B per value), gradients written
                (24 B/node)."""
    nodes = 24 * (n_sn + n_mn)
    conn = 16 * (n_se + n_me)
    csr_idx = 4 * (nnz_D + nnz_M) + 8 * (n_sn + 1)
    vals = 8 * (nnz_D + nnz_M + n_sn)
    search = nodes + conn + 4 * 16 * n_me + 16 * n_cand + 8 * n_pairs
    pattern = 8 * n_pairs + 16 * n_pairs + 16 * n_se + csr_idx
    fwd = nodes + conn + 8 * n_pairs + csr_idx + vals
    bwd = nodes + conn + 8 * n_pairs + csr_idx + vals + 24 * (n_sn + n_mn)
    return {"search": search, "pattern": pattern, "forward": fwd, "backward": bwd,
            "step": search + pattern + fwd + bwd, "forward_path": search + pattern + fwd}


def hbm_entry(nbytes, ms):
    if not ms:
        return None
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"bytes": int(nbytes), "ms": ms, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-dual", action="store_true")
    ap.add_argument("--no-nodal", action="store_true")
    ap.add_argument("--no-elements", action="store_true")
    ap.add_argument("--no-single-stream", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (calibrates HBM traffic counters)")
    ap.add_argument("--cpu-rows", type=int, default=16,
                    help="slave-grid rows per oracle worker in the CPU legs (1024 slave elements a row)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the mortar path on a single MI355X; "
              "sharding over several GPUs is a design note, not a measured mode", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import synth
    itf = synth.interface_config(2)
    # the CPU legs run before anything touches the GPU (their workers are
    # forked processes)
    cpu = model = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(itf, args.cpu_rows)
        model = oracle_flop_model(itf)

    import torch
    from paper_2202_03933_amd import MortarInterface, default_params
    from synth.weights import keyed_normal, TAG_D, TAG_M, TAG_G

    dev = torch.device("cuda", 0)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(dev)[0]
    Xs = torch.from_numpy(itf.slave.X).to(dev)
    Xm = torch.from_numpy(itf.master.X).to(dev)
    iface = MortarInterface(Xs, torch.from_numpy(itf.slave.conn), Xm, torch.from_numpy(itf.master.conn),
                            params=default_params(delta=itf.delta), device=dev)
    iface.setup()
    n_pairs, n_cand, nnz_D, nnz_M = iface.n_pairs, iface.n_cand, iface.nnz_D, iface.nnz_M
    Dr = np.repeat(np.arange(itf.slave.n_nodes), np.diff(iface.D_rowptr.cpu().numpy()))
    Mr = np.repeat(np.arange(itf.slave.n_nodes), np.diff(iface.M_rowptr.cpu().numpy()))
    wD = torch.from_numpy(keyed_normal(3000, TAG_D, Dr, iface.D_col.cpu().numpy())).to(dev)
    wM = torch.from_numpy(keyed_normal(3000, TAG_M, Mr, iface.M_col.cpu().numpy())).to(dev)
    idx = np.arange(itf.slave.n_nodes)
    wg = torch.from_numpy(keyed_normal(3000, TAG_G, idx, 0 * idx)).to(dev)
    outs = iface.alloc_outputs()
    grads = (torch.empty(3, itf.slave.n_nodes, dtype=torch.float64, device=dev),
             torch.empty(3, itf.master.n_nodes, dtype=torch.float64, device=dev))

    def step(sync=True):
        iface.build_pairs(sync=sync)
        iface.csr_pattern(sync=sync)
        iface.integrate(outs)
        iface.backward(wD, wM, wg, grads)

    def step_fused(sync=True):
        # the same step with mt_integrate_backward (the weights are known
        # before the values): the assembly runs beside the reverse sweep
        iface.build_pairs(sync=sync)
        iface.csr_pattern(sync=sync)
        iface.integrate_backward(wD, wM, wg, out=outs, grad_out=grads)

    def wall(fn, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # an instrumented pass: every phase bracketed by events (per-phase times)
    iface.timings(reset=True)
    iface.set_timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    iface.set_timing(False)
    tim_all = iface.timings(reset=True)
    per_step = {k: v[0] / args.steps for k, v in tim_all.items()}
    per_launch = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in tim_all.items()}
    dominant = max(("pair_poly", "pair_fwd", "pair_bwd"), key=lambda k: per_launch.get(k, 0.0))
    # the synchronous step (counts read back by every call), events only
    # around the dominant pair kernel, whose launch time the roofline uses
    iface.set_timing(True, phases=[dominant])
    ms_sync = wall(step, args.steps)
    iface.set_timing(False)
    tim = iface.timings(reset=True)
    assert iface.n_pairs == n_pairs and iface.n_cand == n_cand
    if tim[dominant][1]:
        per_launch[dominant] = tim[dominant][0] / tim[dominant][1]
    # the step without host waits (no count read-backs), then captured once
    # into a HIP graph and replayed: the per-iteration form of a Newton loop
    # (fixed capacities, coordinates updated in place)
    ms_async = wall(lambda: step(False), args.steps)
    iface.check()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step(False)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        step(False)
    ms_graph = wall(graph.replay, args.steps)
    iface.check()
    del graph
    ms_fused = wall(lambda: step_fused(False), args.steps)
    iface.check()
    # the same step with mt_integrate_backward, captured once and replayed
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step_fused(False)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        step_fused(False)
    ms_fused_graph = wall(graph.replay, args.steps)
    iface.check()
    del graph
    # forward path alone (search + pattern + forward), no timers
    fwd_ms = wall(lambda: (iface.build_pairs(sync=False), iface.csr_pattern(sync=False), iface.integrate(outs)),
                  args.steps)
    iface.check()
    st = iface.stats()
    assert st["n_pairs"] == n_pairs
    # device memory of the interface (before the legs below allocate their own)
    mem_gb = (free0 - torch.cuda.mem_get_info(dev)[0]) / 2**30
    # the same step on a context that runs every kernel on the caller's
    # stream (single_stream): what the library's internal concurrency buys,
    # and each phase's time alone
    single = None
    if not args.no_single_stream:
        single = bench_variant(itf, (wD, wM, wg), args.steps, args.warmup, sync=False, single_stream=1)
    ms_step = min(ms_graph, ms_async, ms_fused, ms_fused_graph, single["ms_per_step"] if single else float("inf"))

    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    dual = None if args.no_dual else bench_variant(itf, (wD, wM, wg), args.steps, args.warmup, dual=True)
    nodal = None if args.no_nodal else bench_variant(itf, (wD, wM, wg), args.steps, args.warmup, nodal_normals=True)
    elements = None if args.no_elements else bench_elements(itf, outs, args.steps, args.warmup)
    batched = None if args.no_batched else bench_batched()

    # Roofline of the longest pair kernel (FP64-VALU bound): achieved =
    # executed FP64 flops per launch (rocprofv3 counters of FP64 VALU
    # instructions, committed under profiles/, times 64 lanes, FMA 2 flops)
    # over the launch time measured here; the oracle's operation count per
    # pair is reported beside it as the algorithmic model.
    counters = recorded_counters(FP64_SUMMARY)

    def roofline(k):
        if not per_launch.get(k):
            return None
        launch_s = per_launch[k] * 1e-3
        kern = KERNELS[k][0]
        executed = counters.get(f"{kern}.fp64_flops_per_launch") if counters else None
        valu = counters.get(f"{kern}.valu_insts_per_launch") if counters else None
        achieved = executed / launch_s / 1e12 if executed else None
        r = {"bound": "alu", "kernel": kern, "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
             "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS if achieved else None,
             "traffic": recorded_traffic(k), "traffic_unit": "bytes per launch",
             "flops_source": "executed FP64 VALU instructions per launch (rocprofv3 SQ_INSTS_VALU_{FMA,ADD,MUL,TRANS}_F64"
                             " x 64 lanes, FMA 2 flops)",
             "units_per_launch": n_pairs, "unit_kind": "pair", "launch_ms": per_launch[k],
             "executed_flops_per_pair": executed / n_pairs if executed else None}
        if valu:
            # VALU issue: a wave64 VALU instruction occupies a 16-lane SIMD 4 cycles
            r["valu_issue_frac"] = valu * 4 / (launch_s * 2.4e9 * 256 * 4)
        if model:
            m = model[k] * n_pairs / launch_s / 1e12
            r["oracle_model"] = {"flops_per_pair": model[k], "achieved": m, "frac": m / FP64_VECTOR_PEAK_TFLOPS}
        return r

    roof = roofline(dominant)
    others = {KERNELS[k][0]: roofline(k) for k in ("pair_poly", "pair_fwd", "pair_bwd")
              if k != dominant and per_launch.get(k)}
    # the forward's launch time above is taken beside the pattern kernels (on
    # the internal stream); its time alone comes from the single-stream leg
    fwd_alone = single["phase_ms_per_step"].get("pair_fwd") if single else None
    if fwd_alone and others.get("k_pair_fwd") and others["k_pair_fwd"].get("achieved"):
        e = others["k_pair_fwd"]
        executed = e["executed_flops_per_pair"] * n_pairs
        e["alone"] = {"launch_ms": fwd_alone, "achieved": executed / (fwd_alone * 1e-3) / 1e12,
                      "frac": executed / (fwd_alone * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS}
    ab = algorithmic_bytes(itf.slave.n_nodes, itf.master.n_nodes, itf.slave.n_el, itf.master.n_el, n_cand, n_pairs,
                           nnz_D, nnz_M)
    search_ms = sum(per_step.get(k, 0.0) for k in ("prep", "bin_sort", "cand", "clip", "compact"))
    hbm = {"search": hbm_entry(ab["search"], search_ms),
           "assemble": hbm_entry(ab["forward"] - (24 * (itf.slave.n_nodes + itf.master.n_nodes)
                                                  + 16 * (itf.slave.n_el + itf.master.n_el)), per_step.get("assemble")),
           "forward_path": hbm_entry(ab["forward_path"], fwd_ms),
           "step": hbm_entry(ab["step"], ms_step),
           "definitions": algorithmic_bytes.__doc__.split("\n", 2)[2].strip()}
    out = {
        "metric": "mortar element pairs integrated/sec (D,M,gap) fwd and fwd+bwd, 1 MI355X",
        "value": n_pairs / (ms_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "wavy z=0.05 sin(2 pi x) sin(2 pi y), slave 1024x1024 / master 777x777 quad4, "
                               "normal offsets U[-1e-3,1e-3], delta 1.25e-3: search + forward + backward per step",
                   "n_pairs": n_pairs, "n_candidates": n_cand, "nnz_D": nnz_D, "nnz_M": nnz_M},
        "step_modes_ms": {"graph_replay": ms_graph, "async": ms_async, "sync_counts": ms_sync,
                          "fused_async": ms_fused, "fused_graph_replay": ms_fused_graph,
                          "single_stream_async": single["ms_per_step"] if single else None},
        "single_stream_phase_ms_per_step": single["phase_ms_per_step"] if single else None,
        "step_note": "value: the fastest of the eager no-wait step, its graph replay, the eager step with "
                     "mt_integrate_backward in place of mt_integrate + mt_backward (the same outputs bit for bit; "
                     "the assembly beside the reverse sweep) and its graph replay, and the eager step on a context "
                     "with every kernel on the caller's stream (single_stream); inputs resident, every phase "
                     "recomputed; sync_counts reads the counts back in every call",
        "fwd_pairs_per_s": n_pairs / (fwd_ms * 1e-3),
        "fwd_ms_per_step": fwd_ms,
        "phase_ms_per_step": per_step,
        "phase_note": "instrumented synchronous pass; pair_fwd runs on the internal stream inside the pattern phase",
        "device_memory_gib": mem_gb,
        "workspace_bytes": iface._ws_bytes,
        "roofline": roof,
        "roofline_other_kernels": others,
        "hbm": hbm,
        "dual_basis": dual,
        "nodal_normals": nodal,
        "element_based": elements,
        "batched_64_interfaces": batched,
    }
    if counters and counters.get("step.fp64_flops"):
        out["step_fp64_frac"] = counters["step.fp64_flops"] / (ms_step * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS
    if model and elements:
        elements["segment_integrate_ms"] = per_step["pair_fwd"] + per_step["assemble"]
        for ng in ELEM_RULES:
            e = elements[str(ng)]
            fl = model["elem_flops_per_element"][ng]
            ach = fl * e["slave_elements"] / (e["k_elem_fwd_ms"] * 1e-3) / 1e12
            e["oracle_model"] = {"kernel": "k_elem_fwd", "achieved": ach, "unit": "TFLOP/s",
                                 "frac": ach / FP64_VECTOR_PEAK_TFLOPS, "flops_per_unit": fl,
                                 "unit_kind": "slave element", "units_per_launch": e["slave_elements"]}
            # per slave element its connectivity, nodes and pair range
            # (16 + 96 + 8 B), per pair its master index, connectivity and
            # nodes (4 + 16 + 96 B) read and its 36 block values (288 B) written
            by = e["slave_elements"] * 120 + e["n_pairs"] * 404
            e["roofline_hbm"] = dict(hbm_entry(by, e["k_elem_fwd_ms"]), kernel="k_elem_fwd")
    if cpu:
        one, alln = cpu["one_core"], cpu["all_cores"]
        out["cpu_baseline"] = {
            "value": alln["pairs"] / alln["wall"], "unit": "pairs/s", "cores": alln["cores"], "kind": "oracle",
            "sample": f"slave-grid rows 0..{alln['rows'] - 1} of the workload ({alln['rows'] * 1024} slave elements, "
                      f"{alln['pairs']} pairs) against the whole master side, {alln['cores']} forked oracle "
                      f"processes of {one['rows']} rows each; per process: search + clip + integrate + assemble + "
                      f"forward-mode gradients",
            "one_core": {"value": one["pairs"] / one["t_all"], "fwd_only": one["pairs"] / one["t_fwd"],
                         "pairs": one["pairs"], "rows": one["rows"]}}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
