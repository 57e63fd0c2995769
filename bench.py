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
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2202_03933_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
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


def cpu_baseline(itf, n_slave_el_sample, seed=3000):
    """Oracle (serial C++, one core) on a bounded sample of the workload: the
    slave elements [0, n) against the whole master side -- search, clip,
    integration, assembly and gradients.  Returns a dict; also counts the
    oracle's flops per pair for the forward evaluation."""
    import numpy as np

    import oracle
    import synth
    from synth.weights import keyed_normal, TAG_D, TAG_M, TAG_G

    sub = synth.Mesh(itf.slave.X, itf.slave.conn[:n_slave_el_sample].copy())
    prm = oracle.params(delta=itf.delta)
    oracle._lib()  # load outside the timed region
    t0 = time.perf_counter()
    cs, cm = oracle.search(sub, itf.master, itf.delta)
    nv, blocks, _ = oracle.eval_candidates(sub, itf.master, prm, cs, cm, integrate=True)
    keep = nv >= 3
    ps, pm = cs[keep], cm[keep]
    D, M, g = oracle.assemble(sub, itf.master, ps, pm, blocks[keep])
    t_fwd = time.perf_counter() - t0
    fD = lambda r, c: keyed_normal(seed, TAG_D, r, c)  # noqa: E731
    fM = lambda r, c: keyed_normal(seed, TAG_M, r, c)  # noqa: E731
    fg = lambda r: keyed_normal(seed, TAG_G, r, np.zeros_like(r))  # noqa: E731
    w = oracle.pair_weights(sub, itf.master, ps, pm, fD, fM, fg)
    g24, _ = oracle.pair_grads(sub, itf.master, prm, ps, pm, w)
    oracle.scatter_grads(sub, itf.master, ps, pm, g24)
    t_all = time.perf_counter() - t0
    # algorithmic flops (oracle's flop-counting scalar on every 16th pair and
    # every 16th candidate of the sample).  Per kernel:
    #   k_pair_poly:  the candidate pass of every pair;
    #   k_pair_fwd:   the pair evaluation minus its candidate pass;
    #   k_pair_bwd:   that forward recompute + the reverse-mode adjoint of the
    #     pair evaluation minus that of its candidate pass (cost model: adjoint
    #     of add/sub 2, mul 4, div 4, sqrt 3) + IFT_FLOPS per inverse map.
    f_cp, f_pair, f_adj, n_inv, f_cadj = oracle.count_flops(sub, itf.master, prm, ps[::16], pm[::16], detail=True)
    npp = max(1, ps[::16].size)
    # the same flop model per geometry of the batched interfaces: the first
    # 512 slave elements of the largest instance of each geometry
    geo = {}
    for b in synth.batched_instances(64):
        g = b.meta["geometry"]
        if g not in geo or b.slave.conn.shape[0] > geo[g].slave.conn.shape[0]:
            geo[g] = b
    batched_flops = {}
    for g, b in geo.items():
        bs = synth.Mesh(b.slave.X, b.slave.conn[:512].copy())
        bprm = oracle.params(delta=b.delta)
        bcs, bcm = oracle.search(bs, b.master, b.delta)
        bnv, _, _ = oracle.eval_candidates(bs, b.master, bprm, bcs, bcm, integrate=False)
        bk = bnv >= 3
        q = oracle.count_flops(bs, b.master, bprm, bcs[bk], bcm[bk], detail=True)
        nb = max(1, int(bk.sum()))
        batched_flops[g] = {"fwd": (q[1] - q[0]) / nb, "bwd": (q[1] - q[0] + q[2] - q[4] + IFT_FLOPS * q[3]) / nb,
                            "fwd_full": q[1] / nb}
    # element-based integration: flops per slave element (every element with
    # a pair among the first 2048 of the sample)
    esel = ps < 2048
    n_e = max(1, np.unique(ps[esel]).size)
    elem_flops = {ng: oracle.count_flops_elements(sub, itf.master, prm, ps[esel], pm[esel], ng) / n_e
                  for ng in ELEM_RULES}
    return {"pairs": int(ps.size), "t_fwd": t_fwd, "t_all": t_all, "batched_flops": batched_flops,
            "elem_flops_per_element": elem_flops,
            "flops_per_unit": {"pair_poly": f_cp / npp,
                               "pair_fwd": (f_pair - f_cp) / npp,
                               "pair_bwd": (f_pair - f_cp + f_adj - f_cadj + IFT_FLOPS * n_inv) / npp},
            "sample": f"slave elements 0..{n_slave_el_sample - 1} of the workload (the first "
                      f"{n_slave_el_sample // 1024} rows of the 1024x1024 slave grid) against the whole master "
                      f"side: {ps.size} pairs; search + clip + integrate + assemble + gradients"}


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
    for k in ("fwd", "bwd"):
        res[f"{k}_pairs_per_s_batched"] = pairs / (res[f"{k}_ms_batched_graph"] * 1e-3)
        res[f"{k}_pairs_per_s_per_interface"] = pairs / (res[f"{k}_ms_per_interface"] * 1e-3)
        res[f"{k}_speedup"] = res[f"{k}_ms_per_interface"] / res[f"{k}_ms_batched_graph"]
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


def bench_variant(itf, weights, steps, warmup, **params):
    """The same step with other parameters: the dual Lagrange multiplier basis
    (dual-basis forward and backward, the backward including the adjoint of
    the dual coefficients), or auxiliary planes from the continuous nodal
    normal field (its normals computed in every search, its gradient chain in
    every backward)."""
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
        it.build_pairs()
        it.csr_pattern()
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
    n_pairs = it.n_pairs
    it.close()
    ms = (t1 - t0) * 1e3 / steps
    return {"ms_per_step": ms, "pairs_per_s": n_pairs / (ms * 1e-3), "n_pairs": n_pairs,
            "phase_ms_per_step": {k: v[0] / steps for k, v in tim.items()}}


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
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (calibrates HBM traffic counters)")
    ap.add_argument("--cpu-sample", type=int, default=16384, help="slave elements in the CPU oracle sample")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the mortar path on a single MI355X; "
              "sharding over several GPUs is a design note, not a measured mode", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2202_03933_amd import MortarInterface, default_params
    from synth.weights import keyed_normal, TAG_D, TAG_M, TAG_G

    dev = torch.device("cuda", 0)
    itf = synth.interface_config(2)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(dev)[0]
    iface = MortarInterface(torch.from_numpy(itf.slave.X), torch.from_numpy(itf.slave.conn),
                            torch.from_numpy(itf.master.X), torch.from_numpy(itf.master.conn),
                            params=default_params(delta=itf.delta), device=dev)
    iface.setup()
    n_pairs, n_cand = iface.n_pairs, iface.n_cand
    Dr = np.repeat(np.arange(itf.slave.n_nodes), np.diff(iface.D_rowptr.cpu().numpy()))
    Mr = np.repeat(np.arange(itf.slave.n_nodes), np.diff(iface.M_rowptr.cpu().numpy()))
    wD = torch.from_numpy(keyed_normal(3000, TAG_D, Dr, iface.D_col.cpu().numpy())).to(dev)
    wM = torch.from_numpy(keyed_normal(3000, TAG_M, Mr, iface.M_col.cpu().numpy())).to(dev)
    idx = np.arange(itf.slave.n_nodes)
    wg = torch.from_numpy(keyed_normal(3000, TAG_G, idx, 0 * idx)).to(dev)
    outs = iface.alloc_outputs()
    grads = (torch.empty(3, itf.slave.n_nodes, dtype=torch.float64, device=dev),
             torch.empty(3, itf.master.n_nodes, dtype=torch.float64, device=dev))

    def step():
        iface.build_pairs()
        iface.csr_pattern()
        iface.integrate(outs)
        iface.backward(wD, wM, wg, grads)

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
    # the timed pass: events only around the dominant pair kernel, whose
    # launch time the roofline uses
    iface.set_timing(True, phases=[dominant])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    iface.set_timing(False)
    tim = iface.timings(reset=True)
    assert iface.n_pairs == n_pairs and iface.n_cand == n_cand
    ms_step = (t1 - t0) * 1e3 / args.steps
    # device memory held for the workload: library buffers, torch inputs,
    # outputs, weights and gradients, and torch's cached blocks
    mem_gb = (free0 - torch.cuda.mem_get_info(dev)[0]) / 2**30
    if tim[dominant][1]:
        per_launch[dominant] = tim[dominant][0] / tim[dominant][1]
    # forward path alone (search + pattern + forward), wall clock, no timers;
    # the phase sums cannot give it: the forward runs beside the pattern
    # kernels on the library's internal stream, inside the "pattern" phase
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        iface.build_pairs()
        iface.csr_pattern()
        iface.integrate(outs)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) * 1e3 / args.steps

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
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(itf, args.cpu_sample)

    # roofline of the longest of the pair kernels (FP64-VALU bound; the search
    # and pattern kernels are shorter, latency bound, and are reported by their
    # phase times): achieved = oracle-counted algorithmic flops per unit x
    # units per launch / average launch time from the library's event timers
    # over the timed steps
    units = {"pair_poly": n_pairs, "pair_fwd": n_pairs, "pair_bwd": n_pairs}

    def roofline(k):
        fp = cpu["flops_per_unit"][k] if cpu else None
        if fp is None or not per_launch.get(k):
            return None
        launch_s = per_launch[k] * 1e-3
        achieved = fp * units[k] / launch_s / 1e12
        traffic = recorded_traffic(k)
        return {"bound": "alu", "kernel": KERNELS[k][0], "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                "traffic": traffic, "traffic_unit": "bytes per launch" if traffic else None,
                "flops_per_unit": fp, "unit_kind": "pair",
                "units_per_launch": units[k], "launch_ms": per_launch[k]}

    roof = roofline(dominant)
    others = {KERNELS[k][0]: roofline(k) for k in units if k != dominant and per_launch.get(k)}
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
                   "n_pairs": n_pairs, "n_candidates": n_cand, "nnz_D": iface.nnz_D, "nnz_M": iface.nnz_M},
        "fwd_pairs_per_s": n_pairs / (fwd_ms * 1e-3),
        "fwd_ms_per_step": fwd_ms,
        "phase_ms_per_step": per_step,
        "phase_note": "instrumented pass; pair_fwd runs on the internal stream inside the pattern phase",
        "device_memory_gib": mem_gb,
        "roofline": roof,
        "roofline_other_kernels": others,
        "dual_basis": dual,
        "nodal_normals": nodal,
        "element_based": elements,
        "batched_64_interfaces": batched,
    }
    if cpu and batched:
        # batched vs per-interface as fractions of FP64 peak: algorithmic flops
        # of every pair (per-geometry oracle counts) over the wall time
        bf = cpu["batched_flops"]
        for k in ("fwd", "bwd"):
            fl = sum(batched["pairs_by_geometry"][g] * bf[g][k] for g in bf)
            for mode in ("batched_graph", "per_interface"):
                batched[f"{k}_fp64_frac_{mode}"] = fl / (batched[f"{k}_ms_{mode}"] * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS
    if cpu and elements:
        # element-based kernel against FP64 peak: oracle-counted flops per
        # slave element x elements / launch time
        elements["segment_integrate_ms"] = per_step["pair_fwd"] + per_step["assemble"]
        for ng in ELEM_RULES:
            e = elements[str(ng)]
            fl = cpu["elem_flops_per_element"][ng]
            ach = fl * e["slave_elements"] / (e["k_elem_fwd_ms"] * 1e-3) / 1e12
            e["roofline"] = {"bound": "alu", "kernel": "k_elem_fwd", "achieved": ach,
                             "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": ach / FP64_VECTOR_PEAK_TFLOPS, "flops_per_unit": fl,
                             "unit_kind": "slave element", "units_per_launch": e["slave_elements"]}
            # the same launch against HBM: algorithmic bytes = per slave element
            # its connectivity, nodes and pair range (16 + 96 + 8 B), per pair
            # its master index, connectivity and nodes (4 + 16 + 96 B) read and
            # its 36 staged block values (288 B) written
            by = e["slave_elements"] * 120 + e["n_pairs"] * 404
            gbs = by / (e["k_elem_fwd_ms"] * 1e-3) / 1e9
            e["roofline_hbm"] = {"bound": "hbm", "kernel": "k_elem_fwd", "achieved": gbs,
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                                 "bytes_per_launch": by}
    if cpu:
        # whole step as a fraction of FP64 peak (pair kernels' algorithmic flops over the step time)
        fpu = cpu["flops_per_unit"]
        out["step_fp64_frac"] = (fpu["pair_fwd"] + fpu["pair_bwd"]) * n_pairs / (ms_step * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS
        out["cpu_baseline"] = {"value": cpu["pairs"] / cpu["t_all"], "unit": "pairs/s", "cores": 1,
                               "kind": "oracle", "sample": cpu["sample"],
                               "fwd_only_pairs_per_s": cpu["pairs"] / cpu["t_fwd"]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
