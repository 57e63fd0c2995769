"""Benchmark of the mortar coupling hot path on one MI355X.

One step = the whole path on one synthetic interface with inputs resident in
HBM: contact search and clipping (mt_build_pairs), CSR pattern
(mt_csr_pattern), segment-based integration and assembly of D, M and the
weighted gap (mt_integrate), and the backward pass for seeded upstream
weights (mt_backward).  Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the mortar path here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not a measured mode)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2202_03933_amd import MortarInterface, default_params
    from synth.weights import keyed_normal, TAG_D, TAG_M, TAG_G

    dev = torch.device("cuda", 0)
    itf = synth.interface_config(2)
    iface = MortarInterface(torch.from_numpy(itf.slave.X), torch.from_numpy(itf.slave.conn),
                            torch.from_numpy(itf.master.X), torch.from_numpy(itf.master.conn),
                            params=default_params(delta=itf.delta), device=dev)
    iface.setup()
    n_pairs = iface.n_pairs
    Dr = np.repeat(np.arange(itf.slave.n_nodes), np.diff(iface.D_rowptr.cpu().numpy()))
    Mr = np.repeat(np.arange(itf.slave.n_nodes), np.diff(iface.M_rowptr.cpu().numpy()))
    wD = torch.from_numpy(keyed_normal(3000, TAG_D, Dr, iface.D_col.cpu().numpy())).to(dev)
    wM = torch.from_numpy(keyed_normal(3000, TAG_M, Mr, iface.M_col.cpu().numpy())).to(dev)
    idx = np.arange(itf.slave.n_nodes)
    wg = torch.from_numpy(keyed_normal(3000, TAG_G, idx, 0 * idx)).to(dev)
    outs = iface.alloc_outputs()
    grads = (torch.empty(3, itf.slave.n_nodes, dtype=torch.float64, device=dev),
             torch.empty(3, itf.master.n_nodes, dtype=torch.float64, device=dev))

    phases = ["search", "pattern", "forward", "backward"]
    ev = {p: [] for p in phases}

    def step(record):
        s = torch.cuda.current_stream()
        marks = []
        if record:
            e0 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            marks.append(e0)
        for fn in (iface.build_pairs, iface.csr_pattern, lambda: iface.integrate(outs),
                   lambda: iface.backward(wD, wM, wg, grads)):
            fn()
            if record:
                e = torch.cuda.Event(enable_timing=True)
                e.record(s)
                marks.append(e)
        return marks

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    all_marks = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        all_marks.append(step(True))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for marks in all_marks:
        for i, p in enumerate(phases):
            ev[p].append(marks[i].elapsed_time(marks[i + 1]))
    ms_step = (t1 - t0) * 1e3 / args.steps
    assert iface.n_pairs == n_pairs
    phase_ms = {p: float(np.mean(v)) for p, v in ev.items()}
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
        "config": {"workload": "wavy z=0.05 sin(2pi x) sin(2pi y), slave 1024x1024 / master 777x777 quad4, "
                               "search + forward + backward",
                   "n_pairs": n_pairs, "n_candidates": iface.n_cand, "nnz_D": iface.nnz_D, "nnz_M": iface.nnz_M},
        "phase_ms": phase_ms,
        "fwd_pairs_per_s": n_pairs / ((phase_ms["search"] + phase_ms["pattern"] + phase_ms["forward"]) * 1e-3),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
