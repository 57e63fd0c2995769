"""Many interfaces evaluated with one persistent launch per phase.

Wraps mt_batch_* of the C ABI.  The batch runs on its own (default-priority)
stream, which it orders after the caller's current stream on entry and before
it on exit, so HIP-graph capture never touches the legacy default stream.
"""

import ctypes
import json
import os

import torch

from . import _capi as C
from .interface import _ptr, workspace


def _ptr_table(tensors):
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr() if t is not None and t.numel() > 0 else None
    return arr


class MortarBatch:
    def __init__(self, interfaces, tuning=None, device=None):
        self.ifaces = list(interfaces)
        self.device = torch.device(device) if device is not None else self.ifaces[0].device
        h = ctypes.c_void_p()
        C.check(C.lib().mt_batch_create(ctypes.byref(h), self.device.index or 0))
        self.h = h
        for it in self.ifaces:
            idx = ctypes.c_int32()
            C.check(C.lib().mt_batch_add(self.h, it.h, ctypes.byref(idx)))
        self.stream = torch.cuda.Stream(device=self.device)
        self.build(tuning)

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def build(self, tuning=None):
        self._tuning = tuning
        t = C.mt_batch_tuning()
        if tuning:
            t.bucket = int(tuning.get("bucket", 0))
            t.block = int(tuning.get("block", 0))
            t.blocks_per_cu = int(tuning.get("blocks_per_cu", 0))
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        n = ctypes.c_size_t()
        C.check(C.lib().mt_batch_workspace_size(self.h, ctypes.byref(n)))
        if n.value > getattr(self, "_ws_bytes", 0):
            self._ws = None
            self._ws, self._ws_ptr = workspace(n.value, self.device)
            self._ws_bytes = n.value
        C.check(C.lib().mt_batch_build(self.h, ctypes.byref(t), ctypes.c_void_p(self._ws_ptr), self._ws_bytes,
                                       self._s()))

    def signature(self):
        props = torch.cuda.get_device_properties(self.device)
        pairs = sum(int(i.n_pairs) for i in self.ifaces)
        rule = int(self.ifaces[0].params.rule)
        basis = int(self.ifaces[0].params.lm_basis)
        return f"{props.name}|n={len(self.ifaces)}|pairs={pairs}|rule={rule}|basis={basis}"

    def autotune(self, cache_path=None):
        """Time the forward pair kernel over a grid of (block, blocks per CU,
        bucket) settings and keep the fastest; results are bitwise
        independent of the choice.  With cache_path, a JSON file maps batch
        signatures to earlier choices."""
        key = self.signature()
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        if key in cache:
            self.build(cache[key])
            return dict(cache[key], cached=True)
        self._tuning = None
        t = C.mt_batch_tuning()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        C.check(C.lib().mt_batch_autotune(self.h, ctypes.byref(t), self._s()))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        choice = {"bucket": t.bucket, "block": t.block, "blocks_per_cu": t.blocks_per_cu}
        self._tuning = choice
        if cache_path:
            cache[key] = choice
            os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1)
        return dict(choice, cached=False)

    def search(self, use_graph=False, rebuild=True):
        """mt_batch_search: the pair search and CSR pattern of every instance
        in one call, on the batch's internal streams (use_graph: captured
        into a HIP graph once, replayed while the instances' workspaces,
        capacities and mesh arrays are unchanged).  With rebuild, the
        instances' new counts are read back and the batch is built again for
        the new pair lists, with the same tuning."""
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        C.check(C.lib().mt_batch_search(self.h, 1 if use_graph else 0, self._s()))
        cur.wait_stream(self.stream)
        for it in self.ifaces:
            it._searched()
        if rebuild:
            for it in self.ifaces:
                it.refresh()
            self.build(self._tuning)

    def alloc_outputs(self):
        return [it.alloc_outputs() for it in self.ifaces]

    def forward(self, outs=None, use_graph=False):
        outs = outs if outs is not None else self.alloc_outputs()
        if len(outs) != len(self.ifaces):
            raise ValueError(f"{len(outs)} output triples for {len(self.ifaces)} instances")
        for it, o in zip(self.ifaces, outs):
            it._check_values(*o)
        self._keep = (_ptr_table([o[0] for o in outs]), _ptr_table([o[1] for o in outs]),
                      _ptr_table([o[2] for o in outs]))
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        C.check(C.lib().mt_batch_forward(self.h, *self._keep, 1 if use_graph else 0, self._s()))
        cur.wait_stream(self.stream)
        return outs

    def backward(self, weights, outs=None, use_graph=False):
        """weights: list of (W_D, W_M, w_g) per instance; returns [(gXs, gXm)]
        with structure-of-arrays (3, n) gradients."""
        dev = self.device
        if outs is None:
            outs = [(torch.empty(3, it.n_slave_nodes, dtype=torch.float64, device=dev),
                     torch.empty(3, it.n_master_nodes, dtype=torch.float64, device=dev)) for it in self.ifaces]
        if len(weights) != len(self.ifaces) or len(outs) != len(self.ifaces):
            raise ValueError(f"{len(weights)} weight triples and {len(outs)} gradient pairs for "
                             f"{len(self.ifaces)} instances")
        w = [tuple(x.contiguous() for x in ws) for ws in weights]
        for it, ws, o in zip(self.ifaces, w, outs):
            it._check_values(*ws, what="weights")
            it._check_grads(*o)
        self._keep_w = w
        tabs = (_ptr_table([x[0] for x in w]), _ptr_table([x[1] for x in w]), _ptr_table([x[2] for x in w]),
                _ptr_table([o[0] for o in outs]), _ptr_table([o[1] for o in outs]))
        self._keep_b = tabs
        cur = torch.cuda.current_stream(dev)
        self.stream.wait_stream(cur)
        C.check(C.lib().mt_batch_backward(self.h, *tabs, 1 if use_graph else 0, self._s()))
        cur.wait_stream(self.stream)
        return outs

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            C.lib().mt_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
