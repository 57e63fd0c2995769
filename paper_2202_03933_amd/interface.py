"""Torch-facing wrapper of one mortar interface on the GPU.

Torch tensors provide device memory and the stream; all work runs in the HIP
library through the C ABI.  Coordinates are kept as structure-of-arrays
(3, n) float64 tensors, connectivity as (n_el, 4) int32.
"""

import ctypes

import numpy as np
import torch

from . import _capi as C


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def default_params(**kw):
    """The library's default mt_params with the given fields replaced
    (`dual` and `nodal_normals` as booleans); an unknown name raises
    TypeError."""
    p = C.mt_params()
    C.check(C.lib().mt_default_params(ctypes.byref(p)))
    fields = {f[0] for f in C.mt_params._fields_}
    for k, v in kw.items():
        if k == "dual":
            p.lm_basis = C.MT_BASIS_DUAL if v else C.MT_BASIS_STANDARD
        elif k == "nodal_normals":
            p.normals = C.MT_NORMALS_NODAL if v else C.MT_NORMALS_ELEMENT
        elif k in fields:
            setattr(p, k, v)
        else:
            raise TypeError(f"default_params: mt_params has no field {k!r}")
    return p


def workspace(nbytes, device):
    """A device workspace of at least nbytes from torch's allocator (256-byte
    aligned, as the library requires)."""
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t, t.data_ptr() + off


def _check_mesh_shapes(X, conn, side, n_nodes=None):
    """Coordinates must be (n, 3) and connectivity (n_el, 4) (quad4): the
    kernels read three coordinates per node and four node indices per
    element.  A coordinate update without new connectivity (n_nodes given)
    keeps the node count of the upload.  Raises ValueError."""
    xs = tuple(X.shape) if hasattr(X, "shape") else tuple(np.shape(X))
    if len(xs) != 2 or xs[1] != 3:
        raise ValueError(f"{side} coordinates: shape {xs}, expected (n_nodes, 3)")
    if n_nodes is not None and xs[0] != n_nodes:
        raise ValueError(f"{side} coordinates: {xs[0]} nodes, the uploaded mesh has {n_nodes} "
                         "(new connectivity needs a full upload)")
    if conn is not None:
        cs = tuple(conn.shape) if hasattr(conn, "shape") else tuple(np.shape(conn))
        if len(cs) != 2 or cs[1] != 4:
            raise ValueError(f"{side} connectivity: shape {cs}, expected (n_elements, 4)")


def _check_f64(t, n, name, device, rows=None):
    """A float64 tensor on `device` that the kernels read or write as n
    values (rows x n for gradients); n None: not known on the host (a search
    without read-back), only the type and device are checked.  Outputs and
    gradients must also be contiguous (the library writes through the
    pointer).  Raises TypeError / ValueError."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64:
        raise TypeError(f"{name}: expected a float64 torch tensor, got "
                        f"{t.dtype if isinstance(t, torch.Tensor) else type(t).__name__}")
    if t.device.type != device.type or (device.type == "cuda" and t.device.index != device.index):
        raise ValueError(f"{name}: on {t.device}, the interface is on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: not contiguous")
    if rows is not None:
        if t.dim() != 2 or t.shape[0] != rows or (n is not None and t.shape[1] != n):
            raise ValueError(f"{name}: shape {tuple(t.shape)}, expected ({rows}, {n})")
    elif n is not None and t.numel() < n:
        raise ValueError(f"{name}: {t.numel()} values, at least {n} needed")


class MortarInterface:
    """One slave/master interface registered with a library context.

    The library allocates no device memory: the interface keeps a torch
    workspace sized by mt_workspace_size for its capacities (the library's
    defaults at first; after a build that exceeded one, the counts it
    needed, mt_required_capacity) and passes it to mt_build_pairs."""

    def __init__(self, Xs, conn_s, Xm, conn_m, params=None, device=None, stream=None):
        if device is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream
        h = ctypes.c_void_p()
        C.check(C.lib().mt_create(ctypes.byref(h), self.device.index or 0))
        self.h = h
        self.params = params if params is not None else default_params()
        C.check(C.lib().mt_set_params(self.h, ctypes.byref(self.params)))
        self._uploaded = False
        self.set_coordinates(Xs, Xm, conn_s, conn_m)
        self.n_cand = self.n_pairs = None
        self._nnz = None  # (nnz_D, nnz_M) of the last pattern, None: not read back
        self.capacity = None
        self._ws = None
        self._ws_ptr = 0
        self._ws_bytes = 0
        self.coord_version = 0  # counts coordinate registrations (MortarFunction checks it)

    def set_coordinates(self, Xs, Xm, conn_s=None, conn_m=None):
        """Register coordinates (n, 3) and, optionally, connectivity.  With
        connectivity (or on first use) the meshes are uploaded and the pair
        list is invalidated; without, only the coordinates are replaced and
        the pair list and pattern are kept."""
        dev = self.device
        full = conn_s is not None or conn_m is not None or not self._uploaded
        _check_mesh_shapes(Xs, conn_s, "slave", None if full else self.Xs.shape[1])
        _check_mesh_shapes(Xm, conn_m, "master", None if full else self.Xm.shape[1])
        self.Xs = torch.as_tensor(Xs, dtype=torch.float64, device=dev).t().contiguous()
        self.Xm = torch.as_tensor(Xm, dtype=torch.float64, device=dev).t().contiguous()
        if conn_s is not None:
            self.conn_s = torch.as_tensor(conn_s, dtype=torch.int32, device=dev).contiguous()
        if conn_m is not None:
            self.conn_m = torch.as_tensor(conn_m, dtype=torch.int32, device=dev).contiguous()
        L = C.lib()
        for side, X, conn in ((C.MT_SIDE_SLAVE, self.Xs, self.conn_s), (C.MT_SIDE_MASTER, self.Xm, self.conn_m)):
            n = X.shape[1]
            if full:
                C.check(L.mt_upload(self.h, side, n, _ptr(X[0]), _ptr(X[1]), _ptr(X[2]), conn.shape[0],
                                    _ptr(conn), _stream(self.stream)))
            else:
                C.check(L.mt_update_coordinates(self.h, side, _ptr(X[0]), _ptr(X[1]), _ptr(X[2]),
                                                _stream(self.stream)))
        self._uploaded = True
        self.coord_version = getattr(self, "coord_version", 0) + 1

    def move_coordinates(self, Xs, Xm):
        """Write new coordinates (n, 3) into the registered arrays in place
        (same device pointers, so a captured step stays valid); the pair
        list and pattern are kept until the next build."""
        self.Xs.copy_(torch.as_tensor(Xs, dtype=torch.float64, device=self.device).t())
        self.Xm.copy_(torch.as_tensor(Xm, dtype=torch.float64, device=self.device).t())
        L = C.lib()
        for side, X in ((C.MT_SIDE_SLAVE, self.Xs), (C.MT_SIDE_MASTER, self.Xm)):
            C.check(L.mt_update_coordinates(self.h, side, _ptr(X[0]), _ptr(X[1]), _ptr(X[2]), _stream(self.stream)))
        self.coord_version += 1

    def _searched(self):
        # a search without read-back ran (mt_batch_search): counts unknown
        self.n_cand = self.n_pairs = None
        self._nnz = None
        self._csr = None

    def refresh(self):
        """Read back the counts of the last search (waits for it) and raise
        MortarError for a device-side condition (mt_check)."""
        self.check()
        st = self.stats()
        self.n_cand, self.n_pairs = st["n_candidates"], st["n_pairs"]
        self._nnz = (st["nnz_D"], st["nnz_M"])
        self._csr = None

    @property
    def n_slave_nodes(self):
        return int(self.Xs.shape[1])

    @property
    def n_master_nodes(self):
        return int(self.Xm.shape[1])

    def default_capacity(self):
        cap = C.mt_capacity()
        C.check(C.lib().mt_default_capacity(self.h, ctypes.byref(cap)))
        return cap

    def set_capacity(self, cap=None, candidates=None, screened=None, pairs=None, cells=None):
        """Capacities of the next builds (mt_capacity or keywords; None keeps
        the current / default value) and a workspace that holds them."""
        base = cap if cap is not None else (self.capacity or self.default_capacity())
        new = C.mt_capacity(base.candidates, base.screened, base.pairs, base.cells)
        for k, v in (("candidates", candidates), ("screened", screened), ("pairs", pairs), ("cells", cells)):
            if v is not None:
                setattr(new, k, int(v))
        n = ctypes.c_size_t()
        C.check(C.lib().mt_workspace_size(self.h, ctypes.byref(new), ctypes.byref(n)))
        if n.value > self._ws_bytes:
            self._ws = None
            self._ws, self._ws_ptr = workspace(n.value, self.device)
            self._ws_bytes = n.value
        self.capacity = new
        return new

    def build_pairs(self, sync=True):
        """mt_build_pairs into the interface's workspace.  sync=True reads the
        counts back (and, when a capacity was exceeded, enlarges it to the
        counts the build needed and builds again); sync=False launches the
        build without waiting for the device (check() reports its status)."""
        if self.capacity is None:
            self.set_capacity()
        L = C.lib()
        for _ in range(4):
            if not sync:
                C.check(L.mt_build_pairs(self.h, ctypes.byref(self.capacity), ctypes.c_void_p(self._ws_ptr),
                                         self._ws_bytes, None, None, _stream(self.stream)))
                self.n_cand = self.n_pairs = None
                return None
            nc, npairs = ctypes.c_int64(), ctypes.c_int64()
            rc = L.mt_build_pairs(self.h, ctypes.byref(self.capacity), ctypes.c_void_p(self._ws_ptr), self._ws_bytes,
                                  ctypes.byref(nc), ctypes.byref(npairs), _stream(self.stream))
            if rc != C.MT_ECAPACITY:
                # the counts are written also when a device check failed
                self.n_cand, self.n_pairs = nc.value, npairs.value
                C.check(rc)
                return self.n_cand, self.n_pairs
            need = C.mt_capacity()
            C.check(L.mt_required_capacity(self.h, ctypes.byref(need)))
            cap = self.capacity
            self.set_capacity(candidates=max(cap.candidates, need.candidates),
                              screened=max(cap.screened, need.screened), pairs=max(cap.pairs, need.pairs))
        C.check(rc)

    def check(self):
        """mt_check: raises MortarError for a device-side condition since the
        last build (capacity, non-finite coordinates, degenerate elements,
        non-converged inverse maps)."""
        C.check(C.lib().mt_check(self.h))

    def _counts(self):
        if self.n_pairs is None or self.n_cand is None:
            st = self.stats()
            self.n_cand, self.n_pairs = st["n_candidates"], st["n_pairs"]

    def pairs(self):
        self._counts()
        n = self.n_pairs
        s = torch.empty(n, dtype=torch.int32, device=self.device)
        m = torch.empty(n, dtype=torch.int32, device=self.device)
        nv = torch.empty(n, dtype=torch.uint8, device=self.device)
        C.check(C.lib().mt_get_pairs(self.h, _ptr(s), _ptr(m), _ptr(nv), _stream(self.stream)))
        return s, m, nv

    def candidates(self):
        self._counts()
        n = self.n_cand
        s = torch.empty(n, dtype=torch.int32, device=self.device)
        m = torch.empty(n, dtype=torch.int32, device=self.device)
        nv = torch.empty(n, dtype=torch.uint8, device=self.device)
        C.check(C.lib().mt_get_candidates(self.h, _ptr(s), _ptr(m), _ptr(nv), _stream(self.stream)))
        return s, m, nv

    def csr_pattern(self, sync=True):
        """Build the CSR patterns of D and M; the arrays are copied out on
        first access of D_rowptr / D_col / M_rowptr / M_col.  sync=False:
        no read-back of the nonzero counts."""
        self._csr = None
        if not sync:
            C.check(C.lib().mt_csr_pattern(self.h, None, None, _stream(self.stream)))
            self._nnz = None  # read back on first use of nnz_D / nnz_M (refresh)
            return None
        a, b = ctypes.c_int64(), ctypes.c_int64()
        C.check(C.lib().mt_csr_pattern(self.h, ctypes.byref(a), ctypes.byref(b), _stream(self.stream)))
        self._nnz = (a.value, b.value)
        st = self.stats()
        self.n_cand, self.n_pairs = st["n_candidates"], st["n_pairs"]
        return self._nnz

    @property
    def nnz_D(self):
        """Nonzeros of D in the last pattern (read back first, waiting for
        the device, after a call that did not read the counts)."""
        if self._nnz is None:
            self.refresh()
        return self._nnz[0]

    @property
    def nnz_M(self):
        """Nonzeros of M in the last pattern (read back as nnz_D)."""
        if self._nnz is None:
            self.refresh()
        return self._nnz[1]

    def _fetch_csr(self):
        if getattr(self, "_csr", None) is None:
            n1 = self.n_slave_nodes + 1
            dev = self.device
            t = (torch.empty(n1, dtype=torch.int32, device=dev), torch.empty(self.nnz_D, dtype=torch.int32, device=dev),
                 torch.empty(n1, dtype=torch.int32, device=dev), torch.empty(self.nnz_M, dtype=torch.int32, device=dev))
            C.check(C.lib().mt_get_csr(self.h, _ptr(t[0]), _ptr(t[1]), _ptr(t[2]), _ptr(t[3]), _stream(self.stream)))
            self._csr = t
        return self._csr

    D_rowptr = property(lambda self: self._fetch_csr()[0])
    D_col = property(lambda self: self._fetch_csr()[1])
    M_rowptr = property(lambda self: self._fetch_csr()[2])
    M_col = property(lambda self: self._fetch_csr()[3])

    def setup(self):
        self.build_pairs()
        self.csr_pattern()
        return self

    def alloc_outputs(self):
        dev = self.device
        return (torch.empty(self.nnz_D, dtype=torch.float64, device=dev),
                torch.empty(self.nnz_M, dtype=torch.float64, device=dev),
                torch.empty(self.n_slave_nodes, dtype=torch.float64, device=dev))

    def _check_values(self, D, M, g, what="output"):
        # the counts as known on the host: no read-back (a sync-free step
        # stays sync-free)
        nD, nM = self._nnz if self._nnz is not None else (None, None)
        _check_f64(D, nD, f"D {what}", self.device)
        _check_f64(M, nM, f"M {what}", self.device)
        _check_f64(g, self.n_slave_nodes, f"gap {what}", self.device)

    def _check_grads(self, gXs, gXm):
        _check_f64(gXs, self.n_slave_nodes, "slave gradient", self.device, rows=3)
        _check_f64(gXm, self.n_master_nodes, "master gradient", self.device, rows=3)

    def integrate(self, out=None):
        D, M, g = out if out is not None else self.alloc_outputs()
        self._check_values(D, M, g)
        C.check(C.lib().mt_integrate(self.h, _ptr(D), _ptr(M), _ptr(g), _stream(self.stream)))
        return D, M, g

    def backward(self, W_D, W_M, w_g, out=None):
        dev = self.device
        if out is None:
            gXs = torch.empty(3, self.n_slave_nodes, dtype=torch.float64, device=dev)
            gXm = torch.empty(3, self.n_master_nodes, dtype=torch.float64, device=dev)
        else:
            gXs, gXm = out
        W_D = W_D.contiguous()
        W_M = W_M.contiguous()
        w_g = w_g.contiguous()
        self._check_values(W_D, W_M, w_g, "weights")
        self._check_grads(gXs, gXm)
        C.check(C.lib().mt_backward(self.h, _ptr(W_D), _ptr(W_M), _ptr(w_g), _ptr(gXs), _ptr(gXm),
                                    _stream(self.stream)))
        return gXs, gXm

    def integrate_backward(self, W_D, W_M, w_g, out=None, grad_out=None):
        """mt_integrate_backward: (D, M, g) and (gXs, gXm) of integrate() and
        backward() with the same arguments, the assembly beside the reverse
        sweep; for upstream weights known before the values."""
        dev = self.device
        D, M, g = out if out is not None else self.alloc_outputs()
        if grad_out is None:
            gXs = torch.empty(3, self.n_slave_nodes, dtype=torch.float64, device=dev)
            gXm = torch.empty(3, self.n_master_nodes, dtype=torch.float64, device=dev)
        else:
            gXs, gXm = grad_out
        W_D = W_D.contiguous()
        W_M = W_M.contiguous()
        w_g = w_g.contiguous()
        self._check_values(D, M, g)
        self._check_values(W_D, W_M, w_g, "weights")
        self._check_grads(gXs, gXm)
        C.check(C.lib().mt_integrate_backward(self.h, _ptr(D), _ptr(M), _ptr(g), _ptr(W_D), _ptr(W_M), _ptr(w_g),
                                              _ptr(gXs), _ptr(gXm), _stream(self.stream)))
        return (D, M, g), (gXs, gXm)

    def stats(self):
        st = C.mt_stats()
        C.check(C.lib().mt_get_stats(self.h, ctypes.byref(st)))
        return {"n_candidates": st.n_candidates, "n_pairs": st.n_pairs, "nverts_hist": list(st.nverts_hist),
                "n_noconv": st.n_noconv, "n_overflow": st.n_overflow,
                "n_degenerate_slave": st.n_degenerate_slave, "n_degenerate_master": st.n_degenerate_master,
                "n_lost_pairs": st.n_lost_pairs,
                "nnz_D": st.nnz_D, "nnz_M": st.nnz_M, "n_bins": list(st.n_bins), "bin_size": list(st.bin_size)}

    def set_timing(self, enable=True, phases=None):
        """Phase timers on or off; with phases (names from _capi.MT_T_NAMES)
        only those phases are recorded."""
        if phases is None:
            C.check(C.lib().mt_set_timing(self.h, 1 if enable else 0))
        else:
            mask = 0
            for name in phases:
                mask |= 1 << C.MT_T_NAMES.index(name)
            C.check(C.lib().mt_set_timing_phases(self.h, mask if enable else 0))

    def timings(self, reset=False):
        """{phase: (summed ms, intervals)} of the library's phase timers."""
        t = C.mt_timings()
        C.check(C.lib().mt_get_timings(self.h, ctypes.byref(t), 1 if reset else 0))
        return {n: (t.ms[i], t.intervals[i]) for i, n in enumerate(C.MT_T_NAMES)}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            C.lib().mt_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MortarFunction(torch.autograd.Function):
    """(Xs (n_s, 3), Xm (n_m, 3)) -> (D_val, M_val, gap) on a fixed pair list
    and CSR pattern; backward returns dL/dXs, dL/dXm from the hand-written
    reverse-mode kernel, at the coordinates of this forward (re-registered
    when another forward moved the interface since)."""

    @staticmethod
    def forward(ctx, Xs, Xm, iface):
        Xs_d, Xm_d = Xs.detach(), Xm.detach()
        iface.set_coordinates(Xs_d, Xm_d)
        D, M, g = iface.integrate()
        ctx.iface = iface
        ctx.coords = (Xs_d, Xm_d)
        ctx.version = iface.coord_version
        return D, M, g

    @staticmethod
    def backward(ctx, gD, gM, gg):
        iface = ctx.iface
        if iface.coord_version != ctx.version:
            # another forward (a second loss, a line-search trial point) moved
            # the interface: evaluate the gradient at this forward's point
            iface.set_coordinates(*ctx.coords)
            ctx.version = iface.coord_version
        dev = iface.device
        gD = gD if gD is not None else torch.zeros(iface.nnz_D, dtype=torch.float64, device=dev)
        gM = gM if gM is not None else torch.zeros(iface.nnz_M, dtype=torch.float64, device=dev)
        gg = gg if gg is not None else torch.zeros(iface.n_slave_nodes, dtype=torch.float64, device=dev)
        gXs, gXm = iface.backward(gD, gM, gg)
        return gXs.t().contiguous(), gXm.t().contiguous(), None
