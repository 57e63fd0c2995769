"""Seeded synthetic interface meshes.

The paper's own meshes (two cubes in flat contact, a hollow cylinder rolling
on a block; Sec. "Numerical experiments") are not available, so these
tensor-grid surfaces stand in for them: a flat tied interface, a curved
(cylindrical) interface and a large wavy interface, each with a non-matching
slave/master resolution.  Node order of every quad4 is counter-clockwise in
its parameter plane, i.e. nodes at (-1,-1), (1,-1), (1,1), (-1,1).

Layout: coordinates are float64 arrays of shape (n_nodes, 3); connectivity is
int32 of shape (n_el, 4).  Everything here is pure geometry generation.
"""

from dataclasses import dataclass, field
import math

import numpy as np

CONFIG_NAMES = {
    0: "flat 8x8 / 7x7 tied, jittered interior",
    1: "cylinder r=1 90deg x 1, 256x256 / 199x199",
    2: "wavy z=0.05 sin(2pi x) sin(2pi y), 1024x1024 / 777x777",
}


@dataclass
class Mesh:
    X: np.ndarray  # (n_nodes, 3) float64
    conn: np.ndarray  # (n_el, 4) int32

    @property
    def n_nodes(self):
        return int(self.X.shape[0])

    @property
    def n_el(self):
        return int(self.conn.shape[0])


@dataclass
class Interface:
    slave: Mesh
    master: Mesh
    delta: float
    name: str = ""
    meta: dict = field(default_factory=dict)


def tensor_grid(nx, ny):
    """Parameter grid (s, t) in [0,1]^2 with nx x ny quad4 cells.

    Node (i, j) has id j*(nx+1)+i.  Element (i, j) uses nodes
    (i,j), (i+1,j), (i+1,j+1), (i,j+1): counter-clockwise in (s, t).
    Returns (s, t, conn, boundary_mask).
    """
    i = np.arange(nx + 1)
    j = np.arange(ny + 1)
    I, J = np.meshgrid(i, j, indexing="xy")
    s = (I / nx).reshape(-1).astype(np.float64)
    t = (J / ny).reshape(-1).astype(np.float64)
    bnd = ((I == 0) | (I == nx) | (J == 0) | (J == ny)).reshape(-1)
    ei, ej = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ei = ei.reshape(-1)
    ej = ej.reshape(-1)
    n0 = ej * (nx + 1) + ei
    conn = np.stack([n0, n0 + 1, n0 + (nx + 1) + 1, n0 + (nx + 1)], axis=1).astype(np.int32)
    return s, t, conn, bnd


def flat_tied(ns=8, nm=7, seed=1000, jitter=0.1):
    """Flat tied interface on the unit square, z = 0 for both sides.

    Interior nodes of both meshes are moved in-plane by U[-jitter*h, jitter*h]
    in x and y (h = element size); boundary lines and corners coincide exactly.
    jitter=0 gives the unperturbed tensor grids.
    """
    rng = np.random.default_rng(seed)
    meshes = []
    for n in (ns, nm):
        s, t, conn, bnd = tensor_grid(n, n)
        h = 1.0 / n
        X = np.zeros((s.size, 3))
        X[:, 0] = s
        X[:, 1] = t
        if jitter > 0:
            d = rng.uniform(-jitter * h, jitter * h, size=(s.size, 2))
            d[bnd] = 0.0
            X[:, :2] += d
        meshes.append(Mesh(X, conn))
    return Interface(meshes[0], meshes[1], 0.0, name=f"flat {ns}x{ns}/{nm}x{nm}",
                     meta={"geometry": "flat", "ns": ns, "nm": nm, "seed": seed})


def cylinder(ns=256, nm=199, seed=1001, radius=1.0, normal_offset=1e-3,
             tangential=0.05, delta=1.25e-3):
    """Quarter cylinder r=1, theta in [0, pi/2], axis z in [0, 1].

    x = (r cos(theta), r sin(theta), z); the first parameter direction runs
    along theta and the second along z, so the element normal points outward.
    The slave grid is exact.  Every master node is moved outward by
    U[0, normal_offset] in r and tangentially by U[-tangential, tangential]
    of the master element size in theta and in z.
    """
    rng = np.random.default_rng(seed)
    s, t, conn, _ = tensor_grid(ns, ns)
    th = s * (math.pi / 2)
    Xs = np.stack([radius * np.cos(th), radius * np.sin(th), t], axis=1)
    s, t, connm, _ = tensor_grid(nm, nm)
    dth = (math.pi / 2) / nm
    dz = 1.0 / nm
    r = radius + rng.uniform(0.0, normal_offset, size=s.size)
    thm = s * (math.pi / 2) + rng.uniform(-tangential, tangential, size=s.size) * dth
    zm = t + rng.uniform(-tangential, tangential, size=s.size) * dz
    Xm = np.stack([r * np.cos(thm), r * np.sin(thm), zm], axis=1)
    return Interface(Mesh(Xs, conn), Mesh(Xm, connm), delta, name=f"cylinder {ns}x{ns}/{nm}x{nm}",
                     meta={"geometry": "cylinder", "ns": ns, "nm": nm, "seed": seed})


def _wavy_surface(s, t, amp):
    z = amp * np.sin(2 * math.pi * s) * np.sin(2 * math.pi * t)
    fx = amp * 2 * math.pi * np.cos(2 * math.pi * s) * np.sin(2 * math.pi * t)
    fy = amp * 2 * math.pi * np.sin(2 * math.pi * s) * np.cos(2 * math.pi * t)
    nrm = np.stack([-fx, -fy, np.ones_like(s)], axis=1)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return np.stack([s, t, z], axis=1), nrm


def wavy(ns=1024, nm=777, seed=1002, amp=0.05, normal_offset=1e-3, delta=1.25e-3):
    """Wavy surface z = amp sin(2 pi x) sin(2 pi y) on the unit square.

    The slave grid lies exactly on the surface; every master node is moved
    along the unit surface normal by U[-normal_offset, normal_offset].
    """
    rng = np.random.default_rng(seed)
    s, t, conn, _ = tensor_grid(ns, ns)
    Xs, _ = _wavy_surface(s, t, amp)
    s, t, connm, _ = tensor_grid(nm, nm)
    Xm, nrm = _wavy_surface(s, t, amp)
    Xm = Xm + nrm * rng.uniform(-normal_offset, normal_offset, size=(s.size, 1))
    return Interface(Mesh(Xs, conn), Mesh(Xm, connm), delta, name=f"wavy {ns}x{ns}/{nm}x{nm}",
                     meta={"geometry": "wavy", "ns": ns, "nm": nm, "seed": seed})


def graded_flat(ns=6, nm=40, power=3.0, delta=0.0):
    """Flat unit square, slave grid graded in x (x = s**power), master uniform.

    The slave elements range from much narrower to much wider than the
    master elements, so the number of candidates per slave element spans
    from a few to several dozen within one interface.
    """
    s, t, conn, _ = tensor_grid(ns, ns)
    Xs = np.stack([s ** power, t, np.zeros_like(s)], axis=1)
    s, t, connm, _ = tensor_grid(nm, nm)
    Xm = np.stack([s, t, np.zeros_like(s)], axis=1)
    return Interface(Mesh(Xs, conn), Mesh(Xm, connm), delta, name=f"graded flat {ns}x{ns}/{nm}x{nm}",
                     meta={"geometry": "graded flat", "ns": ns, "nm": nm, "power": power})


def kite_fan(n_slave=6, n_master=7, seed=1003, curvature=0.05, normal_offset=1e-3, delta=1.25e-3):
    """Each side a fan of n convex kites around one centre node (valence n).

    Kite k has nodes (centre, r_k, q_k, r_{k+1}) with r_k on the unit circle
    at angle 2 pi k / n and q_k at radius 1.15 halfway between; the surface
    is the paraboloid z = curvature (x^2 + y^2).  The master fan is rotated by
    a tenth of a sector, its centre moved by (0.03, -0.02), it is scaled by
    1.05 and its nodes are moved up by U[0, normal_offset].  Unlike the
    tensor grids (at most four elements per node) the two centres have n
    incident elements.
    """
    rng = np.random.default_rng(seed)

    def fan(n, rot, centre, scale):
        a = 2 * math.pi * np.arange(n) / n + rot
        b = a + math.pi / n
        xy = np.concatenate([[[0.0, 0.0]], np.stack([np.cos(a), np.sin(a)], 1),
                             1.15 * np.stack([np.cos(b), np.sin(b)], 1)]) * scale + np.asarray(centre)
        X = np.concatenate([xy, curvature * (xy ** 2).sum(1, keepdims=True)], 1)
        k = np.arange(n)
        conn = np.stack([np.zeros(n, dtype=np.int64), 1 + k, 1 + n + k, 1 + (k + 1) % n], 1).astype(np.int32)
        return X, conn

    Xs, cs = fan(n_slave, 0.0, (0.0, 0.0), 1.0)
    Xm, cm = fan(n_master, 0.2 * math.pi / n_master, (0.03, -0.02), 1.05)
    Xm[:, 2] += rng.uniform(0.0, normal_offset, size=Xm.shape[0])
    return Interface(Mesh(Xs, cs), Mesh(Xm, cm), delta, name=f"kite fans {n_slave}/{n_master}",
                     meta={"geometry": "kite fan", "ns": n_slave, "nm": n_master, "seed": seed})


def opposing(itf):
    """The same interface with every master element's node order reversed,
    (0, 1, 2, 3) -> (0, 3, 2, 1): the master normal then points against the
    slave normal, as for two bodies in contact, and the master's projection
    onto a slave plane runs clockwise.  Coordinates are shared."""
    conn = np.ascontiguousarray(itf.master.conn[:, [0, 3, 2, 1]]).astype(np.int32)
    meta = dict(itf.meta)
    meta["opposing"] = True
    return Interface(itf.slave, Mesh(itf.master.X, conn), itf.delta, name=itf.name + ", opposing master",
                     meta=meta)


def renumbered(itf, seed=7):
    """The same interface with the nodes and elements of both sides in a
    random order (each element keeps its own node cycle).  meta["new_of_old"]
    holds, per side, the new index of every old node."""
    rng = np.random.default_rng(seed)

    def renum(mesh):
        new_of_old = rng.permutation(mesh.n_nodes)
        X = np.empty_like(mesh.X)
        X[new_of_old] = mesh.X
        conn = new_of_old[mesh.conn[rng.permutation(mesh.n_el)]]
        return Mesh(X, np.ascontiguousarray(conn, dtype=np.int32)), new_of_old

    s, ps = renum(itf.slave)
    m, pm = renum(itf.master)
    meta = dict(itf.meta)
    meta["new_of_old"] = (ps, pm)
    return Interface(s, m, itf.delta, name=itf.name + ", renumbered", meta=meta)


def interface_config(k, scale=None, opposing_normals=False):
    """The workload of configuration k (0 flat, 1 cylinder, 2 wavy).

    `scale` replaces the slave resolution and scales the master resolution
    by the same ratio (used for reduced-size parity cases).
    `opposing_normals` reverses the master node order (see `opposing`).
    """
    if opposing_normals:
        return opposing(interface_config(k, scale))
    if k == 0:
        if scale is None:
            return flat_tied()
        nm = max(2, int(round(scale * 7 / 8)))
        return flat_tied(scale, nm)
    if k == 1:
        if scale is None:
            return cylinder()
        return cylinder(scale, max(2, int(round(scale * 199 / 256))))
    if k == 2:
        if scale is None:
            return wavy()
        return wavy(scale, max(2, int(round(scale * 777 / 1024))))
    raise ValueError(f"unknown configuration {k}")


def batched_instances(n_inst=64, seed_base=2000, side_lo=16, side_hi=512, max_side=None):
    """Many independent interfaces of uneven size.

    Instance i: slave side N_s = round(16 * 32**u), u ~ U(0, 1) (log-uniform in
    16..512); master side N_m = max(2, round(r N_s)), r ~ U[0.7, 1.3];
    geometry cycles flat, cylinder, wavy and is perturbed as in the single
    configurations, seeded with seed_base + i.  `max_side` caps N_s (used for
    reduced-size parity cases).
    """
    out = []
    for i in range(n_inst):
        rng = np.random.default_rng(seed_base + i)
        u = rng.uniform(0.0, 1.0)
        ns = int(round(side_lo * (side_hi / side_lo) ** u))
        r = rng.uniform(0.7, 1.3)
        if max_side is not None:
            ns = min(ns, max_side)
        nm = max(2, int(round(r * ns)))
        geo = i % 3
        seed = int(rng.integers(0, 2**31 - 1))
        if geo == 0:
            itf = flat_tied(ns, nm, seed=seed)
        elif geo == 1:
            itf = cylinder(ns, nm, seed=seed)
        else:
            itf = wavy(ns, nm, seed=seed)
        itf.meta["instance"] = i
        out.append(itf)
    return out
