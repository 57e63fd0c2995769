"""Small interfaces with degenerate elements, for the error-path tests.

Pure geometry: a flat slave patch with one collapsed element (zero area),
and a flat slave under a master element standing perpendicular to it."""

import numpy as np

from .meshes import Interface, Mesh


def collapsed_slave(collapsed=True):
    """Slave: a 3 x 2 patch of unit-square elements on z = 0 plus one element
    whose four nodes lie on a segment (zero area; with collapsed=False the
    rectangle [1.2, 1.8] x [0.3, 0.7] instead), each element with its own
    nodes; master: one 4 x 3 square covering everything, on z = 0."""
    X, C = [], []
    for j in range(2):
        for i in range(3):
            b = len(X)
            X += [[i, j, 0.0], [i + 1, j, 0.0], [i + 1, j + 1, 0.0], [i, j + 1, 0.0]]
            C.append([b, b + 1, b + 2, b + 3])
    b = len(X)
    if collapsed:
        X += [[1.2, 0.5, 0.0], [1.8, 0.5, 0.0], [1.8, 0.5, 0.0], [1.2, 0.5, 0.0]]  # on a segment
    else:
        X += [[1.2, 0.3, 0.0], [1.8, 0.3, 0.0], [1.8, 0.7, 0.0], [1.2, 0.7, 0.0]]
    C.append([b, b + 1, b + 2, b + 3])
    Xs = np.array(X, float)
    Xm = np.array([[-0.5, -0.5, 0.0], [3.5, -0.5, 0.0], [3.5, 2.5, 0.0], [-0.5, 2.5, 0.0]], float)
    return Interface(Mesh(Xs, np.array(C, np.int32)), Mesh(Xm, np.array([[0, 1, 2, 3]], np.int32)), 0.0,
                     name="flat patch with a collapsed slave element", meta={"geometry": "degenerate"})


def perpendicular_master():
    """Slave: 2 x 2 unit squares on z = 0; master: one element in the plane
    x = 1 (standing on the slave), plus one ordinary flat master element."""
    xs, ys = np.meshgrid(np.arange(3.0), np.arange(3.0), indexing="xy")
    Xs = np.stack([xs.ravel(), ys.ravel(), np.zeros(9)], 1)
    Cs = np.array([[0, 1, 4, 3], [1, 2, 5, 4], [3, 4, 7, 6], [4, 5, 8, 7]], np.int32)
    Xm = np.array([[1.0, 0.2, 0.0], [1.0, 1.8, 0.0], [1.0, 1.8, 1.0], [1.0, 0.2, 1.0],
                   [0.1, 0.1, 0.0], [0.9, 0.1, 0.0], [0.9, 0.9, 0.0], [0.1, 0.9, 0.0]], float)
    Cm = np.array([[0, 1, 2, 3], [4, 5, 6, 7]], np.int32)
    return Interface(Mesh(Xs, Cs), Mesh(Xm, Cm), 0.0, name="flat slave under a perpendicular master",
                     meta={"geometry": "degenerate"})
