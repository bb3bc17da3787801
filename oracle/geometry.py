"""Geometry measurements of Section 4.2.2 (subsection "Geometry measurements"):
the droplet count N as the Euler characteristic of the region phi >= 1/2, and the
mean radius from the interface integral of Eq. Rmoy_2D.

Test infrastructure only (not imported by the GPU path).

The Euler characteristic is taken from its definition on the cell complex made of
the closed unit cells (squares in 2D, cubes in 3D) of the nodes with phi >= level:
chi = #vertices - #edges + #faces (- #cubes), where a vertex, edge or face belongs
to the complex when any cell that contains it does.  For separated simply connected
droplets chi is the droplet count.  Periodic axes close the complex on a torus;
along a wall axis the cells end at the wall.  The paper takes N from a one-pass
Euler characteristic algorithm (after Wiemker); counting the elements of the
complex is one such pass.
"""

import itertools

import numpy as np


def _views(present, bc_axes):
    """For every array axis: (lower, upper) cell views of the element positions that
    lie between two cells along that axis.  Periodic: n positions (wrap); walls: n + 1
    positions, with empty cells beyond the walls."""
    b = present
    pad = [(1, 1) if w else (0, 0) for w in bc_axes]
    bp = np.pad(b, pad, constant_values=False)
    return bp


def _element_count(bp, bc_axes, vertex_axes):
    """Number of elements of the complex that are 'vertex-like' (between two cells)
    along vertex_axes and 'cell-like' (a cell interval) along the other axes."""
    nd = bp.ndim
    acc = None
    for shifts in itertools.product((0, 1), repeat=len(vertex_axes)):
        sl = []
        for ax in range(nd):
            n = bp.shape[ax]
            wall = bc_axes[ax]
            if ax in vertex_axes:
                s = shifts[vertex_axes.index(ax)]
                if wall:   # positions between padded cells j and j + 1, j = 0 .. n - 2
                    sl.append(slice(s, n - 1 + s))
                else:      # periodic: between i and i + 1 (mod n)
                    sl.append((np.arange(n) + s) % n)
            else:
                sl.append(slice(1, n - 1) if wall else slice(0, n))
        v = bp[np.ix_(*[np.arange(bp.shape[ax])[s] if isinstance(s, slice) else s for ax, s in enumerate(sl)])]
        acc = v if acc is None else (acc | v)
    return int(acc.sum())


def euler_characteristic(phi, bc, level=0.5):
    """Euler characteristic of the union of closed cells with phi >= level.
    phi is [z][y][x] (nz = 1 for 2D, treated as a 2D complex); bc per axis x, y, z."""
    phi = np.asarray(phi)
    two_d = phi.shape[0] == 1
    present = phi >= level
    walls = {"x": bc[0] == "walls", "y": bc[1] == "walls", "z": bc[2] == "walls"}
    if two_d:
        present = present[0]
        bc_axes = [walls["y"], walls["x"]]
    else:
        bc_axes = [walls["z"], walls["y"], walls["x"]]
    nd = present.ndim
    bp = _views(present, bc_axes)
    chi = 0
    for k in range(nd + 1):  # elements that are vertex-like along k axes: dimension nd - k
        for vax in itertools.combinations(range(nd), k):
            count = _element_count(bp, bc_axes, list(vax))
            dim = nd - k
            chi += (-1) ** dim * count
    return chi


def interface_integral(phi, W):
    """sum_x (4/W) phi (1 - phi): the left side of Eq. Rmoy_2D (interface length in 2D,
    interface area in 3D)."""
    phi = np.asarray(phi)
    return float(np.sum(4.0 / W * phi * (1.0 - phi)))


def mean_radius(phi, W, n_droplets):
    """<R> from the interface integral: 2D Eq. Rmoy_2D, I = 2 pi N <R>; 3D analogue
    (reading: spheres, I = 4 pi sum R_i^2), <R> = sqrt(I / (4 pi N))."""
    phi = np.asarray(phi)
    I = interface_integral(phi, W)
    if n_droplets <= 0:
        return 0.0
    if phi.shape[0] == 1:
        return I / (2.0 * np.pi * n_droplets)
    return float(np.sqrt(I / (4.0 * np.pi * n_droplets)))
