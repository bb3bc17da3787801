"""Velocity sets of the oracle (test infrastructure only).

D2Q9 and D3Q19 are the paper's Tables tab:D2Q9 and tab:D3Q19 (Section 3),
in the paper's ordering.  D2Q5 and D3Q7 are not in the paper (it uses D2Q9 /
D3Q19 for every equation); they are the scalar lattices of the workloads.  The
reading taken for them: the standard weights that make the second moment
isotropic, sum_k w_k e_k e_k = c_s^2 I, with D2Q5 ordered 0, +x, +y, -x, -y
(the order of the first five D2Q9 vectors) and D3Q7 ordered 0, +x, -x, +y, -y,
+z, -z (the order of the first seven D3Q19 vectors).

Vectors are stored as (ex, ey, ez); 2D lattices have ez = 0.
"""

from fractions import Fraction as Fr

import numpy as np


class Lattice:
    def __init__(self, name, dim, e, w):
        self.name = name
        self.dim = dim
        self.e = np.array([tuple(v) + (0,) * (3 - len(v)) for v in e], dtype=np.int64)
        self.w_exact = [Fr(x) for x in w]
        self.w = np.array([float(x) for x in self.w_exact])
        self.Q = len(self.w)
        # opposite direction: e_opp[k] = -e[k]
        self.opp = np.array([int(np.nonzero((self.e == -self.e[k]).all(axis=1))[0][0])
                             for k in range(self.Q)])
        # c_s^2 from the second moment sum_k w_k e_kx^2 (exact rational)
        self.cs2_exact = sum(wk * int(ek[0]) ** 2 for wk, ek in zip(self.w_exact, self.e))
        self.cs2 = float(self.cs2_exact)

    def __repr__(self):
        return f"Lattice({self.name})"


# Table tab:D2Q9 (Section 3): k = 0; 1..4 axis vectors; 5..8 diagonals.
D2Q9 = Lattice("D2Q9", 2,
               [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
                (1, 1), (-1, 1), (-1, -1), (1, -1)],
               [Fr(4, 9)] + [Fr(1, 9)] * 4 + [Fr(1, 36)] * 4)

# Table tab:D3Q19 (Section 3): k = 0; 1..6 axis vectors; 7..18 edge diagonals.
D3Q19 = Lattice("D3Q19", 3,
                [(0, 0, 0),
                 (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
                 (1, 1, 0), (-1, -1, 0), (1, 0, 1), (-1, 0, -1), (0, 1, 1), (0, -1, -1),
                 (1, -1, 0), (-1, 1, 0), (1, 0, -1), (-1, 0, 1), (0, 1, -1), (0, -1, 1)],
                [Fr(1, 3)] + [Fr(1, 18)] * 6 + [Fr(1, 36)] * 12)

# Scalar lattices (reading stated in the module docstring).
D2Q5 = Lattice("D2Q5", 2,
               [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1)],
               [Fr(1, 3)] + [Fr(1, 6)] * 4)

D3Q7 = Lattice("D3Q7", 3,
               [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)],
               [Fr(1, 4)] + [Fr(1, 8)] * 6)

BY_NAME = {lat.name: lat for lat in (D2Q9, D3Q19, D2Q5, D3Q7)}


# ----------------------------------------------------------------------------------------
# moment basis for multiple-relaxation-time collisions

def _monomials(dim):
    """Polynomials in (cx, cy, cz) whose values on a lattice span its moment space, in
    increasing order; the second order is split into the trace and traceless parts so
    that bulk and shear stresses are separate moments.  Returned as (order, function)."""
    x = lambda e: e[0]
    y = lambda e: e[1]
    z = lambda e: e[2]
    if dim == 2:
        return [(0, lambda e: 1), (1, x), (1, y),
                (2, lambda e: x(e) ** 2 + y(e) ** 2), (2, lambda e: x(e) ** 2 - y(e) ** 2),
                (2, lambda e: x(e) * y(e)),
                (3, lambda e: x(e) ** 2 * y(e)), (3, lambda e: x(e) * y(e) ** 2),
                (4, lambda e: x(e) ** 2 * y(e) ** 2)]
    return [(0, lambda e: 1), (1, x), (1, y), (1, z),
            (2, lambda e: x(e) ** 2 + y(e) ** 2 + z(e) ** 2),
            (2, lambda e: 2 * x(e) ** 2 - y(e) ** 2 - z(e) ** 2), (2, lambda e: y(e) ** 2 - z(e) ** 2),
            (2, lambda e: x(e) * y(e)), (2, lambda e: x(e) * z(e)), (2, lambda e: y(e) * z(e)),
            (3, lambda e: x(e) ** 2 * y(e)), (3, lambda e: x(e) ** 2 * z(e)), (3, lambda e: y(e) ** 2 * x(e)),
            (3, lambda e: y(e) ** 2 * z(e)), (3, lambda e: z(e) ** 2 * x(e)), (3, lambda e: z(e) ** 2 * y(e)),
            (4, lambda e: x(e) ** 2 * y(e) ** 2), (4, lambda e: x(e) ** 2 * z(e) ** 2),
            (4, lambda e: y(e) ** 2 * z(e) ** 2)]


def moment_basis(lat):
    """Rows of an invertible moment matrix M (exact rationals) orthogonal in the
    weighted product <a, b> = sum_k w_k a_k b_k, by Gram-Schmidt over the monomials
    above (skipping those that are dependent on the lattice), with the polynomial
    order of each row.  Its inverse is M^-1_{k i} = w_k M_{i k} / <M_i, M_i>."""
    rows, orders = [], []
    for order, fn in _monomials(lat.dim):
        v = [Fr(fn(tuple(int(c) for c in lat.e[k]))) for k in range(lat.Q)]
        for r in rows:
            num = sum(w * a * b for w, a, b in zip(lat.w_exact, v, r))
            den = sum(w * b * b for w, b in zip(lat.w_exact, r))
            v = [a - num / den * b for a, b in zip(v, r)]
        if any(a != 0 for a in v):
            rows.append(v)
            orders.append(order)
        if len(rows) == lat.Q:
            break
    assert len(rows) == lat.Q, lat.name
    return rows, orders

