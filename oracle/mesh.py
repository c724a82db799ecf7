"""Structured simplex meshes of the unit square and unit cube (oracle).

Section 2.2.1 partitions the domain by a conforming simplicial mesh T_h; the
getting-started example (Section 4.2) builds it with a uniform triangle
generator on [0,1]^2 and its DOF counts (table "convergence_data") are those of
n x n squares split into two triangles each. The split is not stated; the
oracle takes the SW-NE diagonal in 2D and the 6-tetrahedron Kuhn split of each
cube in 3D (every tetrahedron contains the cube's main diagonal), both
conforming.
"""
import itertools

import numpy as np


def unit_square(nx, ny):
    """Vertices (i/nx, j/ny), index j*(nx+1)+i; two counter-clockwise triangles
    (a,b,c), (a,c,e) per square with a=(i,j), b=(i+1,j), c=(i+1,j+1), e=(i,j+1)."""
    X = np.array([(i / nx, j / ny) for j in range(ny + 1) for i in range(nx + 1)],
                 dtype=np.float64)
    cells = []
    for j in range(ny):
        for i in range(nx):
            a = j * (nx + 1) + i
            b = a + 1
            c = a + (nx + 1) + 1
            e = a + (nx + 1)
            cells.append((a, b, c))
            cells.append((a, c, e))
    return X, np.array(cells, dtype=np.int64)


def unit_cube(nx, ny, nz):
    """Vertex (i,j,k) has index (k(ny+1)+j)(nx+1)+i. Each cube gives the six
    Kuhn tetrahedra v0 -> v0+e_a -> v0+e_a+e_b -> v0+(1,1,1) over the six
    orderings (a,b,c) of the axes; vertices are reordered to positive volume."""
    def vid(i, j, k):
        return (k * (ny + 1) + j) * (nx + 1) + i

    X = np.array([(i / nx, j / ny, k / nz)
                  for k in range(nz + 1) for j in range(ny + 1) for i in range(nx + 1)],
                 dtype=np.float64)
    unit = np.eye(3, dtype=np.int64)
    cells = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                base = np.array([i, j, k])
                for perm in itertools.permutations(range(3)):
                    p0 = base
                    p1 = p0 + unit[perm[0]]
                    p2 = p1 + unit[perm[1]]
                    p3 = p2 + unit[perm[2]]
                    tet = [vid(*p) for p in (p0, p1, p2, p3)]
                    cells.append(tet)
    cells = np.array(cells, dtype=np.int64)
    return X, orient(X, cells)


def orient(X, cells):
    """Swap the last two vertices of every cell with negative signed measure."""
    cells = cells.copy()
    J = X[cells[:, 1:]] - X[cells[:, :1]]          # (Nc, d, d) rows = edges
    det = np.linalg.det(J)
    neg = det < 0
    cells[neg, -2], cells[neg, -1] = cells[neg, -1].copy(), cells[neg, -2].copy()
    return cells
