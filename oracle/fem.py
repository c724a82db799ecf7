"""P1/P2/P3 Lagrange spaces, local matrices and assembly (oracle).

Spaces (Section 2.2.1, eqs. (4)-(5)): velocity in continuous P2 per component,
pressure in continuous P1 (Taylor-Hood P2-P1, Section 4.2); or, on triangles,
velocity in P3 and pressure in P2 (the P3-P2 Taylor-Hood pair of the paper's
higher-order study, table "convergence_p3_p2").

Numbering adopted here (the paper does not fix one):
* P1 DOFs are the mesh vertices in input order.
* P2 nodes are the vertices and the edge midpoints (edges = unique vertex
  pairs of cells, listed sorted by (min vertex, max vertex)).
* Velocity DOFs are numbered in listing order: the vertices in input order,
  then the other nodes of the velocity space (P2: the edge midpoints in edge
  order; P3: below). This is the numbering of every velocity array exchanged
  with the library.
* The P3-P2 pressure (P2) keeps the listing order: vertices, then edges.
* Local P2 order in a triangle: v0, v1, v2, e(v1v2), e(v2v0), e(v0v1); in a
  tetrahedron: v0..v3, e01, e02, e03, e12, e13, e23.
* Basis in barycentrics: P1 lam_i; P2 vertex lam_i (2 lam_i - 1); P2 edge
  4 lam_a lam_b.
* P3 (triangles) nodes: the vertices, two per edge (edge k with sorted
  vertices lo < hi has nodes at (2 x_lo + x_hi)/3 and (x_lo + 2 x_hi)/3), one
  per cell at its centroid; numbered in that order.
  Local order: v0, v1, v2; for each local edge (a, b) of (v1v2, v2v0, v0v1)
  the node nearer a, then the node nearer b; the centroid. Basis: vertex
  lam_i (3 lam_i - 1)(3 lam_i - 2) / 2; edge node nearer a
  9/2 lam_a lam_b (3 lam_a - 1); centroid 27 lam_0 lam_1 lam_2.
* P3 (tetrahedra) nodes: the vertices, two per edge (as for triangles), one
  per face at its centroid (faces = unique sorted vertex triples of cells,
  listed lexicographically); a tetrahedron has no interior P3 node. Local
  order: v0..v3; for each local edge (a, b) of (01, 02, 03, 12, 13, 23) the
  node nearer a, then the node nearer b; the centroids of the faces opposite
  v0, v1, v2, v3. Basis as for triangles, face node 27 lam_a lam_b lam_c.
* The space of the pair is chosen by `order` (2: P2-P1, 3: P3-P2). The
  generic names (Nu, c2du, xu, bmask_u for velocity; Np, c2dp, xp for
  pressure) are what the IPCS step uses; N1/N2, c2d1/c2d2, x2, boundary2
  keep their P1/P2 meaning for either pair.

Local matrices are written out as the defining sums over quadrature points
(w_q |det J| times products of basis values and physical gradients), then
summed into a global COO list and converted to CSR with scipy. The CSR
pattern is the full cell-coupling pattern: entries whose contributions cancel
are kept as explicit zeros.
"""
import numpy as np
import scipy.sparse as sp

from . import quadrature

EDGES_2D = [(1, 2), (2, 0), (0, 1)]
EDGES_3D = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
FACES_3D = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]   # face k: opposite vertex k


def local_edges(dim):
    return EDGES_2D if dim == 2 else EDGES_3D


# ----------------------------------------------------------------- basis
def bary_grad(dim):
    """Reference gradients of the barycentric coordinates, shape (dim+1, dim)."""
    g = np.zeros((dim + 1, dim))
    g[0, :] = -1.0
    for k in range(dim):
        g[k + 1, k] = 1.0
    return g


def p1_basis(lam):
    """Values (nq, d+1) and reference gradients (nq, d+1, d) of P1."""
    dim = lam.shape[1] - 1
    G = bary_grad(dim)
    return lam.copy(), np.broadcast_to(G, (lam.shape[0],) + G.shape).copy()


def p2_basis(lam):
    """Values (nq, nloc) and reference gradients (nq, nloc, d) of P2."""
    nq, dp1 = lam.shape
    dim = dp1 - 1
    G = bary_grad(dim)
    edges = local_edges(dim)
    nloc = dp1 + len(edges)
    phi = np.zeros((nq, nloc))
    dphi = np.zeros((nq, nloc, dim))
    for i in range(dp1):
        phi[:, i] = lam[:, i] * (2.0 * lam[:, i] - 1.0)
        dphi[:, i, :] = (4.0 * lam[:, i] - 1.0)[:, None] * G[i][None, :]
    for e, (a, b) in enumerate(edges):
        phi[:, dp1 + e] = 4.0 * lam[:, a] * lam[:, b]
        dphi[:, dp1 + e, :] = 4.0 * (lam[:, b][:, None] * G[a][None, :]
                                     + lam[:, a][:, None] * G[b][None, :])
    return phi, dphi


def p3_basis(lam):
    """Values (nq, nloc) and reference gradients (nq, nloc, d) of P3: nloc = 10
    on triangles, 20 on tetrahedra."""
    nq, dp1 = lam.shape
    dim = dp1 - 1
    G = bary_grad(dim)
    edges = local_edges(dim)
    nloc = 10 if dim == 2 else 20
    phi = np.zeros((nq, nloc))
    dphi = np.zeros((nq, nloc, dim))
    for i in range(dp1):
        L = lam[:, i]
        phi[:, i] = 0.5 * L * (3.0 * L - 1.0) * (3.0 * L - 2.0)
        dphi[:, i, :] = (0.5 * (27.0 * L * L - 18.0 * L + 2.0))[:, None] * G[i][None, :]
    for e, (a, b) in enumerate(edges):
        for k, (p, q) in enumerate(((a, b), (b, a))):   # node nearer p
            Lp, Lq = lam[:, p], lam[:, q]
            j = dp1 + 2 * e + k
            phi[:, j] = 4.5 * Lp * Lq * (3.0 * Lp - 1.0)
            # d/dLp = 4.5 Lq (6 Lp - 1), d/dLq = 4.5 Lp (3 Lp - 1)
            dphi[:, j, :] = ((4.5 * Lq * (6.0 * Lp - 1.0))[:, None] * G[p][None, :]
                             + (4.5 * Lp * (3.0 * Lp - 1.0))[:, None] * G[q][None, :])
    faces = [(0, 1, 2)] if dim == 2 else FACES_3D
    for f, (a, b, c) in enumerate(faces):
        j = dp1 + 2 * len(edges) + f
        La, Lb, Lc = lam[:, a], lam[:, b], lam[:, c]
        phi[:, j] = 27.0 * La * Lb * Lc
        dphi[:, j, :] = 27.0 * ((Lb * Lc)[:, None] * G[a][None, :]
                                + (La * Lc)[:, None] * G[b][None, :]
                                + (La * Lb)[:, None] * G[c][None, :])
    return phi, dphi


# ----------------------------------------------------------------- spaces
class Space:
    """Mesh + DOF maps of a Taylor-Hood pair + geometry for one simplicial mesh."""

    def __init__(self, X, cells, order=2):
        self.X = np.asarray(X, dtype=np.float64)
        self.cells = np.asarray(cells, dtype=np.int64)
        self.dim = self.X.shape[1]
        self.Nv = self.X.shape[0]
        self.Nc = self.cells.shape[0]
        d = self.dim
        edges = local_edges(d)
        pairs = np.stack([np.sort(self.cells[:, [a, b]], axis=1) for (a, b) in edges],
                         axis=1)                                   # (Nc, ne, 2)
        flat = pairs.reshape(-1, 2)
        uniq, inv = np.unique(flat, axis=0, return_inverse=True)   # lexicographic
        self.edges = uniq
        self.N1 = self.Nv
        self.N2 = self.Nv + uniq.shape[0]
        self.c2d1 = self.cells.copy()
        self.c2d2 = np.concatenate(
            [self.cells, self.Nv + inv.reshape(self.Nc, len(edges))], axis=1)
        self.nloc2 = self.c2d2.shape[1]
        # P2 node coordinates: vertices then edge midpoints
        self.x2 = np.concatenate([self.X, 0.5 * (self.X[uniq[:, 0]] + self.X[uniq[:, 1]])])
        # geometry: J has columns x_k - x_0
        x0 = self.X[self.cells[:, 0]]
        self.J = np.stack([self.X[self.cells[:, k + 1]] - x0 for k in range(d)], axis=2)
        self.detJ = np.linalg.det(self.J)
        self.absdet = np.abs(self.detJ)
        self.Jinv = np.linalg.inv(self.J)
        self.boundary2 = self._boundary_p2()
        if order not in (2, 3):
            raise ValueError("pairs: P2-P1 or P3-P2")
        self.order = order
        if order == 2:
            self.Nu, self.c2du, self.xu, self.bmask_u = self.N2, self.c2d2, self.x2, self.boundary2
            self.Np, self.c2dp, self.xp = self.N1, self.c2d1, self.X
            self.basis_u, self.basis_p = p2_basis, p1_basis
        else:
            self._p3_dofs(inv.reshape(self.Nc, len(edges)))
            self.Np, self.c2dp, self.xp = self.N2, self.c2d2, self.x2
            self.basis_u, self.basis_p = p3_basis, p2_basis

    def _p3_dofs(self, cell_edges):
        """P3 DOF numbering, node coordinates and boundary mask."""
        d = self.dim
        Nv, Ne, Nc = self.Nv, self.edges.shape[0], self.Nc
        edges = local_edges(d)
        nloc = 10 if d == 2 else 20
        c2d = np.zeros((Nc, nloc), dtype=np.int64)
        c2d[:, :d + 1] = self.cells
        for e, (a, b) in enumerate(edges):
            k = cell_edges[:, e]
            fwd = self.cells[:, a] < self.cells[:, b]        # a is the edge's lower vertex
            c2d[:, d + 1 + 2 * e] = np.where(fwd, Nv + 2 * k, Nv + 2 * k + 1)
            c2d[:, d + 2 + 2 * e] = np.where(fwd, Nv + 2 * k + 1, Nv + 2 * k)
        lo, hi = self.X[self.edges[:, 0]], self.X[self.edges[:, 1]]
        ex = np.empty((2 * Ne, d))
        ex[0::2] = (2.0 * lo + hi) / 3.0
        ex[1::2] = (lo + 2.0 * hi) / 3.0
        mask = np.zeros(Nv + 2 * Ne, dtype=bool)
        mask[:Nv] = self.boundary2[:Nv]
        be = self.boundary2[Nv:]                  # boundary edges (P2 mask)
        mask[Nv:Nv + 2 * Ne:2] = be
        mask[Nv + 1:Nv + 2 * Ne:2] = be
        if d == 2:
            c2d[:, 9] = Nv + 2 * Ne + np.arange(Nc)
            fx = self.X[self.cells].mean(axis=1)
            fmask = np.zeros(Nc, dtype=bool)
        else:
            tri = np.stack([np.sort(self.cells[:, list(f)], axis=1) for f in FACES_3D],
                           axis=1)                                  # (Nc, 4, 3)
            faces, finv, fcount = np.unique(tri.reshape(-1, 3), axis=0, return_inverse=True,
                                            return_counts=True)
            self.faces = faces
            c2d[:, 16:20] = Nv + 2 * Ne + finv.reshape(Nc, 4)
            fx = self.X[faces].mean(axis=1)
            fmask = fcount == 1                   # faces owned by one cell
        self.N3 = Nv + 2 * Ne + fx.shape[0]
        self.Nu, self.c2du = self.N3, c2d
        self.xu = np.concatenate([self.X, ex, fx])
        self.bmask_u = np.concatenate([mask, fmask])

    def _boundary_p2(self):
        """Topological boundary: facets owned by exactly one cell; their vertices
        and (P2) edges are boundary nodes."""
        d = self.dim
        facets = []
        for k in range(d + 1):
            idx = [m for m in range(d + 1) if m != k]
            facets.append(np.sort(self.cells[:, idx], axis=1))
        F = np.concatenate(facets, axis=0)
        uniq, counts = np.unique(F, axis=0, return_counts=True)
        bf = uniq[counts == 1]
        mask = np.zeros(self.N2, dtype=bool)
        mask[np.unique(bf.ravel())] = True
        # edges of boundary facets
        edge_index = {tuple(e): self.Nv + i for i, e in enumerate(self.edges)}
        for f in bf:
            for a in range(d):
                for b in range(a + 1, d):
                    mask[edge_index[(min(f[a], f[b]), max(f[a], f[b]))]] = True
        return mask

    # physical gradients: grad phi = J^{-T} grad_ref phi
    def phys_grad(self, dref):
        return np.einsum('cab,qia->cqib', self.Jinv, dref)

    def map_points(self, lam):
        """Physical coordinates of barycentric points, (Nc, nq, d)."""
        return np.einsum('qk,ckd->cqd', lam, self.X[self.cells])


# ----------------------------------------------------------------- local matrices
def _rule(space):
    """Cell rule: degree 5 for P2-P1 (every integrand has degree <= 5); for
    P3-P2 (convection P3 (P3 . grad P3) has degree 8) the collapsed 5 x 5
    Gauss-Legendre rule on triangles (exact to degree 8) and Stroud's conical
    product of 5-point Gauss-Jacobi rules on tetrahedra (125 points, exact to
    degree 9)."""
    if space.order == 2:
        return quadrature.cell_rule(space.dim)
    if space.dim == 2:
        return quadrature.triangle_collapsed_gl(5)
    return quadrature.tet_collapsed(5)


def local_mass_u(space):
    lam, w = _rule(space)
    phi, _ = space.basis_u(lam)
    return np.einsum('q,c,qi,qj->cij', w, space.absdet, phi, phi)


def local_mass_p(space):
    lam, w = _rule(space)
    psi, _ = space.basis_p(lam)
    return np.einsum('q,c,qi,qj->cij', w, space.absdet, psi, psi)


def local_stiff_u(space):
    lam, w = _rule(space)
    _, dref = space.basis_u(lam)
    g = space.phys_grad(dref)
    return np.einsum('q,c,cqia,cqja->cij', w, space.absdet, g, g)


def local_stiff_p(space):
    lam, w = _rule(space)
    _, dref = space.basis_p(lam)
    g = space.phys_grad(dref)
    return np.einsum('q,c,cqia,cqja->cij', w, space.absdet, g, g)


# the P2-P1 names (the pair's velocity/pressure spaces when order == 2)
local_mass_p2, local_mass_p1 = local_mass_u, local_mass_p
local_stiff_p2, local_stiff_p1 = local_stiff_u, local_stiff_p


def local_convection(space, U):
    """C_ij = sum_q w |J| phi_i (u_h . grad phi_j), u_h = sum_m U_m phi_m.
    U has shape (d, Nu)."""
    lam, w = _rule(space)
    phi, dref = space.basis_u(lam)
    g = space.phys_grad(dref)                                  # (Nc,nq,nloc,d)
    Uloc = U[:, space.c2du]                                    # (d, Nc, nloc)
    uq = np.einsum('qm,acm->cqa', phi, Uloc)                  # (Nc, nq, d)
    adv = np.einsum('cqa,cqja->cqj', uq, g)                   # u_h . grad phi_j
    return np.einsum('q,c,qi,cqj->cij', w, space.absdet, phi, adv)


def local_div(space, c):
    """(D_c)_kj = sum_q w |J| psi_k d_c phi_j  (pressure rows, velocity columns)."""
    lam, w = _rule(space)
    psi, _ = space.basis_p(lam)
    _, dref = space.basis_u(lam)
    g = space.phys_grad(dref)
    return np.einsum('q,c,qk,cqj->ckj', w, space.absdet, psi, g[..., c])


def local_grad(space, c):
    """(G_c)_ik = sum_q w |J| phi_i d_c psi_k  (velocity rows, pressure columns)."""
    lam, w = _rule(space)
    phi, _ = space.basis_u(lam)
    _, dref1 = space.basis_p(lam)
    g1 = space.phys_grad(dref1)
    return np.einsum('q,c,qi,cqk->cik', w, space.absdet, phi, g1[..., c])


def local_load(space, f, t):
    """F_{c,i} = sum_q w |J| f_c(x_q, t) phi_i ; f(x, t) -> (..., d)."""
    lam, w = _rule(space)
    phi, _ = space.basis_u(lam)
    xq = space.map_points(lam)                                 # (Nc, nq, d)
    fq = f(xq, t)                                              # (Nc, nq, d)
    return np.einsum('q,c,cqa,qi->aci', w, space.absdet, fq, phi)  # (d, Nc, nloc)


# ----------------------------------------------------------------- assembly
def assemble(loc, rows_map, cols_map, shape):
    """Sum local matrices loc[c, i, j] into a CSR matrix with the full
    cell-coupling pattern (explicit zeros kept, column indices sorted)."""
    Nc, ni, nj = loc.shape
    r = np.broadcast_to(rows_map[:, :, None], (Nc, ni, nj)).ravel()
    c = np.broadcast_to(cols_map[:, None, :], (Nc, ni, nj)).ravel()
    A = sp.coo_matrix((loc.ravel(), (r, c)), shape=shape).tocsr()
    A.sort_indices()
    return A


def assemble_vector(loc, rows_map, n):
    out = np.zeros(n)
    np.add.at(out, rows_map.ravel(), loc.ravel())
    return out


def mass_u(space):
    return assemble(local_mass_u(space), space.c2du, space.c2du, (space.Nu, space.Nu))


def mass_p(space):
    return assemble(local_mass_p(space), space.c2dp, space.c2dp, (space.Np, space.Np))


def stiff_u(space):
    return assemble(local_stiff_u(space), space.c2du, space.c2du, (space.Nu, space.Nu))


def stiff_p(space):
    return assemble(local_stiff_p(space), space.c2dp, space.c2dp, (space.Np, space.Np))


mass_p2, mass_p1, stiff_p2, stiff_p1 = mass_u, mass_p, stiff_u, stiff_p


def convection(space, U):
    return assemble(local_convection(space, U), space.c2du, space.c2du,
                    (space.Nu, space.Nu))


def divergence(space, c):
    return assemble(local_div(space, c), space.c2dp, space.c2du, (space.Np, space.Nu))


def gradient(space, c):
    return assemble(local_grad(space, c), space.c2du, space.c2dp, (space.Nu, space.Np))


def load(space, f, t):
    loc = local_load(space, f, t)
    return np.stack([assemble_vector(loc[a], space.c2du, space.Nu)
                     for a in range(space.dim)])


# ----------------------------------------------------------------- Dirichlet
def eliminate(A, bmask):
    """Symmetric elimination of the rows/columns flagged in bmask: A_IB = 0,
    A_BI = 0, A_BB = I. The sparsity pattern is kept."""
    A = A.tocsr(copy=True)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    kill = bmask[rows] | bmask[cols]
    A.data[kill] = 0.0
    diag = kill & (rows == cols)
    A.data[diag] = 1.0
    return A


def lift(A, b, bmask, g):
    """Right-hand side for the eliminated system: b_I - A_IB g, and g on B."""
    gext = np.where(bmask, g, 0.0)
    out = b - A @ gext
    out[bmask] = g[bmask]
    return out
