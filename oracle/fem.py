"""P1/P2 Lagrange spaces, local matrices and assembly (oracle).

Spaces (Section 2.2.1, eqs. (4)-(5)): velocity in continuous P2 per component,
pressure in continuous P1 (Taylor-Hood P2-P1, Section 4.2).

Numbering adopted here (the paper does not fix one):
* P1 DOFs are the mesh vertices in input order.
* P2 DOFs are the vertices, then the edges (unique vertex pairs of cells)
  sorted lexicographically by (min vertex, max vertex).
* Local P2 order in a triangle: v0, v1, v2, e(v1v2), e(v2v0), e(v0v1); in a
  tetrahedron: v0..v3, e01, e02, e03, e12, e13, e23.
* Basis in barycentrics: P1 lam_i; P2 vertex lam_i (2 lam_i - 1); P2 edge
  4 lam_a lam_b.

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


# ----------------------------------------------------------------- spaces
class Space:
    """Mesh + P1/P2 DOF maps + geometry for one simplicial mesh."""

    def __init__(self, X, cells):
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
    lam, w = quadrature.cell_rule(space.dim)
    return lam, w


def local_mass_p2(space):
    lam, w = _rule(space)
    phi, _ = p2_basis(lam)
    return np.einsum('q,c,qi,qj->cij', w, space.absdet, phi, phi)


def local_mass_p1(space):
    lam, w = _rule(space)
    psi, _ = p1_basis(lam)
    return np.einsum('q,c,qi,qj->cij', w, space.absdet, psi, psi)


def local_stiff_p2(space):
    lam, w = _rule(space)
    _, dref = p2_basis(lam)
    g = space.phys_grad(dref)
    return np.einsum('q,c,cqia,cqja->cij', w, space.absdet, g, g)


def local_stiff_p1(space):
    lam, w = _rule(space)
    _, dref = p1_basis(lam)
    g = space.phys_grad(dref)
    return np.einsum('q,c,cqia,cqja->cij', w, space.absdet, g, g)


def local_convection(space, U):
    """C_ij = sum_q w |J| phi_i (u_h . grad phi_j), u_h = sum_m U_m phi_m.
    U has shape (d, N2)."""
    lam, w = _rule(space)
    phi, dref = p2_basis(lam)
    g = space.phys_grad(dref)                                  # (Nc,nq,nloc,d)
    Uloc = U[:, space.c2d2]                                    # (d, Nc, nloc)
    uq = np.einsum('qm,acm->cqa', phi, Uloc)                  # (Nc, nq, d)
    adv = np.einsum('cqa,cqja->cqj', uq, g)                   # u_h . grad phi_j
    return np.einsum('q,c,qi,cqj->cij', w, space.absdet, phi, adv)


def local_div(space, c):
    """(D_c)_kj = sum_q w |J| psi_k d_c phi_j  (P1 rows, P2 columns)."""
    lam, w = _rule(space)
    psi, _ = p1_basis(lam)
    _, dref = p2_basis(lam)
    g = space.phys_grad(dref)
    return np.einsum('q,c,qk,cqj->ckj', w, space.absdet, psi, g[..., c])


def local_grad(space, c):
    """(G_c)_ik = sum_q w |J| phi_i d_c psi_k  (P2 rows, P1 columns)."""
    lam, w = _rule(space)
    phi, _ = p2_basis(lam)
    _, dref1 = p1_basis(lam)
    g1 = space.phys_grad(dref1)
    return np.einsum('q,c,qi,cqk->cik', w, space.absdet, phi, g1[..., c])


def local_load(space, f, t):
    """F_{c,i} = sum_q w |J| f_c(x_q, t) phi_i ; f(x, t) -> (..., d)."""
    lam, w = _rule(space)
    phi, _ = p2_basis(lam)
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


def mass_p2(space):
    return assemble(local_mass_p2(space), space.c2d2, space.c2d2, (space.N2, space.N2))


def mass_p1(space):
    return assemble(local_mass_p1(space), space.c2d1, space.c2d1, (space.N1, space.N1))


def stiff_p2(space):
    return assemble(local_stiff_p2(space), space.c2d2, space.c2d2, (space.N2, space.N2))


def stiff_p1(space):
    return assemble(local_stiff_p1(space), space.c2d1, space.c2d1, (space.N1, space.N1))


def convection(space, U):
    return assemble(local_convection(space, U), space.c2d2, space.c2d2,
                    (space.N2, space.N2))


def divergence(space, c):
    return assemble(local_div(space, c), space.c2d1, space.c2d2, (space.N1, space.N2))


def gradient(space, c):
    return assemble(local_grad(space, c), space.c2d2, space.c2d1, (space.N2, space.N1))


def load(space, f, t):
    loc = local_load(space, f, t)
    return np.stack([assemble_vector(loc[a], space.c2d2, space.N2)
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
