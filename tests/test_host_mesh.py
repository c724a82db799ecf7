"""Host-side logic of the C-ABI library (no GPU needed): the library loads,
exports every symbol declared in include/ipcs.h, and its mesh, DOF maps,
boundary flags and CSR patterns equal the oracle's bit for bit. The
library's own quadrature table is checked against the closed-form simplex
moments."""
import itertools
import os
import re
from math import factorial

import numpy as np
import pytest

from oracle import fem, mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
I = pytest.importorskip("paper_2605_25403_amd.ipcs",
                        reason="libipcs.so not built (run __graft_entry__.build())")


def header_symbols():
    text = open(os.path.join(ROOT, "include", "ipcs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ipcs_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    syms = header_symbols()
    assert len(syms) >= 25
    for s in syms:
        assert hasattr(I.lib, s), s
    assert set(syms) == set(I.EXPORTED)


def oracle_space(dim, n):
    return fem.Space(*(mesh.unit_square(n, n) if dim == 2 else mesh.unit_cube(n, n, n)))


def lib_mesh(dim, n):
    return I.Mesh.unit_square(n) if dim == 2 else I.Mesh.unit_cube(n)


def compare(S, m):
    """Counts, DOF numbering and coordinates, boundary and the four patterns of
    the mesh's pair (velocity: the P2 names, pressure: the P1 names) against
    the oracle's space of the same pair, exactly."""
    c = m.counts
    assert (c.dim, c.nv, c.nc, c.n1, c.n2) == (S.dim, S.Nv, S.Nc, S.Np, S.Nu)
    np.testing.assert_array_equal(I.ipcs_mesh_dof_coords(m.h, I.IPCS_SPACE_P2), S.xu)
    np.testing.assert_array_equal(I.ipcs_mesh_dof_coords(m.h, I.IPCS_SPACE_P1), S.xp)
    np.testing.assert_array_equal(I.ipcs_mesh_cell_dofs(m.h, I.IPCS_SPACE_P2), S.c2du)
    np.testing.assert_array_equal(I.ipcs_mesh_cell_dofs(m.h, I.IPCS_SPACE_P1), S.c2dp)
    np.testing.assert_array_equal(I.ipcs_mesh_boundary(m.h).astype(bool), S.bmask_u)
    assert c.nb2 == S.bmask_u.sum()
    ones = lambda rows, cols: fem.assemble(np.ones((S.Nc, rows.shape[1], cols.shape[1])),
                                           rows, cols, (rows.max() + 1, cols.max() + 1))
    for which, (r, cc) in {I.IPCS_PATTERN_P2P2: (S.c2du, S.c2du),
                           I.IPCS_PATTERN_P1P1: (S.c2dp, S.c2dp),
                           I.IPCS_PATTERN_P1P2: (S.c2dp, S.c2du),
                           I.IPCS_PATTERN_P2P1: (S.c2du, S.c2dp)}.items():
        A = ones(r, cc)
        rp, col = I.ipcs_mesh_pattern(m.h, which)
        np.testing.assert_array_equal(rp, A.indptr)
        np.testing.assert_array_equal(col, A.indices)
        assert c.nnz[which] == A.nnz


@pytest.mark.parametrize("dim,n", [(2, 1), (2, 2), (2, 5), (2, 16), (3, 1), (3, 2), (3, 3)])
def test_structured_meshes_match_oracle_exactly(dim, n):
    compare(oracle_space(dim, n), lib_mesh(dim, n))


def test_unstructured_mesh_from_arrays_matches_oracle():
    rng = np.random.default_rng(11)
    X, cells = mesh.unit_square(6, 5)
    X = X.copy()
    interior = (X[:, 0] > 0) & (X[:, 0] < 1) & (X[:, 1] > 0) & (X[:, 1] < 1)
    X[interior] += 0.04 * rng.standard_normal((interior.sum(), 2))
    cells = cells[rng.permutation(len(cells))]
    flip = rng.random(len(cells)) < 0.5
    cells[flip] = cells[flip][:, [0, 2, 1]]          # clockwise cells are allowed
    compare(fem.Space(X, cells), I.Mesh.from_arrays(X, cells))


def test_library_quadrature_rules_are_degree_5_exact():
    for dim, nq in ((2, 7), (3, 14)):
        lam, w = I.ipcs_quadrature_rule(dim)
        assert lam.shape == (nq, dim + 1)
        np.testing.assert_allclose(lam.sum(axis=1), 1.0, atol=1e-15)
        assert abs(w.sum() - 1.0 / factorial(dim)) < 1e-16
        for alpha in itertools.product(range(6), repeat=dim + 1):
            if sum(alpha) <= 5:
                ex = np.prod([factorial(a) for a in alpha]) / factorial(sum(alpha) + dim)
                got = np.sum(w * np.prod(lam ** np.array(alpha), axis=1))
                assert abs(got - ex) < 5e-17, (dim, alpha)


@pytest.mark.parametrize("dim,nq,deg", [(2, 25, 8), (3, 125, 9)])
def test_library_p3_p2_rules_are_exact_to_their_degree(dim, nq, deg):
    """The P3-P2 cell rules (tetrahedra: nodes from the library's own
    Gauss-Jacobi root finder) integrate every monomial in the barycentric
    coordinates up to their degree to the closed-form simplex moment
    prod(a_k!) / (|a| + dim)!, and are the oracle's rules point by point."""
    from oracle import quadrature
    lam, w = I.ipcs_quadrature_rule_pair(dim, I.IPCS_PAIR_P3P2)
    assert lam.shape == (nq, dim + 1)
    np.testing.assert_allclose(lam.sum(axis=1), 1.0, atol=1e-15)
    assert np.all(w > 0) and np.all(lam >= 0)
    for alpha in itertools.product(range(deg + 1), repeat=dim + 1):
        if sum(alpha) <= deg:
            ex = np.prod([factorial(a) for a in alpha]) / factorial(sum(alpha) + dim)
            got = np.sum(w * np.prod(lam ** np.array(alpha), axis=1))
            assert abs(got - ex) < 5e-17 + 1e-14 * ex, (dim, alpha)
    lo, wo = quadrature.triangle_collapsed_gl(5) if dim == 2 else quadrature.tet_collapsed(5)
    np.testing.assert_allclose(lam, lo, rtol=0, atol=2e-15)
    np.testing.assert_allclose(w, wo, rtol=1e-14, atol=0)
    l2, w2 = I.ipcs_quadrature_rule_pair(dim, I.IPCS_PAIR_P2P1)
    l1, w1 = I.ipcs_quadrature_rule(dim)
    np.testing.assert_array_equal(l2, l1)
    np.testing.assert_array_equal(w2, w1)


def test_invalid_arguments_are_reported():
    with pytest.raises(I.IpcsError) as e:
        I.ipcs_mesh_unit_square(0, 4)
    assert e.value.code == I.IPCS_E_INVALID and "nx" in I.ipcs_last_error()
    m = I.Mesh.unit_square(2)
    out = np.empty(3, dtype=np.float64)
    rc = I.lib.ipcs_mesh_dof_coords(m.h, I.IPCS_SPACE_P2, out.ctypes.data_as(I.C.c_void_p), 3)
    assert rc == I.IPCS_E_INVALID
    with pytest.raises(I.IpcsError):
        I.ipcs_mesh_from_arrays(np.zeros((3, 2)), np.array([[0, 1, 2]]))   # degenerate
    with pytest.raises(I.IpcsError):
        I.ipcs_mesh_from_arrays(np.eye(3, 2), np.array([[0, 1, 5]]))       # bad index
    p = I.ipcs_params_default(dt=-1.0)
    with pytest.raises(I.IpcsError):
        I.ipcs_run_workspace_bytes(m.h, p)
    with pytest.raises(I.IpcsError):
        I.ipcs_run_workspace_bytes(m.h, I.ipcs_params_default(convection=5))
    with pytest.raises(I.IpcsError):
        I.ipcs_run_workspace_bytes(m.h, I.ipcs_params_default(scheme=2))
    with pytest.raises(I.IpcsError):
        I.ipcs_run_workspace_bytes(m.h, I.ipcs_params_default(poisson_start=2))
    warm = I.ipcs_params_default(poisson_start=I.IPCS_START_PREVIOUS)
    assert I.ipcs_run_workspace_bytes(m.h, warm) == I.ipcs_run_workspace_bytes(
        m.h, I.ipcs_params_default())
    with pytest.raises(I.IpcsError):
        I.ipcs_run_workspace_bytes(m.h, I.ipcs_params_default(momentum_start=2))
    # the extrapolated momentum start keeps three tentative velocities (dim x N2 doubles each)
    c = I.ipcs_mesh_counts(m.h)
    pure = I.ipcs_params_default(momentum_start=I.IPCS_MSTART_STATE)
    extra = I.ipcs_run_workspace_bytes(m.h, I.ipcs_params_default()) - \
        I.ipcs_run_workspace_bytes(m.h, pure)
    assert 3 * 8 * c.dim * c.n2 <= extra <= 3 * 8 * c.dim * c.n2 + 3 * 256
    semi = I.ipcs_params_default(convection=I.IPCS_CONV_SEMI_IMPLICIT)
    assert I.ipcs_run_workspace_bytes(m.h, semi) == I.ipcs_run_workspace_bytes(
        m.h, I.ipcs_params_default())


def test_workspace_size_grows_with_the_mesh_and_covers_the_values():
    p = I.ipcs_params_default()
    ms = I.Mesh.unit_square(8)
    small = I.ipcs_run_workspace_bytes(ms.h, p)
    m = I.Mesh.unit_square(32)
    big = I.ipcs_run_workspace_bytes(m.h, p)
    assert big > 4 * small          # fixed-size scratch dominates tiny meshes
    # at least the five P2P2 value arrays and the velocity vectors
    assert big > 5 * 8 * m.counts.nnz[0] + 6 * 8 * 2 * m.counts.n2


@pytest.mark.parametrize("dim,n,seed", [(2, 7, 0), (2, 12, 5), (3, 3, 1)])
def test_jittered_relabelled_meshes_match_oracle(dim, n, seed):
    """Seeded unstructured meshes (moved interior vertices, random vertex
    labels, cell order and orientation): DOF numbering, boundary and patterns
    agree exactly."""
    from paper_2605_25403_amd.workloads import jittered_mesh
    X, cells = jittered_mesh(dim, n, seed)
    compare(fem.Space(X, cells), I.Mesh.from_arrays(X, cells))


@pytest.mark.parametrize("n", [1, 2, 5, 16])
def test_p3_p2_square_matches_oracle_exactly(n):
    m = I.Mesh.unit_square(n, pair=I.IPCS_PAIR_P3P2)
    assert m.pair == I.IPCS_PAIR_P3P2
    compare(fem.Space(*mesh.unit_square(n, n), order=3), m)


@pytest.mark.parametrize("n,seed", [(7, 0), (12, 5)])
def test_p3_p2_jittered_meshes_match_oracle(n, seed):
    """Random vertex labels and orientations exercise the edge-node order (the
    node nearer the edge's lower vertex first)."""
    from paper_2605_25403_amd.workloads import jittered_mesh
    X, cells = jittered_mesh(2, n, seed)
    compare(fem.Space(X, cells, order=3), I.Mesh.from_arrays(X, cells, pair=I.IPCS_PAIR_P3P2))


@pytest.mark.parametrize("n", [1, 2, 3])
def test_p3_p2_cube_matches_oracle_exactly(n):
    """P3 on tetrahedra: vertices, two nodes per edge, one node per face (the
    faces in the order of their sorted vertex triples), boundary faces'
    nodes on the boundary."""
    m = I.Mesh.unit_cube(n, pair=I.IPCS_PAIR_P3P2)
    assert m.pair == I.IPCS_PAIR_P3P2
    compare(fem.Space(*mesh.unit_cube(n, n, n), order=3), m)


def test_p3_p2_jittered_tetrahedra_match_oracle():
    from paper_2605_25403_amd.workloads import jittered_mesh
    X, cells = jittered_mesh(3, 3, 1)
    compare(fem.Space(X, cells, order=3), I.Mesh.from_arrays(X, cells, pair=I.IPCS_PAIR_P3P2))


def test_pair_arguments_are_checked():
    with pytest.raises(I.IpcsError):
        I.ipcs_mesh_unit_square_pair(2, 2, 7)
    with pytest.raises(I.IpcsError):
        I.ipcs_mesh_unit_cube_pair(2, 2, 2, 7)
    assert "pair" in I.ipcs_last_error()
    from paper_2605_25403_amd.workloads import jittered_mesh
    X, cells = jittered_mesh(3, 2, 0)
    with pytest.raises(I.IpcsError):
        I.ipcs_mesh_from_arrays_pair(X, cells, -1)
    assert I.Mesh.unit_square(3).pair == I.IPCS_PAIR_P2P1
    assert I.Mesh.from_arrays(X, cells, pair=I.IPCS_PAIR_P3P2).pair == I.IPCS_PAIR_P3P2


@pytest.mark.parametrize("dim,n,pair", [(2, 3, 0), (3, 2, 0), (2, 3, 1), (3, 2, 1)])
def test_interface_velocity_numbering_is_the_listing_order(dim, n, pair):
    """The velocity numbering of the interface, built here by brute force from
    the library's own vertex and cell tables (independently of the oracle): the
    vertices in input order, then the edges' nodes with the edges sorted by
    (lower, higher) vertex (P2: the midpoint; P3: the node at
    (2 x_lo + x_hi)/3, then the one at (x_lo + 2 x_hi)/3), then (P3) the cell
    centroids in cell order (triangles) or the face centroids with the faces
    sorted by vertex triple (tetrahedra). The library numbers these nodes
    differently inside and converts at the interface."""
    m = I.Mesh.unit_square(n, pair=pair) if dim == 2 else I.Mesh.unit_cube(n, pair=pair)
    c = I.ipcs_mesh_counts(m.h)
    xp = I.ipcs_mesh_dof_coords(m.h, I.IPCS_SPACE_P1).reshape(-1, dim)
    X = xp[:c.nv]
    cp = I.ipcs_mesh_cell_dofs(m.h, I.IPCS_SPACE_P1).reshape(c.nc, -1)[:, :dim + 1]
    edges = sorted({tuple(sorted((int(a), int(b)))) for cell in cp
                    for a, b in itertools.combinations(cell, 2)})
    if pair == 0:
        want = np.vstack([X] + [0.5 * (X[a] + X[b]) for a, b in edges])
    else:
        nodes = [X]
        for a, b in edges:
            nodes += [(2.0 * X[a] + X[b]) / 3.0, (X[a] + 2.0 * X[b]) / 3.0]
        if dim == 2:
            nodes += [X[cell].mean(axis=0) for cell in cp]
        else:
            faces = sorted({tuple(sorted(int(v) for v in f)) for cell in cp
                            for f in itertools.combinations(cell, 3)})
            nodes += [(X[a] + X[b] + X[c]) / 3.0 for a, b, c in faces]
        want = np.vstack(nodes)
    x2 = I.ipcs_mesh_dof_coords(m.h, I.IPCS_SPACE_P2).reshape(-1, dim)
    assert x2.shape == want.shape
    np.testing.assert_allclose(x2, want, rtol=0, atol=1e-15)
    # the cell table and the boundary mask speak the same numbering
    c2 = I.ipcs_mesh_cell_dofs(m.h, I.IPCS_SPACE_P2).reshape(c.nc, -1)
    np.testing.assert_array_equal(c2[:, :dim + 1], cp)
    b = I.ipcs_mesh_boundary(m.h)
    on_edge = np.any((np.abs(want) < 1e-14) | (np.abs(want - 1.0) < 1e-14), axis=1)
    np.testing.assert_array_equal(b.astype(bool), on_edge)
