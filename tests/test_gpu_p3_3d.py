"""GPU parity of the P3-P2 Taylor-Hood pair on tetrahedra (the higher-order
pair of the paper's convergence study, carried to 3D) against the FP64
oracle, through the C ABI.

Bars as for the other pairs: assembled matrices max|dA|/max|A| <= 1e-12,
fields ||dx||/||x|| (and max-entry) <= 1e-10 per step, both sides solving to
1e-13; the mixed form within its stated bounds. Cases: the structured cube
from one cube (every velocity node but 4 face and 12 edge nodes on the
boundary) to sizes whose velocity rows span many SELL slices with ragged
tails and whose FP64 row blocks exceed LDS (vertex rows of 175 entries: the
global-accumulation row kernel), a jittered relabelled mesh, Beltrami flow,
the cubic steady state (a fixed point of the step: every integrand has degree
<= 8 and the cell rule is exact to degree 9) with built-in and with host
callback data, both Poisson CG forms, and the mixed form.
"""
import numpy as np
import pytest

from oracle import fem, problems
from paper_2605_25403_amd.workloads import jittered_mesh
from tests.gpu_common import field_errors, make_pair, mat_rel, rel, require_gpu

pytestmark = pytest.mark.gpu

MAT_TOL = 1e-12
FIELD_TOL = 1e-10
NU, DT = 0.05, 0.01


def _matrices_match(I, o, r, tol):
    errs = {"M": mat_rel(r.matrix(I.IPCS_MAT_M), o.M),
            "K": mat_rel(r.matrix(I.IPCS_MAT_K), o.K),
            "Kp": mat_rel(r.matrix(I.IPCS_MAT_KP), o.Kp),
            "A_el": mat_rel(r.matrix(I.IPCS_MAT_A_ELIM), o.A_el),
            "M_el": mat_rel(r.matrix(I.IPCS_MAT_M_ELIM), o.M_el)}
    for c in range(3):
        errs[f"D{c}"] = mat_rel(r.matrix(I.IPCS_MAT_D0 + c), o.D[c])
        errs[f"G{c}"] = mat_rel(r.matrix(I.IPCS_MAT_G0 + c), o.G[c])
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("n", [1, 2, 4])
def test_p3_tet_constant_matrices(n):
    torch, I = require_gpu()
    print(f"P3-P2 tetrahedra constant matrices n={n}", flush=True)
    S, o, r = make_pair(I, 3, n, "beltrami", NU, DT, p3=True)
    assert r.mesh.pair == I.IPCS_PAIR_P3P2
    assert r.mesh.counts.n2 == S.Nu and r.mesh.counts.n1 == S.Np
    _matrices_match(I, o, r, MAT_TOL)


def test_p3_tet_constant_matrices_unstructured():
    torch, I = require_gpu()
    print("P3-P2 tetrahedra constant matrices, jittered mesh", flush=True)
    S, o, r = make_pair(I, 3, 0, "beltrami", NU, DT, p3=True, arrays=jittered_mesh(3, 4, 3))
    _matrices_match(I, o, r, MAT_TOL)


@pytest.mark.parametrize("semi", [False, True])
def test_p3_tet_convection_operator_and_momentum_rhs(semi):
    torch, I = require_gpu()
    print(f"P3-P2 tetrahedra convection/rhs semi={semi}", flush=True)
    S, o, r = make_pair(I, 3, 3, "beltrami", NU, DT, p3=True, semi=semi)
    r.phase(I.IPCS_PHASE_ASM)
    C = fem.convection(S, o.U)
    E = (o.M / DT + (C if semi else -C)).tocsr()
    E.sort_indices()
    assert mat_rel(r.matrix(I.IPCS_MAT_E), E) <= MAT_TOL
    if semi:
        return
    t1 = o.t + DT
    g = o.dirichlet(t1)
    b = r.field(I.IPCS_FIELD_RHS_MOM)
    for c in range(3):
        ref = o.M @ o.U[c] / DT - o.G[c] @ o.P - C @ o.U[c]
        ref = fem.lift(o.A, ref, o.bmask, g[c])
        assert rel(b[c], ref) <= MAT_TOL


@pytest.mark.parametrize("n,arrays", [(4, None), (0, "jittered")])
def test_p3_tet_each_substep_from_identical_state(n, arrays):
    torch, I = require_gpu()
    print(f"P3-P2 tetrahedra substeps n={n} {arrays}", flush=True)
    arr = jittered_mesh(3, 4, 8) if arrays else None
    S, o, r = make_pair(I, 3, n, "beltrami", NU, DT, p3=True, arrays=arr)
    t1 = o.t + DT
    g = o.dirichlet(t1)
    r.phase(I.IPCS_PHASE_ASM)
    st = r.phase(I.IPCS_PHASE_MOMENTUM)
    Us_o, _, _ = o.momentum(t1, g)
    Us = r.field(I.IPCS_FIELD_USTAR)
    for c in range(3):
        assert rel(Us[c], Us_o[c]) <= FIELD_TOL, (c, st)
    st = r.phase(I.IPCS_PHASE_PRESSURE)
    dP_o, _ = o.pressure(Us_o)
    assert rel(r.field(I.IPCS_FIELD_DP), dP_o) <= FIELD_TOL, st
    r.phase(I.IPCS_PHASE_CORRECTION)
    Un_o, _ = o.correction(Us_o, dP_o, g)
    U = r.velocity()
    for c in range(3):
        assert rel(U[c], Un_o[c]) <= FIELD_TOL
    assert rel(r.pressure(), o.P + dP_o) <= FIELD_TOL


@pytest.mark.parametrize("semi", [False, True])
def test_p3_tet_beltrami_steps(semi):
    """Five steps from the library's own device-evaluated start (P3 velocity
    and P2 pressure interpolation at its node coordinates)."""
    torch, I = require_gpu()
    print(f"P3-P2 tetrahedra Beltrami five steps semi={semi}", flush=True)
    S, o, r = make_pair(I, 3, 4, "beltrami", NU, DT, same_state=False, semi=semi, p3=True)
    errs = field_errors(o, r)
    assert max(errs) <= 1e-13, errs
    for step in range(5):
        st = r.advance(1)[0]
        o.step()
        errs = field_errors(o, r)
        assert max(errs) <= FIELD_TOL, (step, errs, st)


@pytest.mark.parametrize("n,semi", [(2, False), (3, True), (12, False)])
def test_p3_tet_cubic_fixed_point(n, semi):
    """Cubic velocity and quadratic pressure are reproduced by the step. n = 12:
    50653 velocity nodes per component, the fused Poisson CG over several
    parts. The start state is checked against the closed form at the oracle
    space's nodes."""
    torch, I = require_gpu()
    print(f"P3-P2 tetrahedra cubic fixed point n={n} semi={semi}", flush=True)
    from oracle import mesh
    pb = problems.PolySteady3DCubic(0.07)
    S = fem.Space(*mesh.unit_cube(n, n, n), order=3)
    kw = dict(convection=I.IPCS_CONV_SEMI_IMPLICIT) if semi else {}
    p = I.ipcs_params_default(nu=0.07, dt=0.05, tol_mom=1e-14, tol_p=1e-14, tol_corr=1e-14, **kw)
    r = I.Run(I.Mesh.unit_cube(n, pair=I.IPCS_PAIR_P3P2), p)
    r.set_builtin(I.IPCS_SOL_POLY_CUBIC_3D)
    U0, P0 = r.velocity().copy(), r.pressure().copy()
    np.testing.assert_allclose(U0, pb.u(S.xu, 0.0).T, atol=1e-14)
    np.testing.assert_allclose(P0, pb.p(S.xp, 0.0), atol=1e-14)
    r.advance(2)
    scale = np.abs(U0).max()
    assert np.abs(r.velocity() - U0).max() < 1e-11 * scale
    assert np.abs(r.pressure() - P0).max() < 1e-10


def test_p3_tet_host_callbacks_match_builtin_data():
    """Forcing at the 125 points of every cell's rule and Dirichlet data at
    the boundary nodes from host callbacks, against the built-in closed forms
    of the same cubic problem."""
    torch, I = require_gpu()
    print("P3-P2 tetrahedra callbacks", flush=True)
    pb = problems.PolySteady3DCubic(0.07)
    m = I.Mesh.unit_cube(3, pair=I.IPCS_PAIR_P3P2)
    p = I.ipcs_params_default(nu=0.07, dt=0.05, callbacks=1, tol_mom=1e-14, tol_p=1e-14,
                              tol_corr=1e-14)
    a = I.Run(m, p)
    a.set_builtin(I.IPCS_SOL_POLY_CUBIC_3D)
    b = I.Run(m, p)
    b.set_state(a.velocity(), a.pressure(), 0.0)
    b.set_dirichlet(lambda x, t: pb.u(x, t))
    b.set_forcing(lambda x, t: pb.f(x, t))
    a.advance(2)
    b.advance(2)
    assert rel(b.velocity(), a.velocity()) <= 1e-12
    assert rel(b.pressure(), a.pressure()) <= 1e-10


def test_p3_tet_mixed_form_within_bound():
    """FP32 matrices within 1e-6 of the FP64 oracle's (their own rounding).
    Fields: velocity within 3e-6 and pressure within 6e-5 over three steps,
    five times the measured 6.4e-7 and 1.2e-5; the pressure error is larger
    for the reason given for the triangle pair (the increment is a small sum
    of large FP32-rounded terms)."""
    torch, I = require_gpu()
    print("P3-P2 tetrahedra mixed form", flush=True)
    S, o, r = make_pair(I, 3, 4, "beltrami", NU, DT, p3=True, precision=I.IPCS_MIXED,
                        tol_ir=1e-10)
    _matrices_match(I, o, r, 1e-6)
    for step in range(3):
        r.advance(1)
        o.step()
        errs = field_errors(o, r)
        print("  mixed step", step, errs, flush=True)
        assert max(errs[:3]) <= 3e-6 and errs[3] <= 6e-5, (step, errs)


def test_p3_tet_fused_and_two_kernel_poisson_forms_agree():
    torch, I = require_gpu()
    print("P3-P2 tetrahedra fused vs two-kernel", flush=True)
    m = I.Mesh.unit_cube(8, pair=I.IPCS_PAIR_P3P2)
    out = []
    for rows in (0, -1):
        p = I.ipcs_params_default(nu=NU, dt=DT, tol_p=1e-13, poisson_part_rows=rows)
        r = I.Run(m, p)
        r.set_builtin(I.IPCS_SOL_BELTRAMI_3D)
        r.advance(2)
        out.append(r)
    a, b = out
    assert a.poisson_partition()["rows_max"] > 0 and b.poisson_partition()["rows_max"] == 0
    for c in range(3):
        assert rel(a.velocity()[c], b.velocity()[c]) <= FIELD_TOL
    assert rel(a.pressure(), b.pressure()) <= FIELD_TOL


@pytest.mark.parametrize("rows", [0, -1])
@pytest.mark.parametrize("n", [1, 2])
def test_p3_tet_degenerate_small_meshes(n, rows):
    """One or two cubes per direction: at n = 1 the only interior velocity
    nodes are the two nodes of the main diagonal and the six nodes of the
    interior faces (8 of 64), and the P2 pressure system has 27 rows in one
    part. Three Beltrami
    steps against the oracle in both Poisson CG forms (fields that vanish up to
    rounding are compared with an RMS floor of 0.01, as for the other pairs)."""
    torch, I = require_gpu()
    print(f"P3-P2 tetrahedra degenerate n={n} poisson_part_rows={rows}", flush=True)
    S, o, r = make_pair(I, 3, n, "beltrami", NU, DT, p3=True, poisson_part_rows=rows)

    def err(a, b):
        return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-2 * np.sqrt(b.size))

    for step in range(3):
        st = r.advance(1)[0]
        o.step()
        U, P = r.velocity(), r.pressure()
        errs = [err(U[c], o.U[c]) for c in range(3)] + [err(P, o.P)]
        assert max(errs) <= FIELD_TOL, (step, errs, st)
