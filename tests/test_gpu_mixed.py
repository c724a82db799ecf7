"""The mixed-precision form on the GPU, through the C ABI.

FP32 quadrature, assembly arithmetic and matrix values; FP64 fields, Krylov
vectors, sums and the iterative refinement of the pressure Poisson solve
(||r - Kp dP|| <= tol_ir ||r|| with the FP64 Kp). No oracle computes this form
(its exact result depends on FP32 rounding); the reference is the FP64 oracle
and the bars are the stated error bounds of the form:
* matrices: max|dA| / max|A| <= 1e-6 (FP32 rounding of sums of at most a few
  hundred products, each exact to 2^-24);
* fields, per step: ||dx|| / ||x|| <= 1e-5 per velocity component and for the
  pressure, against the FP64 oracle from the same initial state;
* the Poisson refinement reaches tol_ir = 1e-10 on the FP64 operator, checked
  here with the oracle's own FP64 Kp.
"""
import numpy as np
import pytest

from oracle import fem
from tests.gpu_common import field_errors, make_pair, mat_rel, rel, require_gpu

pytestmark = pytest.mark.gpu

MIX_MAT_TOL = 1e-6
MIX_FIELD_TOL = 1e-5
TOL_IR = 1e-10


def mixed_pair(I, dim, n, kind, nu, dt, **kw):
    return make_pair(I, dim, n, kind, nu, dt, precision=I.IPCS_MIXED, tol_ir=TOL_IR, **kw)


@pytest.mark.parametrize("dim,n,p3", [(2, 16, False), (3, 3, False), (2, 8, True), (3, 2, True)])
def test_mixed_matrices_within_fp32_bound(dim, n, p3):
    """The constant matrices and the convection matrix E = M/dt - C(U) of the
    first step (in 3D and for P3-P2 formed by the two-pass assembly: FP32
    matrix cores for P2 tetrahedra and P3 triangles) within the FP32 bound."""
    torch, I = require_gpu()
    print(f"mixed matrices dim={dim} n={n} p3={p3}", flush=True)
    kind = "tg" if dim == 2 else "beltrami"
    S, o, r = mixed_pair(I, dim, n, kind, 0.013, 0.007, p3=p3)
    errs = {"M": mat_rel(r.matrix(I.IPCS_MAT_M), o.M),
            "K": mat_rel(r.matrix(I.IPCS_MAT_K), o.K),
            "Kp": mat_rel(r.matrix(I.IPCS_MAT_KP), o.Kp),
            "A": mat_rel(r.matrix(I.IPCS_MAT_A_ELIM), o.A_el)}
    for c in range(dim):
        errs[f"D{c}"] = mat_rel(r.matrix(I.IPCS_MAT_D0 + c), o.D[c])
        errs[f"G{c}"] = mat_rel(r.matrix(I.IPCS_MAT_G0 + c), o.G[c])
    r.phase(I.IPCS_PHASE_ASM)
    E = (o.M / o.prm.dt - fem.convection(S, o.U)).tocsr()
    E.sort_indices()
    errs["E"] = mat_rel(r.matrix(I.IPCS_MAT_E), E)
    print(errs, flush=True)
    assert max(errs.values()) <= MIX_MAT_TOL, errs
    # the values really are FP32: exactly representable in single precision
    v = r.matrix(I.IPCS_MAT_M).data
    np.testing.assert_array_equal(v.astype(np.float32).astype(np.float64), v)


def test_mixed_c1_ten_steps_within_bound():
    """C1 (16 x 16 TG, k = pi, nu = 0.01, dt = 0.01, 10 steps) in mixed form."""
    torch, I = require_gpu()
    print("mixed C1 ten steps", flush=True)
    S, o, r = mixed_pair(I, 2, 16, "tg", 0.01, 0.01, same_state=False)
    worst = 0.0
    for step in range(10):
        st = r.advance(1)[0]
        o.step()
        errs = field_errors(o, r)
        worst = max(worst, max(errs))
        assert max(errs) <= MIX_FIELD_TOL, (step, errs, st)
        assert st["status"] == 0 and st["ir_outer"] >= 1 and st["res_p"] <= TOL_IR, st
    print(f"worst field error over 10 steps {worst:.3e}", flush=True)


def test_mixed_refinement_reaches_fp64_tolerance():
    """After the pressure phase the increment solves the FP64 system to
    tol_ir, measured with the oracle's FP64 Kp."""
    torch, I = require_gpu()
    print("mixed IR residual", flush=True)
    S, o, r = mixed_pair(I, 2, 24, "tg", 0.005, 0.004)
    r.phase(I.IPCS_PHASE_ASM)
    r.phase(I.IPCS_PHASE_MOMENTUM)
    r.phase(I.IPCS_PHASE_PRESSURE)
    rhs = r.field(I.IPCS_FIELD_RHS_P)
    dP = r.field(I.IPCS_FIELD_DP)
    res = rhs - o.Kp @ dP
    res -= res.mean()
    assert np.linalg.norm(res) <= 2 * TOL_IR * np.linalg.norm(rhs), \
        np.linalg.norm(res) / np.linalg.norm(rhs)
    r.phase(I.IPCS_PHASE_CORRECTION)


def test_mixed_beltrami_3d_steps_within_bound():
    torch, I = require_gpu()
    print("mixed Beltrami 3D n=4", flush=True)
    S, o, r = mixed_pair(I, 3, 4, "beltrami", 0.01, 0.01)
    for step in range(3):
        r.advance(1)
        o.step()
        errs = field_errors(o, r)
        assert max(errs) <= MIX_FIELD_TOL, (step, errs)


def test_mixed_close_to_fp64_form_on_larger_mesh():
    """64 x 64 TG, 3 steps: mixed vs the FP64 form of the library, same start."""
    torch, I = require_gpu()
    print("mixed vs fp64 n=64", flush=True)
    k, nu, dt = 2 * np.pi, 0.004, 1e-3
    m = I.Mesh.unit_square(64)
    runs = []
    for prec in (I.IPCS_FP64, I.IPCS_MIXED):
        p = I.ipcs_params_default(nu=nu, dt=dt, precision=prec, tol_ir=TOL_IR)
        r = I.Run(m, p)
        r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (k,))
        r.advance(3)
        runs.append(r)
    U64, U32 = runs[0].velocity(), runs[1].velocity()
    P64, P32 = runs[0].pressure(), runs[1].pressure()
    errs = [rel(U32[c], U64[c]) for c in range(2)] + [rel(P32, P64)]
    print(errs, flush=True)
    assert max(errs) <= MIX_FIELD_TOL, errs
