"""Semi-implicit convection (the convection operator at u^n moved into the
momentum matrix, A^n = M/dt + nu K + C(U^n), re-formed and re-eliminated every
step) on the GPU against the oracle's semi-implicit IPCS. Bars as for the
explicit form: matrices max|dA|/max|A| <= 1e-12, fields ||dx||/||x|| <= 1e-10
per component and for the pressure; the mixed form within its stated 1e-5."""
import numpy as np
import pytest

from oracle import fem
from tests.gpu_common import field_errors, make_pair, mat_rel, rel, require_gpu

pytestmark = pytest.mark.gpu

MAT_TOL = 1e-12
FIELD_TOL = 1e-10


@pytest.mark.parametrize("dim,n,kind", [(2, 16, "tg"), (2, 7, "john"), (3, 3, "beltrami")])
def test_semi_matrix_and_rhs(dim, n, kind):
    torch, I = require_gpu()
    print(f"semi matrix/rhs dim={dim} n={n} {kind}", flush=True)
    nu, dt = 0.02, 0.01
    S, o, r = make_pair(I, dim, n, kind, nu, dt, semi=True)
    r.phase(I.IPCS_PHASE_ASM)
    C = fem.convection(S, o.U)
    E = (o.M / dt + C).tocsr()
    E.sort_indices()
    assert mat_rel(r.matrix(I.IPCS_MAT_E), E) <= MAT_TOL
    A = (o.A + C).tocsr()
    A.sort_indices()
    assert mat_rel(r.matrix(I.IPCS_MAT_A_ELIM), fem.eliminate(A, o.bmask)) <= MAT_TOL
    t1 = o.t + dt
    g = o.dirichlet(t1)
    F = o.forcing(t1)
    b = r.field(I.IPCS_FIELD_RHS_MOM)
    for c in range(dim):
        ref = o.M @ o.U[c] / dt - o.G[c] @ o.P + F[c]
        ref = fem.lift(A, ref, o.bmask, g[c])
        assert rel(b[c], ref) <= MAT_TOL


@pytest.mark.parametrize("dim,n,kind", [(2, 16, "tg"), (2, 9, "john"), (3, 3, "beltrami")])
def test_semi_substeps_and_steps(dim, n, kind):
    torch, I = require_gpu()
    print(f"semi steps dim={dim} n={n} {kind}", flush=True)
    nu, dt = (1.0, 0.002) if kind == "john" else (0.01, 0.01)
    S, o, r = make_pair(I, dim, n, kind, nu, dt, semi=True)
    t1 = o.t + dt
    g = o.dirichlet(t1)
    r.phase(I.IPCS_PHASE_ASM)
    st = r.phase(I.IPCS_PHASE_MOMENTUM)
    Us_o, _, _ = o.momentum(t1, g)
    Us = r.field(I.IPCS_FIELD_USTAR)
    assert max(rel(Us[c], Us_o[c]) for c in range(dim)) <= FIELD_TOL, st
    r.phase(I.IPCS_PHASE_PRESSURE)
    dP_o, _ = o.pressure(Us_o)
    assert rel(r.field(I.IPCS_FIELD_DP), dP_o) <= FIELD_TOL
    r.phase(I.IPCS_PHASE_CORRECTION)
    o.step()
    assert max(field_errors(o, r)) <= FIELD_TOL
    for step in range(3):
        st = r.advance(1)[0]
        o.step()
        errs = field_errors(o, r)
        assert max(errs) <= FIELD_TOL, (step, errs, st)


def test_semi_c1_ten_steps_and_mixed():
    """C1 (16 x 16 TG, k = pi, nu = 0.01, dt = 0.01, 10 steps) in the
    semi-implicit form, FP64 to 1e-10 and mixed to 1e-5 against the oracle."""
    torch, I = require_gpu()
    print("semi C1 ten steps, FP64 and mixed", flush=True)
    S, o, r = make_pair(I, 2, 16, "tg", 0.01, 0.01, same_state=False, semi=True)
    _, _, rm = make_pair(I, 2, 16, "tg", 0.01, 0.01, same_state=False, semi=True,
                         precision=I.IPCS_MIXED, tol_ir=1e-10)
    for step in range(10):
        st = r.advance(1)[0]
        rm.advance(1)
        o.step()
        assert max(field_errors(o, r)) <= FIELD_TOL, (step, st)
        assert max(field_errors(o, rm)) <= 1e-5, step


def test_semi_and_explicit_share_a_batch_bitwise():
    torch, I = require_gpu()
    print("batch with both convection forms", flush=True)
    cases = [(12, I.IPCS_CONV_SEMI_IMPLICIT, I.IPCS_FP64), (12, I.IPCS_CONV_EXPLICIT, I.IPCS_FP64),
             (16, I.IPCS_CONV_SEMI_IMPLICIT, I.IPCS_MIXED)]

    def mk(n, conv, prec, stream=None):
        p = I.ipcs_params_default(nu=0.01, dt=0.005, precision=prec, tol_ir=1e-10,
                                  convection=conv)
        r = I.Run(I.Mesh.unit_square(n), p, stream=stream)
        r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (np.pi,))
        return r

    alone = []
    for c in cases:
        r = mk(*c)
        r.advance(2)
        alone.append((r.velocity(), r.pressure()))
    s = torch.cuda.Stream()
    runs = [mk(*c, stream=s) for c in cases]
    for _ in range(2):
        rc, st = I.ipcs_batch_step([r.h for r in runs], s.cuda_stream)
        assert rc == I.IPCS_OK, st
    for (U, P), r in zip(alone, runs):
        np.testing.assert_array_equal(r.velocity(), U)
        np.testing.assert_array_equal(r.pressure(), P)


def test_semi_viscosity_change_matches_fresh_run():
    torch, I = require_gpu()
    print("semi set_viscosity", flush=True)
    kw = dict(convection=I.IPCS_CONV_SEMI_IMPLICIT)
    a = I.Run(I.Mesh.unit_square(16), I.ipcs_params_default(nu=0.01, dt=0.01, **kw))
    a.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (np.pi,))
    a.advance(2)
    I.ipcs_set_viscosity(a.h, 0.03)
    b = I.Run(I.Mesh.unit_square(16), I.ipcs_params_default(nu=0.03, dt=0.01, **kw))
    b.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (np.pi,))
    b.set_state(a.velocity(), a.pressure(), a.time())
    a.advance(2)
    b.advance(2)
    np.testing.assert_array_equal(a.velocity(), b.velocity())
    np.testing.assert_array_equal(a.pressure(), b.pressure())
