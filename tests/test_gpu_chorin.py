"""The Chorin-Temam projection (no pressure term in the momentum step, the
Poisson solve gives the new pressure itself) on the GPU against the oracle's
Chorin step. Bars as for IPCS: fields ||dx||/||x|| <= 1e-10 per component and
for the pressure, per step; the mixed form within its stated 1e-5."""
import numpy as np
import pytest

from tests.gpu_common import field_errors, make_pair, rel, require_gpu

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-10


@pytest.mark.parametrize("dim,n,kind,semi", [(2, 16, "tg", False), (2, 9, "john", False),
                                             (3, 3, "beltrami", False), (2, 12, "tg", True)])
def test_chorin_substeps_and_steps(dim, n, kind, semi):
    torch, I = require_gpu()
    print(f"chorin dim={dim} n={n} {kind} semi={semi}", flush=True)
    nu, dt = (1.0, 0.002) if kind == "john" else (0.01, 0.01)
    S, o, r = make_pair(I, dim, n, kind, nu, dt, chorin=True, semi=semi)
    t1 = o.t + dt
    g = o.dirichlet(t1)
    r.phase(I.IPCS_PHASE_ASM)
    r.phase(I.IPCS_PHASE_MOMENTUM)
    Us_o, _, _ = o.momentum(t1, g)
    Us = r.field(I.IPCS_FIELD_USTAR)
    assert max(rel(Us[c], Us_o[c]) for c in range(dim)) <= FIELD_TOL
    r.phase(I.IPCS_PHASE_PRESSURE)
    P_o, _ = o.pressure(Us_o)
    assert rel(r.field(I.IPCS_FIELD_DP), P_o) <= FIELD_TOL
    r.phase(I.IPCS_PHASE_CORRECTION)
    o.step()
    assert max(field_errors(o, r)) <= FIELD_TOL
    assert rel(r.pressure(), P_o) <= FIELD_TOL      # P^{n+1} is the solve's result
    for step in range(3):
        st = r.advance(1)[0]
        o.step()
        assert max(field_errors(o, r)) <= FIELD_TOL, (step, st)


def test_chorin_ignores_old_pressure_bitwise():
    torch, I = require_gpu()
    print("chorin independence from P^n", flush=True)
    S, o, a = make_pair(I, 2, 16, "tg", 0.01, 0.01, chorin=True)
    _, _, b = make_pair(I, 2, 16, "tg", 0.01, 0.01, chorin=True)
    rng = np.random.default_rng(5)
    b.set_state(o.U, rng.standard_normal(S.N1), o.t)
    a.advance(2)
    b.advance(2)
    np.testing.assert_array_equal(a.velocity(), b.velocity())
    np.testing.assert_array_equal(a.pressure(), b.pressure())


def test_chorin_mixed_and_batch():
    """Mixed form against the FP64 oracle (1e-5), and a batch that mixes the
    two schemes and precisions, bitwise equal to the runs alone."""
    torch, I = require_gpu()
    print("chorin mixed and batch", flush=True)
    S, o, rm = make_pair(I, 2, 16, "tg", 0.01, 0.01, same_state=False, chorin=True,
                         precision=I.IPCS_MIXED, tol_ir=1e-10)
    for step in range(5):
        rm.advance(1)
        o.step()
        assert max(field_errors(o, rm)) <= 1e-5, step
    cases = [(12, I.IPCS_SCHEME_CHORIN, I.IPCS_FP64), (12, I.IPCS_SCHEME_IPCS, I.IPCS_FP64),
             (16, I.IPCS_SCHEME_CHORIN, I.IPCS_MIXED)]

    def mk(n, scheme, prec, stream=None):
        p = I.ipcs_params_default(nu=0.01, dt=0.005, precision=prec, tol_ir=1e-10,
                                  scheme=scheme)
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
