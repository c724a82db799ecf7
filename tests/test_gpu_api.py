"""The C ABI's behaviour on the GPU beyond parity: failures leave the state at
the last completed step, phase order is enforced, a failing run in a batch
does not disturb the others, results are deterministic and resumable, and
host callbacks give the built-in data's results."""
import numpy as np
import pytest

from oracle import problems
from tests.gpu_common import rel, require_gpu

pytestmark = pytest.mark.gpu


def tg_run(I, n=12, k=np.pi, nu=0.01, dt=0.01, stream=None, **kw):
    p = I.ipcs_params_default(nu=nu, dt=dt, **kw)
    r = I.Run(I.Mesh.unit_square(n), p, stream=stream)
    r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (k,))
    return r


def test_maxit_failure_keeps_last_completed_step():
    torch, I = require_gpu()
    print("maxit failure", flush=True)
    r = tg_run(I, maxit=3)
    U0, P0, t0 = r.velocity().copy(), r.pressure().copy(), r.time()
    with pytest.raises(I.IpcsError) as e:
        r.advance(1)
    assert e.value.code == I.IPCS_E_NOT_CONVERGED
    st = e.value.stats[0]
    assert st.status == I.IPCS_E_NOT_CONVERGED and st.failed_solve in (1, 2, 3)
    np.testing.assert_array_equal(r.velocity(), U0)
    np.testing.assert_array_equal(r.pressure(), P0)
    assert r.time() == t0


def test_nonfinite_state_is_reported():
    torch, I = require_gpu()
    print("nonfinite", flush=True)
    r = tg_run(I)
    U, P = r.velocity().copy(), r.pressure().copy()
    U[0, 5] = np.nan
    r.set_state(U, P, 0.0)
    with pytest.raises(I.IpcsError) as e:
        r.advance(1)
    assert e.value.code == I.IPCS_E_NONFINITE
    assert r.time() == 0.0


def test_phase_order_is_enforced():
    torch, I = require_gpu()
    print("phase order", flush=True)
    r = tg_run(I)
    with pytest.raises(I.IpcsError) as e:
        r.phase(I.IPCS_PHASE_PRESSURE)
    assert e.value.code == I.IPCS_E_STATE
    r.phase(I.IPCS_PHASE_ASM)
    with pytest.raises(I.IpcsError) as e:
        r.advance(1)          # a step is in progress
    assert e.value.code == I.IPCS_E_STATE
    for ph in (I.IPCS_PHASE_MOMENTUM, I.IPCS_PHASE_PRESSURE, I.IPCS_PHASE_CORRECTION):
        r.phase(ph)
    r.advance(1)
    assert abs(r.time() - 0.02) < 1e-15


def test_batch_failure_is_isolated():
    torch, I = require_gpu()
    print("batch failure isolation", flush=True)
    s = torch.cuda.Stream()
    good = tg_run(I, n=10, stream=s)
    bad = tg_run(I, n=14, maxit=2, stream=s)
    ref = tg_run(I, n=10)
    ref.advance(2)
    U0, t0 = bad.velocity().copy(), bad.time()
    for _ in range(2):
        rc, st = I.ipcs_batch_step([good.h, bad.h], s.cuda_stream)
        assert rc == I.IPCS_E_NOT_CONVERGED
        assert st[0]["status"] == 0 and st[1]["status"] == I.IPCS_E_NOT_CONVERGED
    np.testing.assert_array_equal(good.velocity(), ref.velocity())
    np.testing.assert_array_equal(good.pressure(), ref.pressure())
    np.testing.assert_array_equal(bad.velocity(), U0)
    assert bad.time() == t0


@pytest.mark.parametrize("mstart", ["state", "extrapolated"])
def test_runs_are_deterministic_and_resumable(mstart):
    """Runs of the same problem are bitwise equal. With the momentum solve
    started from U^n a step is a function of the state alone, so a run
    resumed through the host is bitwise the uninterrupted one; with the
    extrapolated start (the default) the resumed run's first two steps start
    from U^n, and it stays within the parity bar of the uninterrupted run."""
    torch, I = require_gpu()
    print(f"determinism and resume, momentum start {mstart}", flush=True)
    ms = I.IPCS_MSTART_STATE if mstart == "state" else I.IPCS_MSTART_EXTRAPOLATED

    def run():
        return tg_run(I, n=20, k=2 * np.pi, nu=0.004, dt=0.003, momentum_start=ms)

    a, b = run(), run()
    a.advance(6)
    b.advance(4)
    U, P, t = b.velocity(), b.pressure(), b.time()
    c = run()
    c.set_state(U, P, t)          # checkpoint / resume through the host
    b.advance(2)
    c.advance(2)
    np.testing.assert_array_equal(b.velocity(), a.velocity())
    np.testing.assert_array_equal(b.pressure(), a.pressure())
    assert b.time() == a.time() == c.time()
    if mstart == "state":
        np.testing.assert_array_equal(c.velocity(), a.velocity())
        np.testing.assert_array_equal(c.pressure(), a.pressure())
    else:
        eu, ep = rel(c.velocity(), a.velocity()), rel(c.pressure(), a.pressure())
        print(f"resumed against uninterrupted: u {eu:.2e} p {ep:.2e}", flush=True)
        assert eu <= 1e-10 and ep <= 1e-10, (eu, ep)


def test_set_time_step_matches_a_fresh_run():
    """A new time step re-forms A = M/dt + nu K and clears the solve-start
    history (an extrapolation needs equal steps): after five steps at
    dt = 0.003 (the quadratic momentum start in use) and a change to 0.002,
    the run is bitwise a fresh run at 0.002 started from the same state,
    with both history starts on."""
    torch, I = require_gpu()
    print("set_time_step", flush=True)
    kw = dict(n=16, k=2 * np.pi, nu=0.004, poisson_start=I.IPCS_START_PREVIOUS)
    a = tg_run(I, dt=0.003, **kw)
    a.advance(5)
    I.ipcs_set_time_step(a.h, 0.002)
    b = tg_run(I, dt=0.002, **kw)
    b.set_state(a.velocity(), a.pressure(), a.time())
    sa, sb = a.advance(4), b.advance(4)
    np.testing.assert_array_equal(a.velocity(), b.velocity())
    np.testing.assert_array_equal(a.pressure(), b.pressure())
    assert [s["it_mom"] for s in sa] == [s["it_mom"] for s in sb]
    assert a.time() == b.time()


def test_set_viscosity_matches_a_fresh_run():
    torch, I = require_gpu()
    print("set_viscosity", flush=True)
    a = tg_run(I, n=16, nu=0.01)
    a.advance(2)
    I.ipcs_set_viscosity(a.h, 0.03)
    b = tg_run(I, n=16, nu=0.03)
    b.set_state(a.velocity(), a.pressure(), a.time())
    # the built-in data (Dirichlet values) follow the run's own viscosity
    a.advance(2)
    b.advance(2)
    np.testing.assert_array_equal(a.velocity(), b.velocity())
    np.testing.assert_array_equal(a.pressure(), b.pressure())


def test_host_callbacks_match_builtin_data():
    """John's forced problem: forcing and Dirichlet data from host callbacks
    (quadrature points and boundary nodes) against the built-in closed forms."""
    torch, I = require_gpu()
    print("callbacks", flush=True)
    pb = problems.John2D(1.0)
    m = I.Mesh.unit_square(12)
    p = I.ipcs_params_default(nu=1.0, dt=0.002, callbacks=1)
    a = I.Run(m, p)
    a.set_builtin(I.IPCS_SOL_JOHN_2D)
    U0, P0 = a.velocity().copy(), a.pressure().copy()
    b = I.Run(m, p)
    b.set_state(U0, P0, 0.0)
    b.set_dirichlet(lambda x, t: pb.u(x, t))
    b.set_forcing(lambda x, t: pb.f(x, t))
    a.advance(3)
    b.advance(3)
    assert rel(b.velocity(), a.velocity()) <= 1e-12
    assert rel(b.pressure(), a.pressure()) <= 1e-10


@pytest.mark.parametrize("rows", [0, -1])
def test_unreachable_tolerance_stops_early(rows):
    """A tolerance below what FP64 can attain: the solve ends with an error
    long before maxit (20000) and the state stays at the last completed step.
    Either the recursive residual gets there and three restarts in a row
    bring the true residual no 10% below its best (NOT_CONVERGED), or the CG
    scalars lose positivity at the rounding level first (BREAKDOWN)."""
    torch, I = require_gpu()
    print(f"unreachable tolerance (poisson_part_rows={rows})", flush=True)
    r = tg_run(I, n=24, tol_p=1e-15, poisson_part_rows=rows)
    U0 = r.velocity().copy()
    with pytest.raises(I.IpcsError) as e:
        r.advance(1)
    assert e.value.code in (I.IPCS_E_NOT_CONVERGED, I.IPCS_E_BREAKDOWN)
    st = e.value.stats[0]
    print(e.value.code, st.checks_p, st.it_p, flush=True)
    assert st.failed_solve == 2 and 0 < st.it_p < 5000, (st.checks_p, st.it_p)
    if e.value.code == I.IPCS_E_NOT_CONVERGED:
        assert st.checks_p >= 3
    np.testing.assert_array_equal(r.velocity(), U0)


@pytest.mark.parametrize("pair,arrays", [(0, False), (0, True), (1, False)])
def test_state_round_trip_in_interface_numbering(pair, arrays):
    """set_state then velocity()/pressure() give back the arrays bit for bit,
    and the velocity the library interpolates itself sits at the interface
    numbering's node coordinates (the library renumbers internally)."""
    torch, I = require_gpu()
    print(f"state round trip pair={pair} arrays={arrays}", flush=True)
    from paper_2605_25403_amd.workloads import jittered_mesh
    if arrays:
        x, cells = jittered_mesh(2, 9, 3)
        m = I.Mesh.from_arrays(x, cells, pair=pair)
    else:
        m = I.Mesh.unit_square(7, pair=pair)
    r = I.Run(m, I.ipcs_params_default(nu=0.01, dt=0.01))
    c = I.ipcs_mesh_counts(m.h)
    rng = np.random.default_rng(5)
    U = rng.standard_normal((2, c.n2))
    P = rng.standard_normal(c.n1)
    r.set_state(U, P, 0.25)
    np.testing.assert_array_equal(r.velocity(), U)
    np.testing.assert_array_equal(r.pressure(), P)
    k = np.pi
    r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (k,))
    X = I.ipcs_mesh_dof_coords(m.h, I.IPCS_SPACE_P2).reshape(-1, 2)
    want = problems.TaylorGreen2D(k, 0.01).u(X, r.time())       # [n2, 2]
    assert np.abs(r.velocity() - want.T).max() < 1e-12
