"""GPU parity of the steady Navier-Stokes solver (Newton's method, P2-P1,
the monolithic system solved by flexible GMRES with a block-triangular
preconditioner) against the oracle's Newton iteration with sparse direct
solves (Section 2.2.1, Newton linearization; Section 4.2 example).

* the polynomial steady state is reproduced exactly (2D and 3D);
* Section 4.2's example at n = 4, 8, 16: the first step's residual equals
  the oracle's from the same start (entry by entry, 1e-12 of its largest
  entry); the increment solves the oracle's Newton matrix (relative residual
  1e-10: the linear tolerance 1e-12 plus the rounding of J x); both sides
  take the same number of steps, and the solutions agree to 1e-10 in norm
  and per entry.
"""
import numpy as np
import pytest

from oracle import fem, mesh, problems, steady
from tests.gpu_common import rel, require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,n", [(2, 6), (3, 2)])
def test_steady_polynomial_state_is_reproduced(dim, n):
    torch, I = require_gpu()
    print(f"steady polynomial dim={dim} n={n}", flush=True)
    nu = 0.3
    m = I.Mesh.unit_square(n) if dim == 2 else I.Mesh.unit_cube(n)
    s = I.Steady(m, nu=nu)
    s.set_builtin(I.IPCS_SOL_POLY_STEADY_2D if dim == 2 else I.IPCS_SOL_POLY_STEADY_3D)
    st = s.solve()
    print(st, flush=True)
    S = fem.Space(*(mesh.unit_square(n, n) if dim == 2 else mesh.unit_cube(n, n, n)))
    pb = problems.PolySteady2D(nu) if dim == 2 else problems.PolySteady3D(nu)
    U, P = s.velocity(), s.pressure()
    assert np.abs(U - pb.u(S.xu, 0.0).T).max() <= 1e-11
    assert np.abs(P - pb.p(S.xp, 0.0)).max() <= 1e-10
    assert st["newton_steps"] <= 5


@pytest.mark.parametrize("n", [4, 8, 16])
def test_steady_paper_example_against_oracle(n):
    torch, I = require_gpu()
    print(f"steady example n={n}", flush=True)
    nu = 1.0
    S = fem.Space(*mesh.unit_square(n, n))
    o = steady.SteadyNewton(S, problems.SteadyPaper2D(nu), nu)
    s = I.Steady(I.Mesh.unit_square(n), nu=nu)
    s.set_builtin(I.IPCS_SOL_STEADY_PAPER_2D)
    # first step from the common start
    Ru, Rp = o.residual()
    J = o.jacobian()
    st = s.step()
    gRu, gRp = s.vector(I.IPCS_STEADY_RESIDUAL)
    scale = max(np.abs(Ru).max(), np.abs(Rp).max())
    eR = max(np.abs(gRu - Ru).max(), np.abs(gRp - Rp).max()) / scale
    dU, dP = s.vector(I.IPCS_STEADY_INCREMENT)
    b = np.concatenate([Ru.ravel(), Rp])
    res = np.linalg.norm(b - J @ np.concatenate([dU.ravel(), dP])) / np.linalg.norm(b)
    print(f"step 1: residual diff {eR:.2e}, increment residual {res:.2e}", st, flush=True)
    assert eR <= 1e-12 and res <= 1e-10
    # the rest of the iteration on both sides
    o.step()
    o.run()
    st2 = s.solve()
    U, P = s.velocity(), s.pressure()
    eu = max(rel(U[c], o.U[c]) for c in range(2))
    ep = rel(P, o.P)
    print(f"final: u {eu:.2e} p {ep:.2e}, steps gpu {1 + st2['newton_steps']} oracle "
          f"{len(o.history)}", st2, o.history, flush=True)
    assert eu <= 1e-10 and ep <= 1e-10
    assert abs(1 + st2["newton_steps"] - len(o.history)) <= 1
