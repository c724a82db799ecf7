"""Helpers shared by the GPU tests: build matching oracle / library runs and
compare them. Nothing here computes any part of the method."""
import numpy as np
import pytest

from oracle import fem, ipcs, mesh, problems


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_25403_amd import ipcs as I
    return torch, I


def oracle_problem(kind, dim, nu, k=np.pi):
    if kind == "tg":
        return problems.TaylorGreen2D(k, nu)
    if kind == "john":
        return problems.John2D(nu)
    if kind == "beltrami":
        return problems.Beltrami3D(nu=nu)
    if kind == "poly":
        return problems.PolySteady2D(nu) if dim == 2 else problems.PolySteady3D(nu)
    if kind == "cubic":
        return problems.PolySteady2DCubic(nu)
    raise KeyError(kind)


def builtin_kind(I, kind, dim):
    return {"tg": I.IPCS_SOL_TAYLOR_GREEN_2D, "john": I.IPCS_SOL_JOHN_2D,
            "beltrami": I.IPCS_SOL_BELTRAMI_3D,
            "poly": I.IPCS_SOL_POLY_STEADY_2D if dim == 2 else I.IPCS_SOL_POLY_STEADY_3D,
            "cubic": I.IPCS_SOL_POLY_CUBIC_2D}[kind]


def oracle_space(dim, n, order=2):
    return fem.Space(*(mesh.unit_square(n, n) if dim == 2 else mesh.unit_cube(n, n, n)),
                     order=order)


def make_pair(I, dim, n, kind, nu, dt, tol=1e-13, k=np.pi, t0=0.0, same_state=True,
              arrays=None, semi=False, chorin=False, p3=False, **kw):
    """Oracle IPCS object and library run for the same problem. With
    same_state the library starts from the oracle's initial arrays. arrays =
    (x, cells) replaces the structured n-mesh by that mesh on both sides; semi
    selects the semi-implicit convection form, chorin the Chorin-Temam
    projection and p3 the P3-P2 pair (triangles) on both sides."""
    order = 3 if p3 else 2
    pair = I.IPCS_PAIR_P3P2 if p3 else I.IPCS_PAIR_P2P1
    if arrays is None:
        S = oracle_space(dim, n, order)
        m = I.Mesh.unit_square(n, pair=pair) if dim == 2 else I.Mesh.unit_cube(n)
    else:
        S = fem.Space(*arrays, order=order)
        m = I.Mesh.from_arrays(*arrays, pair=pair)
    pb = oracle_problem(kind, dim, nu, k)
    o = ipcs.IPCS(S, pb, ipcs.Params(nu=nu, dt=dt, t0=t0, tol_mom=tol, tol_p=tol,
                                     tol_corr=tol, semi_implicit=semi, chorin=chorin))
    if semi:
        kw["convection"] = I.IPCS_CONV_SEMI_IMPLICIT
    if chorin:
        kw["scheme"] = I.IPCS_SCHEME_CHORIN
    p = I.ipcs_params_default(nu=nu, dt=dt, t0=t0, tol_mom=tol, tol_p=tol, tol_corr=tol, **kw)
    r = I.Run(m, p)
    prm = (k,) if kind == "tg" else ()
    r.set_builtin(builtin_kind(I, kind, dim), prm)
    if same_state:
        r.set_state(o.U, o.P, o.t)
    return S, o, r


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def field_errors(o, r):
    U, P = r.velocity(), r.pressure()
    return [rel(U[c], o.U[c]) for c in range(o.S.dim)] + [rel(P, o.P)]


def mat_rel(Agpu, Aor):
    """max |dA| / max |A| on identical patterns (patterns compared exactly)."""
    np.testing.assert_array_equal(Agpu.indptr, Aor.indptr)
    np.testing.assert_array_equal(Agpu.indices, Aor.indices)
    return np.abs(Agpu.data - Aor.data).max() / np.abs(Aor.data).max()
