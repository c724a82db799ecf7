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
        return problems.PolySteady2DCubic(nu) if dim == 2 else problems.PolySteady3DCubic(nu)
    raise KeyError(kind)


def builtin_kind(I, kind, dim):
    return {"tg": I.IPCS_SOL_TAYLOR_GREEN_2D, "john": I.IPCS_SOL_JOHN_2D,
            "beltrami": I.IPCS_SOL_BELTRAMI_3D,
            "poly": I.IPCS_SOL_POLY_STEADY_2D if dim == 2 else I.IPCS_SOL_POLY_STEADY_3D,
            "cubic": I.IPCS_SOL_POLY_CUBIC_2D if dim == 2 else I.IPCS_SOL_POLY_CUBIC_3D}[kind]


def oracle_space(dim, n, order=2):
    return fem.Space(*(mesh.unit_square(n, n) if dim == 2 else mesh.unit_cube(n, n, n)),
                     order=order)


def make_pair(I, dim, n, kind, nu, dt, tol=1e-13, k=np.pi, t0=0.0, same_state=True,
              arrays=None, semi=False, chorin=False, p3=False, **kw):
    """Oracle IPCS object and library run for the same problem. With
    same_state the library starts from the oracle's initial arrays. arrays =
    (x, cells) replaces the structured n-mesh by that mesh on both sides; semi
    selects the semi-implicit convection form, chorin the Chorin-Temam
    projection and p3 the P3-P2 pair on both sides."""
    order = 3 if p3 else 2
    pair = I.IPCS_PAIR_P3P2 if p3 else I.IPCS_PAIR_P2P1
    if arrays is None:
        S = oracle_space(dim, n, order)
        m = I.Mesh.unit_square(n, pair=pair) if dim == 2 else I.Mesh.unit_cube(n, pair=pair)
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
    """Relative difference of a field from its reference, in norm and per
    entry: the larger of ||a - b|| / ||b|| and max|a - b| / max|b|, so that an
    error confined to a few rows (a part halo, a boundary row) cannot hide
    under the norm."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    nb, mb = np.linalg.norm(b), np.abs(b).max(initial=0.0)
    d = a - b
    return max(np.linalg.norm(d) / (nb if nb > 0 else 1.0),
               np.abs(d).max(initial=0.0) / (mb if mb > 0 else 1.0))


def residual(A, x, b):
    """||b - A x|| / ||b|| of a candidate solution x on a given system."""
    nb = np.linalg.norm(b)
    return np.linalg.norm(b - A @ x) / (nb if nb > 0 else 1.0)


def step_residuals(I, o, r):
    """One library step, phase by phase, from the oracle's current state;
    each of the library's three solve outputs (U*, dP, U^{n+1}) is put into
    the oracle's own matrix of that sub-step, with the right-hand side formed
    from the library's inputs to it: the common state for the momentum
    system, the library's U* and dP for the correction. Returns relative
    residuals (bar: the solve tolerance, up to the rounding of b - A x), the
    largest deviation of the library's P^{n+1} - P^n from its dP, the check
    of the library's pressure right-hand side below, and the library's
    outputs. The oracle's state is unchanged.

    The pressure right-hand side r = -(rho/dt) sum_c D_c U*_c is a sum of
    terms far larger than itself (U* is close to discretely divergence-free:
    at 512^2 the summed magnitudes exceed |r| by ~1e7), so the last-bit
    differences of two correct evaluations move r by ~1e-9 relative. The
    library's dP is therefore put into the oracle's Kp with the library's own
    r, and that r is held against the oracle's sum over the library's U*
    entry by entry, relative to the rounding scale of the sum (the summed
    magnitudes (rho/dt) sum_c |D_c| |U*_c| plus their mean, for the
    projection to zero sum)."""
    dim, dt = o.S.dim, o.prm.dt
    t1 = o.t + dt
    g = o.dirichlet(t1)
    res = {}
    r.phase(I.IPCS_PHASE_ASM)
    r.phase(I.IPCS_PHASE_MOMENTUM)
    Us = r.field(I.IPCS_FIELD_USTAR)
    A_el, bs, _, _, _ = o.momentum_system(t1, g)
    for c in range(dim):
        res[f"momentum{c}"] = residual(A_el, Us[c], bs[c])
    r.phase(I.IPCS_PHASE_PRESSURE)
    dP = r.field(I.IPCS_FIELD_DP)
    rp_lib = r.field(I.IPCS_FIELD_RHS_P)
    Kp, rp = o.pressure_system(Us)
    mag = (o.prm.rho / dt) * sum(abs(o.D[c]) @ np.abs(Us[c]) for c in range(dim))
    res["pressure_rhs"] = np.max(np.abs(rp_lib - rp) / (mag + mag.mean()))
    res["pressure"] = residual(Kp, dP, rp_lib)
    r.phase(I.IPCS_PHASE_CORRECTION)
    U = r.velocity()
    M_el, bc = o.correction_system(Us, dP, g)
    for c in range(dim):
        res[f"correction{c}"] = residual(M_el, U[c], bc[c])
    P = r.pressure()
    res["p_update"] = np.abs((P - o.P) - dP).max() / max(np.abs(dP).max(), 1e-300)
    return res, Us, dP, U, P


def field_errors(o, r):
    U, P = r.velocity(), r.pressure()
    return [rel(U[c], o.U[c]) for c in range(o.S.dim)] + [rel(P, o.P)]


def mat_rel(Agpu, Aor):
    """max |dA| / max |A| on identical patterns (patterns compared exactly)."""
    np.testing.assert_array_equal(Agpu.indptr, Aor.indptr)
    np.testing.assert_array_equal(Agpu.indices, Aor.indices)
    return np.abs(Agpu.data - Aor.data).max() / np.abs(Aor.data).max()
