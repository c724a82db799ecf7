"""L2 errors of discrete fields against exact ones (oracle, reporting only).

Used the way the paper's convergence tables use them (Section 4.2 and
Section 5.1): ||u - u_h||_{L2} over all velocity components and
||p - p_h||_{L2} with the integral means of p and p_h removed (the pressure
is only determined up to a constant).
"""
import numpy as np

from . import quadrature


def _rule(space):
    return quadrature.error_rule(space.dim)


def l2_velocity(space, U, u_exact, t):
    lam, w = _rule(space)
    phi, _ = space.basis_u(lam)
    xq = space.map_points(lam)
    uex = u_exact(xq, t)                                          # (Nc, nq, d)
    uh = np.einsum('qm,acm->cqa', phi, U[:, space.c2du])
    e2 = np.einsum('q,c,cqa->', w, space.absdet, (uex - uh) ** 2)
    return float(np.sqrt(e2))


def l2_pressure(space, P, p_exact, t):
    lam, w = _rule(space)
    psi, _ = space.basis_p(lam)
    xq = space.map_points(lam)
    pex = p_exact(xq, t)
    ph = np.einsum('qm,cm->cq', psi, P[space.c2dp])
    wq = np.einsum('q,c->cq', w, space.absdet)
    vol = wq.sum()
    diff = (pex - (wq * pex).sum() / vol) - (ph - (wq * ph).sum() / vol)
    return float(np.sqrt((wq * diff ** 2).sum()))
