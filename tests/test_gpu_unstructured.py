"""GPU parity on unstructured meshes: interior vertices moved at random,
vertices relabelled, cells reordered and half of them of opposite orientation.
Geometry then differs from cell to cell, matrix rows have irregular lengths and
column indices are scattered, which the structured meshes do not exercise.
Both Taylor-Hood pairs: with P3-P2 the convection assembly takes its two-pass
form (the matrix-core cell pass on triangles, the per-thread one on
tetrahedra), whose cell batches then hold cells of every shape and orientation
and end in a ragged last batch.
Bars as for the structured meshes: matrices max|dA|/max|A| <= 1e-12, fields
||dx||/||x|| <= 1e-10 per component and for the pressure, per step."""
import numpy as np
import pytest

from oracle import fem
from paper_2605_25403_amd.workloads import jittered_mesh
from tests.gpu_common import field_errors, make_pair, mat_rel, rel, require_gpu

pytestmark = pytest.mark.gpu

MAT_TOL = 1e-12
FIELD_TOL = 1e-10
# (dim, n, seed, P3-P2 pair)
CASES = [(2, 9, 0, False), (2, 21, 4, False), (3, 3, 1, False), (2, 7, 2, True),
         (3, 2, 3, True)]


def pair(I, dim, n, seed, nu, dt, p3=False, **kw):
    kind = "tg" if dim == 2 else "beltrami"
    return make_pair(I, dim, n, kind, nu, dt, arrays=jittered_mesh(dim, n, seed), p3=p3, **kw)


@pytest.mark.parametrize("dim,n,seed,p3", CASES)
def test_unstructured_matrices(dim, n, seed, p3):
    torch, I = require_gpu()
    print(f"unstructured matrices dim={dim} n={n} seed={seed} p3={p3}", flush=True)
    S, o, r = pair(I, dim, n, seed, 0.013, 0.007, p3=p3)
    errs = {"M": mat_rel(r.matrix(I.IPCS_MAT_M), o.M),
            "K": mat_rel(r.matrix(I.IPCS_MAT_K), o.K),
            "Kp": mat_rel(r.matrix(I.IPCS_MAT_KP), o.Kp),
            "A": mat_rel(r.matrix(I.IPCS_MAT_A_ELIM), o.A_el),
            "Mel": mat_rel(r.matrix(I.IPCS_MAT_M_ELIM), o.M_el)}
    for c in range(dim):
        errs[f"D{c}"] = mat_rel(r.matrix(I.IPCS_MAT_D0 + c), o.D[c])
        errs[f"G{c}"] = mat_rel(r.matrix(I.IPCS_MAT_G0 + c), o.G[c])
    r.phase(I.IPCS_PHASE_ASM)
    E = (o.M / o.prm.dt - fem.convection(S, o.U)).tocsr()
    E.sort_indices()
    errs["E"] = mat_rel(r.matrix(I.IPCS_MAT_E), E)
    assert max(errs.values()) <= MAT_TOL, errs


@pytest.mark.parametrize("dim,n,seed,p3", CASES)
def test_unstructured_substeps_and_steps(dim, n, seed, p3):
    torch, I = require_gpu()
    print(f"unstructured steps dim={dim} n={n} seed={seed} p3={p3}", flush=True)
    dt = 0.01
    S, o, r = pair(I, dim, n, seed, 0.01, dt, p3=p3)
    t1 = o.t + dt
    g = o.dirichlet(t1)
    r.phase(I.IPCS_PHASE_ASM)
    r.phase(I.IPCS_PHASE_MOMENTUM)
    Us_o, _, _ = o.momentum(t1, g)
    Us = r.field(I.IPCS_FIELD_USTAR)
    assert max(rel(Us[c], Us_o[c]) for c in range(dim)) <= FIELD_TOL
    r.phase(I.IPCS_PHASE_PRESSURE)
    dP_o, _ = o.pressure(Us_o)
    assert rel(r.field(I.IPCS_FIELD_DP), dP_o) <= FIELD_TOL
    r.phase(I.IPCS_PHASE_CORRECTION)
    o.step()
    errs = field_errors(o, r)
    assert max(errs) <= FIELD_TOL, errs
    for step in range(2):
        st = r.advance(1)[0]
        o.step()
        errs = field_errors(o, r)
        assert max(errs) <= FIELD_TOL, (step, errs, st)
