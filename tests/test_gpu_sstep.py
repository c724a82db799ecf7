"""The two-iterations-per-launch Poisson CG (s-step CG with s = 2: a basis of
the matrix powers p, Bp, B^2p, z, Bz, one reduction of its D-weighted Gram
matrix per launch, two CG iterations in its coordinates; the part's second
halo ring in LDS) on the GPU, through the C ABI.

* Against the FP64 oracle, for part sizes that give many small parts with
  ragged last slices, halo rows in several slices and one part holding
  everything (no halo at all): the pressure increment of one step from an
  identical state, bar 1e-10 as for every field; triangles and tetrahedra.
* Against the one-iteration-per-launch form of the same library: in exact
  arithmetic both are Jacobi-PCG, so over three steps the fields agree to the
  solve tolerance and the total iteration counts to 5% (per step they scatter
  where a true-residual check restarts the iteration); FP64 and mixed.
* At the 2D workload's size (512^2, 686 parts): one step against the
  one-iteration form, to the full-size bars.
* In batches: runs of both forms, both precisions, share launches by form and
  each gets bitwise its alone result.
"""
import numpy as np
import pytest

from tests.gpu_common import make_pair, rel, require_gpu

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-10


@pytest.mark.parametrize("dim,n,rows", [(2, 16, 64), (2, 23, 128), (2, 40, 2048), (3, 3, 64),
                                        (3, 4, 128)])
def test_sstep_pressure_step_matches_oracle(dim, n, rows):
    torch, I = require_gpu()
    print(f"s-step pressure dim={dim} n={n} rows={rows}", flush=True)
    kind = "tg" if dim == 2 else "beltrami"
    S, o, r = make_pair(I, dim, n, kind, 0.01, 0.01, poisson_part_rows=rows, poisson_s=2)
    part = r.poisson_partition()
    assert part["rows_max"] == rows
    t1 = o.t + 0.01
    g = o.dirichlet(t1)
    r.phase(I.IPCS_PHASE_ASM)
    r.phase(I.IPCS_PHASE_MOMENTUM)
    st = r.phase(I.IPCS_PHASE_PRESSURE)
    Us_o, _, _ = o.momentum(t1, g)
    dP_o, it_o = o.pressure(Us_o)
    print("  iterations", st["it_p"], "oracle", it_o, flush=True)
    assert rel(r.field(I.IPCS_FIELD_DP), dP_o) <= FIELD_TOL, st
    r.phase(I.IPCS_PHASE_CORRECTION)
    o.step()
    assert rel(r.pressure(), o.P) <= FIELD_TOL
    for step in range(2):
        r.advance(1)
        o.step()
        assert rel(r.pressure(), o.P) <= FIELD_TOL
        for c in range(dim):
            assert rel(r.velocity()[c], o.U[c]) <= FIELD_TOL


@pytest.mark.parametrize("prec_name", ["fp64", "mixed"])
def test_sstep_and_one_step_forms_agree(prec_name):
    torch, I = require_gpu()
    print(f"s-step vs one iteration per launch ({prec_name})", flush=True)
    prec = I.IPCS_FP64 if prec_name == "fp64" else I.IPCS_MIXED
    m = I.Mesh.unit_square(48)
    out = []
    for s in (1, 2):
        p = I.ipcs_params_default(nu=0.004, dt=0.003, precision=prec, tol_ir=1e-10, tol_p=1e-13,
                                  poisson_s=s)
        r = I.Run(m, p)
        r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (2 * np.pi,))
        st = r.advance(3)
        out.append((r, [x["it_p"] for x in st]))
    (a, ita), (b, itb) = out
    print(ita, itb, flush=True)
    # per step the counts scatter after a true-residual restart (tol 1e-13 is
    # near the attainable accuracy, and the forms round differently); their
    # totals agree
    assert abs(sum(ita) - sum(itb)) <= 0.05 * sum(itb)
    bar = FIELD_TOL if prec_name == "fp64" else 1e-7
    for c in range(2):
        assert rel(a.velocity()[c], b.velocity()[c]) <= bar
    assert rel(a.pressure(), b.pressure()) <= bar


def test_sstep_full_size_step_against_one_step_form():
    """512^2 (686 parts of at most 384 rows), the workload's problem, one step
    at tolerance 1e-13 in both forms from the same start: the two solutions of
    the same systems differ by at most the full-size bars of the oracle
    comparison (u 1e-13, p 1.6e-11)."""
    torch, I = require_gpu()
    from paper_2605_25403_amd.workloads import resolve
    w = resolve("c2")
    print("s-step full size 512^2", flush=True)
    m = I.Mesh.unit_square(512)
    res = []
    for s in (1, 2):
        p = I.ipcs_params_default(nu=w["nu"], dt=w["dt"], tol_mom=1e-13, tol_p=1e-13,
                                  tol_corr=1e-13, poisson_s=s)
        r = I.Run(m, p)
        r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (w["k"],))
        st = r.advance(1)[0]
        print(f"  s={s}: pressure iterations {st['it_p']}", flush=True)
        res.append((r.velocity(), r.pressure()))
        del r
    (U1, P1), (U2, P2) = res
    eu = max(rel(U2[c], U1[c]) for c in range(2))
    ep = rel(P2, P1)
    print(f"  u {eu:.2e} p {ep:.2e}", flush=True)
    assert eu <= 1e-13 and ep <= 1.6e-11


def test_sstep_runs_in_batches_bitwise():
    torch, I = require_gpu()
    print("batch with both iteration counts per launch", flush=True)
    cases = [(12, 0, 2, I.IPCS_FP64), (12, 0, 1, I.IPCS_FP64), (20, 128, 2, I.IPCS_FP64),
             (16, 0, 2, I.IPCS_MIXED), (9, 64, 2, I.IPCS_MIXED), (10, -1, 0, I.IPCS_FP64)]

    def mk(n, rows, s, prec, stream=None):
        p = I.ipcs_params_default(nu=0.01, dt=0.005, precision=prec, tol_ir=1e-10,
                                  poisson_part_rows=rows, poisson_s=s)
        r = I.Run(I.Mesh.unit_square(n), p, stream=stream)
        r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (np.pi,))
        return r

    alone = []
    for c in cases:
        r = mk(*c)
        r.advance(3)
        alone.append((r.velocity(), r.pressure()))
    s = torch.cuda.Stream()
    runs = [mk(*c, stream=s) for c in cases]
    for _ in range(3):
        rc, st = I.ipcs_batch_step([r.h for r in runs], s.cuda_stream)
        assert rc == I.IPCS_OK, st
    for (U, P), r in zip(alone, runs):
        np.testing.assert_array_equal(r.velocity(), U)
        np.testing.assert_array_equal(r.pressure(), P)
