"""The one-kernel-per-iteration Poisson CG (row partition, halo recomputation,
u in LDS) on the GPU, through the C ABI.

* Against the FP64 oracle, for part sizes that give many small parts with
  ragged last slices (and one part holding everything): the pressure
  increment of one step from an identical state, bar 1e-10 as for every field.
* Against the two-kernel CG of the same library: both forms compute the same
  iterates in exact arithmetic, so over three steps the fields agree to the
  solve tolerance and the iteration counts to within rounding (2 iterations).
* In batches: runs in either form and in both precisions share launches and
  each gets bitwise its alone result.
"""
import numpy as np
import pytest

from tests.gpu_common import make_pair, rel, require_gpu

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-10


@pytest.mark.parametrize("dim,n,rows", [(2, 16, 64), (2, 23, 128), (2, 40, 2048), (3, 3, 64),
                                        (3, 4, 128)])
def test_fused_pressure_step_matches_oracle(dim, n, rows):
    torch, I = require_gpu()
    print(f"fused pressure dim={dim} n={n} rows={rows}", flush=True)
    kind = "tg" if dim == 2 else "beltrami"
    S, o, r = make_pair(I, dim, n, kind, 0.01, 0.01, poisson_part_rows=rows)
    part = r.poisson_partition()
    assert part["rows_max"] == rows and part["nparts"] >= -(-S.N1 // rows)
    t1 = o.t + 0.01
    g = o.dirichlet(t1)
    r.phase(I.IPCS_PHASE_ASM)
    r.phase(I.IPCS_PHASE_MOMENTUM)
    st = r.phase(I.IPCS_PHASE_PRESSURE)
    Us_o, _, _ = o.momentum(t1, g)
    dP_o, it_o = o.pressure(Us_o)
    assert rel(r.field(I.IPCS_FIELD_DP), dP_o) <= FIELD_TOL, st
    r.phase(I.IPCS_PHASE_CORRECTION)
    o.step()
    assert rel(r.pressure(), o.P) <= FIELD_TOL


@pytest.mark.parametrize("prec_name", ["fp64", "mixed"])
def test_fused_and_two_kernel_forms_agree(prec_name):
    torch, I = require_gpu()
    print(f"fused vs two-kernel ({prec_name})", flush=True)
    prec = I.IPCS_FP64 if prec_name == "fp64" else I.IPCS_MIXED
    m = I.Mesh.unit_square(48)
    out = []
    for rows in (0, -1):
        p = I.ipcs_params_default(nu=0.004, dt=0.003, precision=prec, tol_ir=1e-10, tol_p=1e-13,
                                  poisson_part_rows=rows)
        r = I.Run(m, p)
        r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (2 * np.pi,))
        st = r.advance(3)
        out.append((r, [s["it_p"] for s in st]))
    (a, ita), (b, itb) = out
    assert a.poisson_partition()["rows_max"] == 384 and b.poisson_partition()["rows_max"] == 0
    print(ita, itb, flush=True)
    assert max(abs(x - y) for x, y in zip(ita, itb)) <= (2 if prec_name == "fp64" else 30)
    bar = FIELD_TOL if prec_name == "fp64" else 1e-7
    for c in range(2):
        assert rel(a.velocity()[c], b.velocity()[c]) <= bar
    assert rel(a.pressure(), b.pressure()) <= bar


def test_batch_mixes_poisson_forms_bitwise():
    torch, I = require_gpu()
    print("batch with both Poisson forms", flush=True)
    cases = [(12, 0, I.IPCS_FP64), (12, -1, I.IPCS_FP64), (20, 128, I.IPCS_FP64),
             (16, 0, I.IPCS_MIXED), (9, 64, I.IPCS_MIXED)]

    def mk(n, rows, prec, stream=None):
        p = I.ipcs_params_default(nu=0.01, dt=0.005, precision=prec, tol_ir=1e-10,
                                  poisson_part_rows=rows)
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


def test_fused_kernel_profile_hook():
    torch, I = require_gpu()
    print("fused profile hook", flush=True)
    m = I.Mesh.unit_square(64)
    r = I.Run(m, I.ipcs_params_default())
    r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (np.pi,))
    r.advance(1)
    us = I.ipcs_profile_kernel(r.h, I.IPCS_KERNEL_PCG_FUSED_P, 20)
    assert us > 0.0
    with pytest.raises(I.IpcsError):
        I.ipcs_profile_kernel(r.h, I.IPCS_KERNEL_PCG_SPMV_P, 5)
    r.advance(1)   # the run still steps after profiling (tolerances restored)
    two = I.Run(m, I.ipcs_params_default(poisson_part_rows=-1))
    two.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (np.pi,))
    with pytest.raises(I.IpcsError):
        I.ipcs_profile_kernel(two.h, I.IPCS_KERNEL_PCG_FUSED_P, 5)
    for k in (I.IPCS_KERNEL_PCG_SPMV_P, I.IPCS_KERNEL_PCG_UPDATE_P, I.IPCS_KERNEL_BICG_UPDATE_X):
        assert I.ipcs_profile_kernel(two.h, k, 5) > 0.0
    two.advance(1)   # profiling leaves the tolerances as they were


def test_wide_halo_parts_block_and_map_paths_bitwise():
    """Parts whose halo exceeds one block's threads (3D, parts of up to 2048
    rows: 8 rows per thread, up to 376 halo rows). Alone, a run's iterations
    take its per-block descriptors; in a batch, the block map. The two must
    give bitwise the same fields, and agree with the two-kernel CG."""
    torch, I = require_gpu()
    print("wide-halo parts: descriptor vs block-map launches", flush=True)
    m = I.Mesh.unit_cube(16)
    q = I.ipcs_mesh_p1_partition(m.h, 2048)
    assert np.diff(q["halo_ptr"]).max() > 256

    def new_run(rows, stream=None):
        p = I.ipcs_params_default(nu=0.01, dt=0.01, tol_p=1e-13, poisson_part_rows=rows)
        r = I.Run(m, p, stream=stream)
        r.set_builtin(I.IPCS_SOL_BELTRAMI_3D, ())
        return r

    alone = new_run(2048)
    alone.advance(2)
    two = new_run(-1)
    two.advance(2)
    s = torch.cuda.Stream()
    pair = [new_run(2048, stream=s), new_run(2048, stream=s)]
    for _ in range(2):
        rc, st = I.ipcs_batch_step([r.h for r in pair], s.cuda_stream)
        assert rc == I.IPCS_OK, st
    for r in pair:
        np.testing.assert_array_equal(r.velocity(), alone.velocity())
        np.testing.assert_array_equal(r.pressure(), alone.pressure())
    for c in range(3):
        assert rel(alone.velocity()[c], two.velocity()[c]) <= FIELD_TOL
    assert rel(alone.pressure(), two.pressure()) <= FIELD_TOL
