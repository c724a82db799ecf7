"""ipcs_batch_step_noalloc, the batch step for callers that cannot allocate,
against ipcs_batch_step: two calls in a row (the second with a smaller
batch) give bitwise the same fields, times and iteration counts, since both
run the same kernels with the same block decompositions and per-run
reductions; a batch beyond the fixed arrays is refused before any work."""
import numpy as np
import pytest

from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu

# (n, k, nu, dt, precision, pair): FP64 and mixed runs, both Taylor-Hood pairs
CASES = [(24, np.pi, 0.05, 0.01, "fp64", "p2p1"), (16, 2 * np.pi, 0.005, 0.004, "mixed", "p2p1"),
         (10, np.pi, 0.02, 0.01, "fp64", "p3p2"), (12, 4 * np.pi, 0.002, 0.002, "mixed", "p2p1"),
         (8, np.pi, 0.02, 0.01, "mixed", "p3p2")]


def new_run(I, case, stream):
    n, k, nu, dt, prec, pair = case
    p = I.ipcs_params_default(nu=nu, dt=dt, tol_ir=1e-10,
                              precision=I.IPCS_FP64 if prec == "fp64" else I.IPCS_MIXED)
    m = I.Mesh.unit_square(n, pair=I.IPCS_PAIR_P2P1 if pair == "p2p1" else I.IPCS_PAIR_P3P2)
    r = I.Run(m, p, stream=stream)
    r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (k,))
    return r


def same(a, b, sa, sb):
    for x, y, u, v in zip(a, b, sa, sb):
        np.testing.assert_array_equal(x.velocity(), y.velocity())
        np.testing.assert_array_equal(x.pressure(), y.pressure())
        assert x.time() == y.time()
        assert u["status"] == v["status"] == 0
        assert (u["it_mom"], u["it_p"], u["it_corr"]) == (v["it_mom"], v["it_p"], v["it_corr"])


def test_noalloc_batch_equals_allocating_batch():
    torch, I = require_gpu()
    print("batch step without allocation vs with", flush=True)
    s = torch.cuda.Stream()
    ref = [new_run(I, c, s) for c in CASES]
    new = [new_run(I, c, s) for c in CASES]
    for rounds, size in ((2, len(CASES)), (2, 2)):   # then a smaller batch
        for _ in range(rounds):
            rc1, st1 = I.ipcs_batch_step([r.h for r in ref[:size]], s.cuda_stream)
            rc2, st2 = I.ipcs_batch_step_noalloc([r.h for r in new[:size]], s.cuda_stream)
            assert rc1 == rc2 == I.IPCS_OK, (st1, st2)
            same(ref[:size], new[:size], st1, st2)
        print(f"batch of {size}: equal after {rounds} steps", flush=True)
    # the runs left out of the smaller batch are where the larger one left them
    for x, y in zip(ref[size:], new[size:]):
        np.testing.assert_array_equal(x.velocity(), y.velocity())
        np.testing.assert_array_equal(x.pressure(), y.pressure())
        assert x.time() == y.time()


def test_noalloc_batch_refuses_more_runs_than_its_arrays_hold():
    torch, I = require_gpu()
    print("batch step without allocation: capacity", flush=True)
    s = torch.cuda.Stream()
    m = I.Mesh.unit_square(1)
    runs = []
    for _ in range(I.IPCS_BATCH_NOALLOC_MAX_RUNS + 1):
        r = I.Run(m, I.ipcs_params_default(nu=0.01, dt=0.01), stream=s)
        r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (np.pi,))
        runs.append(r)
    U0 = runs[0].velocity().copy()
    with pytest.raises(I.IpcsError) as e:
        I.ipcs_batch_step_noalloc([r.h for r in runs], s.cuda_stream)
    assert e.value.code == I.IPCS_E_CAPACITY
    assert all(r.time() == 0.0 for r in runs)
    np.testing.assert_array_equal(runs[0].velocity(), U0)
    # the largest batch the arrays hold steps, and equals the allocating step
    rc, st = I.ipcs_batch_step_noalloc([r.h for r in runs[:-1]], s.cuda_stream)
    assert rc == I.IPCS_OK and all(x["status"] == 0 for x in st)
    rc, st = I.ipcs_batch_step([runs[-1].h], s.cuda_stream)
    assert rc == I.IPCS_OK
    np.testing.assert_array_equal(runs[0].velocity(), runs[-1].velocity())
    np.testing.assert_array_equal(runs[0].pressure(), runs[-1].pressure())
