"""Serving form on the GPU: runs stepped together with ipcs_batch_step give
bitwise the results they get alone (integer-exact bar: the same kernels and
the same per-run reductions run in both cases), match the FP64 oracle when
stepped in a batch, and the request loop completes a small stream with each
result equal to the alone result."""
import numpy as np
import pytest

from tests.gpu_common import field_errors, make_pair, require_gpu

pytestmark = pytest.mark.gpu

CASES = [(8, np.pi, 0.02, 0.01), (16, 2 * np.pi, 0.005, 0.004), (24, np.pi, 0.05, 0.01),
         (12, 4 * np.pi, 0.002, 0.002)]


def new_run(I, n, k, nu, dt, prec, stream=None):
    p = I.ipcs_params_default(nu=nu, dt=dt, precision=prec, tol_ir=1e-10)
    r = I.Run(I.Mesh.unit_square(n), p, stream=stream)
    r.set_builtin(I.IPCS_SOL_TAYLOR_GREEN_2D, (k,))
    return r


@pytest.mark.parametrize("prec_name", ["fp64", "mixed"])
def test_batch_equals_alone_bitwise(prec_name):
    torch, I = require_gpu()
    print(f"batch == alone ({prec_name})", flush=True)
    prec = I.IPCS_FP64 if prec_name == "fp64" else I.IPCS_MIXED
    alone = []
    for n, k, nu, dt in CASES:
        r = new_run(I, n, k, nu, dt, prec)
        r.advance(3)
        alone.append((r.velocity(), r.pressure(), r.time()))
    s = torch.cuda.Stream()
    runs = [new_run(I, n, k, nu, dt, prec, stream=s) for n, k, nu, dt in CASES]
    for step in range(3):
        rc, st = I.ipcs_batch_step([r.h for r in runs], s.cuda_stream)
        assert rc == I.IPCS_OK, st
        assert all(x["status"] == 0 and x["it_p"] > 0 for x in st), st
    for (U, P, t), r in zip(alone, runs):
        np.testing.assert_array_equal(r.velocity(), U)
        np.testing.assert_array_equal(r.pressure(), P)
        assert r.time() == t


def test_batch_mixes_forms_and_matches_oracle():
    """An FP64 run batched with mixed runs still matches the FP64 oracle."""
    torch, I = require_gpu()
    print("batch vs oracle", flush=True)
    S, o, r = make_pair(I, 2, 16, "tg", 0.01, 0.01, same_state=False)
    s = torch.cuda.Stream()
    others = [new_run(I, n, k, nu, dt, I.IPCS_MIXED, stream=s) for n, k, nu, dt in CASES[:2]]
    for step in range(4):
        rc, st = I.ipcs_batch_step([r.h] + [x.h for x in others], s.cuda_stream)
        assert rc == I.IPCS_OK, st
        o.step()
        errs = field_errors(o, r)
        assert max(errs) <= 1e-10, (step, errs)


@pytest.mark.parametrize("fp64", [False, True])
def test_serving_loop_small_stream_equals_alone(fp64):
    torch, I = require_gpu()
    print(f"serving loop fp64={fp64}", flush=True)
    from paper_2605_25403_amd.serve import Request, Server
    prec = I.IPCS_FP64 if fp64 else I.IPCS_MIXED
    reqs = [Request(id=i, t_arrive=0.002 * i, n=n, k=k, nu=nu, steps=3 + (i % 4), dt=dt)
            for i, (n, k, nu, dt) in enumerate(CASES * 2)]
    srv = Server(max_slots=3, hbm_budget=1 << 34, precision=prec)
    report, res = srv.serve(reqs, keep_fields=True)
    print(report, flush=True)
    assert report["failed"] == 0 and len(res) == len(reqs)
    assert report["max_active"] <= 3
    for q in reqs:
        r = new_run(I, q.n, q.k, q.nu, q.dt, prec)
        r.advance(q.steps)
        np.testing.assert_array_equal(res[q.id]["U"], r.velocity())
        np.testing.assert_array_equal(res[q.id]["P"], r.pressure())
        assert len(res[q.id]["lat"]) == q.steps


@pytest.mark.parametrize("cus", [None, (8, None)])
def test_serving_lanes_by_size_equal_alone(cus):
    """Lanes by mesh size, each with its own stream and host thread, sharing
    the slot cap, without and with CU masks (8 CUs reserved for the first
    lane, the rest for the second): every result is bitwise the result
    alone, and the report gives per-size latencies."""
    torch, I = require_gpu()
    print(f"serving lanes cus={cus}", flush=True)
    from paper_2605_25403_amd.serve import Request, Server
    reqs = [Request(id=i, t_arrive=0.001 * i, n=n, k=k, nu=nu, steps=2 + (i % 4), dt=dt)
            for i, (n, k, nu, dt) in enumerate(CASES * 3)]
    srv = Server(max_slots=4, hbm_budget=1 << 34, lanes=((8, 12), (16, 24)), lane_cus=cus)
    report, res = srv.serve(reqs, keep_fields=True)
    print(report, flush=True)
    assert report["failed"] == 0 and len(res) == len(reqs)
    assert report["max_active"] <= 4
    assert set(report["step_ms_by_n"]) == {"8", "12", "16", "24"}
    for q in reqs:
        r = new_run(I, q.n, q.k, q.nu, q.dt, I.IPCS_MIXED)
        r.advance(q.steps)
        np.testing.assert_array_equal(res[q.id]["U"], r.velocity())
        np.testing.assert_array_equal(res[q.id]["P"], r.pressure())
        assert len(res[q.id]["lat"]) == q.steps


def test_serving_admission_by_footprint_queues_requests():
    torch, I = require_gpu()
    print("serving admission", flush=True)
    from paper_2605_25403_amd.serve import Request, Server
    reqs = [Request(id=i, t_arrive=0.0, n=16, k=np.pi, nu=0.01, steps=2, dt=0.01)
            for i in range(5)]
    srv = Server(max_slots=64)
    one = srv.footprint(reqs[0])
    srv.hbm_budget = 2 * one + one // 2          # room for two runs at a time
    report, res = srv.serve(reqs)
    assert report["failed"] == 0 and report["max_active"] == 2
    assert report["rounds"] >= 6                 # 5 runs x 2 steps, two at a time
