"""Serving loop on the GPU: device-cached plans, continuously batched requests of uneven size,
memory-budget admission, and results that do not depend on the mix.

Tolerances: a request solved in the mix and the same request solved alone differ only in the
order of FP64 atomic additions (last-bit differences that CG carries through its iterations):
relative L2 <= 1e-8.  Against the FP64 oracle: the map tolerance of the plain solve, 1e-6.
"""

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _problems():
    return [
        synth.make_raster(cfg_id=71, n_dets=3, side=16, dwell=8, lam=200, n_rhs=2),
        synth.make_raster(cfg_id=72, n_dets=4, side=24, dwell=8, lam=600, n_rhs=3),
        synth.make_random_small(seed=11, n_samples=7001, n_pix=80, n_dets=4, lam_max=40,
                                flag_frac=0.1, gap_frac=0.2, dwell=5, n_rhs=1),
        synth.make_ground(cfg_id=73, n_dets=6, samples_per_det=40000, interval=9000, side=32,
                          lam=700, flag_frac=0.02, n_rhs=2),
        synth.make_raster(cfg_id=74, n_dets=2, side=16, dwell=4, lam=0, noise="white", n_rhs=1),
    ]


_probs = None


def problems():
    global _probs
    if _probs is None:
        _probs = _problems()
    return _probs


def _alone(lib, prob):
    plan = lib.Plan.from_problem(prob)
    x, _ = plan.pcg_solve(_dev(prob.d), tol=1e-8)
    out = x.cpu().numpy().reshape(prob.d.shape[0], plan.n_kept, 3)
    plan.close()
    return out


def test_requests_in_the_mix_match_alone_and_oracle(gpu_lib):
    import torch
    probs = problems()
    alone = [_alone(gpu_lib, p) for p in probs]
    srv = gpu_lib.Server(n_slots=4)
    infos = [srv.plan_from_problem(100 + i, p) for i, p in enumerate(probs)]
    # every geometry twice, all submitted at once: the solves overlap on the device
    tickets = []
    for rep in range(2):
        for i, p in enumerate(probs):
            d = _dev(p.d)
            x = torch.empty((p.d.shape[0], infos[i]["n_kept"], 3), dtype=torch.float64,
                            device="cuda")
            tickets.append((i, srv.submit(100 + i, d, x, tol=1e-8)))
    for i, t in tickets:
        res = srv.wait(t)
        assert res["status"] == "MM_OK"
        m = res["x"].cpu().numpy().reshape(alone[i].shape)
        err = float(_rel(m, alone[i]))
        assert err <= 1e-8, (i, err)
        for inf in res["info"]:
            assert inf["converged"] == 1
        assert res["times"]["total_ms"] >= res["times"]["run_ms"] >= 0.0
    st = srv.stats()
    assert st["completed"] == len(tickets) and st["queued"] == 0 and st["running"] == 0
    assert st["peak_running"] >= 2, st
    assert st["plan_misses"] == len(probs)
    srv.close()
    # the mix against the oracle, on the small cases
    for i in (0, 2):
        ref = O.plan_from_problem(probs[i])
        for j in range(probs[i].d.shape[0]):
            want = O.pcg(ref, O.rhs(ref, probs[i].d[j]), tol=1e-8).x
            err = float(_rel(alone[i][j], want))
            assert err <= 1e-6, (i, j, err)


def test_size_classes_hold_large_requests_to_their_slots(gpu_lib):
    # work n_samples x k: the 4-detector raster (3 RHS) and the ground case (2 RHS) are large
    import torch
    probs = problems()
    alone = [_alone(gpu_lib, p) for p in probs]
    work = [p.n_samples * p.d.shape[0] for p in probs]
    large_work = 50000
    assert [w >= large_work for w in work] == [False, True, False, True, False], work
    srv = gpu_lib.Server(n_slots=4, large_work=large_work, large_slots=1)
    infos = [srv.plan_from_problem(200 + i, p) for i, p in enumerate(probs)]
    tickets = []
    for rep in range(3):
        for i, p in enumerate(probs):
            x = torch.empty((p.d.shape[0], infos[i]["n_kept"], 3), dtype=torch.float64,
                            device="cuda")
            tickets.append((i, srv.submit(200 + i, _dev(p.d), x, tol=1e-8)))
    for i, t in tickets:
        res = srv.wait(t)
        assert res["status"] == "MM_OK"
        err = float(_rel(res["x"].cpu().numpy().reshape(alone[i].shape), alone[i]))
        assert err <= 1e-8, (i, err)
    st = srv.stats()
    assert st["completed"] == len(tickets) and st["queued"] == 0
    assert st["peak_large"] == 1, st
    assert st["peak_running"] >= 2, st
    srv.close()


def test_budget_admission_serializes_requests_of_one_plan(gpu_lib):
    import torch
    p = problems()[1]
    srv0 = gpu_lib.Server(n_slots=1)
    info = srv0.plan_from_problem(1, p)
    plan_bytes = info["device_bytes"]
    srv0.close()
    # room for the plan (with its own workspace) and half of one more workspace: requests on
    # that plan must run one at a time
    srv = gpu_lib.Server(hbm_budget=plan_bytes + 4096, n_slots=4)
    srv.plan_from_problem(1, p)
    d = _dev(p.d)
    xs = [torch.empty((p.d.shape[0], info["n_kept"], 3), dtype=torch.float64, device="cuda")
          for _ in range(5)]
    ts = [srv.submit(1, d, x) for x in xs]
    outs = [srv.wait(t)["x"].cpu().numpy() for t in ts]
    for o in outs[1:]:
        assert float(_rel(o, outs[0])) <= 1e-8
    st = srv.stats()
    assert st["peak_running"] == 1, st
    assert st["peak_bytes"] <= plan_bytes + 4096
    # a block solve needs more than the budget: refused at submission
    with pytest.raises(gpu_lib.MMError) as e:
        srv.submit(1, d, xs[0], block=3)
    assert e.value.status == -6  # MM_ERR_BUDGET
    srv.close()


def test_plan_cache_evicts_least_recently_used(gpu_lib):
    import torch
    probs = problems()
    srv0 = gpu_lib.Server(n_slots=1)
    sizes = [srv0.plan_from_problem(i, probs[i])["device_bytes"] for i in range(3)]
    srv0.close()
    srv = gpu_lib.Server(hbm_budget=sizes[0] + sizes[1] + sizes[2] - 1, n_slots=2)
    for i in range(3):
        srv.plan_from_problem(10 + i, probs[i])
    st = srv.stats()
    assert st["evictions"] >= 1 and st["n_plans"] <= 2
    with pytest.raises(gpu_lib.MMError) as e:  # key 10 was the least recently used
        srv.plan(10)
    assert e.value.status == -1
    d = _dev(probs[0].d)
    x = torch.empty((probs[0].d.shape[0], 1, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.MMError) as e:
        srv.submit(10, d, x)
    assert e.value.status == -8  # MM_ERR_NOT_FOUND
    # a hit needs no geometry and refreshes the entry
    info = srv.plan(12)
    assert info["n_kept"] > 0
    srv.close()


def test_block_request_in_the_server(gpu_lib):
    import torch
    p = synth.make_raster(cfg_id=75, n_dets=2, side=12, dwell=8, lam=96, n_rhs=10)
    plan = gpu_lib.Plan.from_problem(p)
    want, _ = plan.pcg_solve(_dev(p.d), tol=1e-8, block=5)
    want = want.cpu().numpy()
    srv = gpu_lib.Server(n_slots=2)
    info = srv.plan_from_problem(5, p)
    x = torch.empty((10, info["n_kept"], 3), dtype=torch.float64, device="cuda")
    res = srv.wait(srv.submit(5, _dev(p.d), x, block=5))
    assert all(i["block"] == 5 and i["converged"] == 1 for i in res["info"])
    err = float(_rel(res["x"].cpu().numpy(), want))
    assert err <= 1e-8, err
    srv.close()


def test_poll_and_tickets(gpu_lib):
    import time

    import torch
    p = problems()[0]
    srv = gpu_lib.Server(n_slots=2)
    info = srv.plan_from_problem(7, p)
    x = torch.empty((p.d.shape[0], info["n_kept"], 3), dtype=torch.float64, device="cuda")
    t = srv.submit(7, _dev(p.d), x)
    res = None
    t0 = time.time()
    while res is None and time.time() - t0 < 60:
        res = srv.poll(t)
        time.sleep(0.001)
    assert res is not None and res["status"] == "MM_OK"
    with pytest.raises(gpu_lib.MMError) as e:  # released by the poll that returned it
        srv.poll(t)
    assert e.value.status == -8
    with pytest.raises(gpu_lib.MMError):
        srv.poll(123456789)
    srv.close()


def test_destroy_with_queued_requests(gpu_lib):
    import torch
    p = problems()[3]
    srv = gpu_lib.Server(n_slots=1)
    info = srv.plan_from_problem(9, p)
    d = _dev(p.d)
    xs = [torch.empty((p.d.shape[0], info["n_kept"], 3), dtype=torch.float64, device="cuda")
          for _ in range(6)]
    for x in xs:
        srv.submit(9, d, x)
    srv.close()  # drops the queued requests, waits for the running one


def test_plan_builds_while_solves_capture_graphs(gpu_lib):
    # plan construction on the calling thread must not touch the legacy stream while worker
    # threads capture their PCG iterations into graphs
    import torch
    probs = problems()
    srv = gpu_lib.Server(n_slots=4)
    info = srv.plan_from_problem(200, probs[3])
    d = _dev(probs[3].d)
    xs = [torch.empty((probs[3].d.shape[0], info["n_kept"], 3), dtype=torch.float64, device="cuda")
          for _ in range(8)]
    ts = [srv.submit(200, d, x) for x in xs]
    for i, p in enumerate(probs[:3] + probs[4:]):
        srv.plan_from_problem(300 + i, p)  # builds while the requests above run
    for t in ts:
        assert srv.wait(t)["status"] == "MM_OK"
    srv.close()
