"""GPU two-level a posteriori preconditioner (Eq. 2lvlDef, Alg. 3) through the C ABI.

Tolerances: maps relative L2 <= 1e-6 against the FP64 oracle's PCG map (the solution A^-1 b is
the same whatever the preconditioner); the A-DEF1 identity M_2lvl A Z = Z holds to the FP32
rounding of the time-domain products (relative 1e-5); iteration counts within 3 of the oracle's
two-level PCG built with the same number of Lanczos steps from the same start vector.
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


_cache = {}


def case(name):
    if name not in _cache:
        if name == "raster":
            prob = synth.make_raster(cfg_id=81, n_dets=3, side=12, dwell=8, lam=96, n_rhs=4)
        else:
            prob = synth.make_ground(cfg_id=82, n_dets=6, samples_per_det=40000, interval=9000,
                                     side=32, lam=700, flag_frac=0.02, n_rhs=3)
        _cache[name] = (prob, O.plan_from_problem(prob))
    return _cache[name]


@pytest.mark.parametrize("name,m", [("raster", 24), ("ground", 32)])
def test_two_level_pcg_matches_oracle(gpu_lib, name, m):
    prob, ref = case(name)
    plan = gpu_lib.Plan.from_problem(prob)
    info = plan.deflation_build(_dev(prob.d[0]), m)
    assert info["m"] == m and 1 <= info["rank"] <= m and 0 < info["e_min"] <= info["e_max"]
    defl = O.deflation_from_lanczos(O.lanczos(ref, O.rhs(ref, prob.d[0]), m))
    for j in range(prob.d.shape[0]):
        b = O.rhs(ref, prob.d[j])
        bd = O.pcg(ref, b, tol=1e-8)
        tl = O.pcg(ref, b, tol=1e-8, precond=lambda r: O.precond_2lvl(ref, defl, r))
        x, inf = plan.pcg_solve(_dev(prob.d[j]), tol=1e-8, precond=1)
        err = float(_rel(x.cpu().numpy(), bd.x))
        assert err <= 1e-6, (j, err)
        assert inf["converged"] == 1 and inf["true_relres"] < 1e-7, inf
        assert abs(inf["iterations"] - tl.iterations) <= 3, (j, inf["iterations"], tl.iterations)
        assert inf["iterations"] <= bd.iterations + 2
    # the start vector's own system gains most
    _, inf0 = plan.pcg_solve(_dev(prob.d[0]), tol=1e-8, precond=1)
    _, bd0 = plan.pcg_solve(_dev(prob.d[0]), tol=1e-8)
    assert inf0["iterations"] < bd0["iterations"], (inf0, bd0)


def test_two_level_maps_deflation_space_to_itself(gpu_lib):
    prob, ref = case("raster")
    plan = gpu_lib.Plan.from_problem(prob)
    info = plan.deflation_build(_dev(prob.d[1]), 16)
    assert info["rank"] == 16
    Z = plan.deflation_vectors()
    AZ = plan.apply_A(Z)
    got = plan.precond_2lvl(AZ).cpu().numpy()
    err = float(_rel(got, Z.cpu().numpy()))
    assert err <= 1e-5, err


def test_two_level_graph_and_eager_agree(gpu_lib):
    import torch
    prob, ref = case("raster")
    plan = gpu_lib.Plan.from_problem(prob)
    plan.deflation_build(_dev(prob.d[0]), 20)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        d = _dev(prob.d[2])
        xg, ig = plan.pcg_solve(d, precond=1, use_graph=True, stream=s)
        xe, ie = plan.pcg_solve(d, precond=1, use_graph=False, stream=s)
    s.synchronize()
    assert ig["iterations"] == ie["iterations"]
    err = float(_rel(xg.cpu().numpy(), xe.cpu().numpy()))
    assert err <= 1e-8, err


def test_two_level_errors(gpu_lib):
    prob, ref = case("raster")
    plan = gpu_lib.Plan.from_problem(prob)
    d = _dev(prob.d[0])
    with pytest.raises(gpu_lib.MMError) as e:
        plan.pcg_solve(d, precond=1)
    assert e.value.status == -1
    for m in (0, 129):
        with pytest.raises(gpu_lib.MMError):
            plan.deflation_build(d, m)
    plan.deflation_build(d, 8)
    with pytest.raises(gpu_lib.MMError) as e:
        plan.pcg_solve(_dev(prob.d[:3]), precond=1, block=3)
    assert e.value.status == -7
    plan.deflation_clear()
    assert plan.deflation_info()["m"] == 0
    with pytest.raises(gpu_lib.MMError):
        plan.pcg_solve(d, precond=1)
