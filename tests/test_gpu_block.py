"""GPU parity of stacked right-hand sides: the multi-column product A X and the enlarged-CG
solve (Alg. 2, Orthomin form) through the C ABI, against the FP64 oracle.

Tolerances as for single columns: A X relative L2 <= 3e-6 per column (FP32 time domain);
maps relative L2 <= 1e-6 against the oracle's FP64 block iteration and against independent
PCG solves (both reach the same solution A^-1 b_j to tol 1e-8; the FP32 floor is ~1.3e-7).
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


CASES = {
    "raster_rhs6": lambda: synth.make_raster(cfg_id=61, n_dets=3, side=16, dwell=8, lam=200,
                                             n_rhs=6),
    "random_rhs5": lambda: synth.make_random_small(seed=9, n_samples=6007, n_pix=70, n_dets=4,
                                                   lam_max=48, flag_frac=0.1, gap_frac=0.2,
                                                   dwell=5, n_rhs=5),
    "ground_rhs4": lambda: synth.make_ground(cfg_id=62, n_dets=6, samples_per_det=40000,
                                             interval=9000, side=32, lam=700, flag_frac=0.02,
                                             n_rhs=4),
    # lambda = 8192: 2^15-sample segments through the register-resident kernel, several columns
    "ground_lam8192_rhs3": lambda: synth.make_ground(cfg_id=65, n_dets=3, samples_per_det=70001,
                                                     interval=35001, side=24, lam=8192,
                                                     flag_frac=0.01, n_rhs=3),
    # lambda = 2^14: 2^16-sample segments through the persistent four-step kernel, several
    # columns sharing its workgroups
    "satellite_lam16384_rhs2": lambda: synth.make_satellite(cfg_id=66, n_dets=2,
                                                            samples_per_det=1 << 18,
                                                            interval=1 << 17, n_rings=32,
                                                            n_phi=64, lam=1 << 14, n_rhs=2),
}

_cache = {}


def case(name):
    if name not in _cache:
        prob = CASES[name]()
        _cache[name] = (prob, O.plan_from_problem(prob))
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("unfused", [False, True])
def test_apply_A_multi_column_parity(gpu_lib, name, unfused):
    prob, ref = case(name)
    plan = gpu_lib.Plan.from_problem(prob, flags=gpu_lib.FLAG_UNFUSED if unfused else 0)
    if name == "ground_lam8192_rhs3":
        assert plan.info["fused"] == (0 if unfused else 2), plan.info
    if name.startswith("satellite"):
        assert plan.info["fused"] == (0 if unfused else 3), plan.info
    X = np.random.default_rng(7).standard_normal((5, ref.n_kept, 3))
    Y = plan.apply_A(_dev(X)).cpu().numpy()
    for j in range(5):
        err = float(_rel(Y[j], O.apply_A(ref, X[j])))
        assert err <= 3e-6, (j, err)


@pytest.mark.parametrize("name", list(CASES))
def test_block_solve_matches_oracle(gpu_lib, name):
    prob, ref = case(name)
    k = prob.d.shape[0]
    plan = gpu_lib.Plan.from_problem(prob)
    B = np.stack([O.rhs(ref, prob.d[j]) for j in range(k)])
    want = O.block_ecg(ref, B, tol=1e-8)
    indep = O.block_pcg(ref, B, tol=1e-8)
    assert want.converged.all()
    x, infos = plan.pcg_solve(_dev(prob.d), tol=1e-8, block=k)
    m = x.cpu().numpy()
    for j in range(k):
        inf = infos[j]
        assert inf["converged"] == 1 and inf["block"] == k
        err = float(_rel(m[j], want.x[j]))
        assert err <= 1e-6, (j, err)
        err = float(_rel(m[j], indep.x[j]))
        assert err <= 1e-6, (j, err)
        assert abs(inf["iterations"] - int(want.iterations[j])) <= 2, (j, inf, want.iterations)
        assert inf["relres"] < 1e-8
        assert inf["true_relres"] < 1e-7, inf
    # the block shares one search space: it never needs more iterations than the slowest column
    assert max(i["iterations"] for i in infos) <= int(indep.iterations.max()) + 2


def test_block_size_two_and_partial_groups(gpu_lib):
    prob, ref = case("raster_rhs6")
    plan = gpu_lib.Plan.from_problem(prob)
    x, infos = plan.pcg_solve(_dev(prob.d[:5]), tol=1e-8, block=2)  # groups 2, 2, 1
    m = x.cpu().numpy()
    for j in range(5):
        B = np.stack([O.rhs(ref, prob.d[i]) for i in range(2 * (j // 2), min(5, 2 * (j // 2) + 2))])
        want = O.block_ecg(ref, B, tol=1e-8)
        err = float(_rel(m[j], want.x[j % 2]))
        assert err <= 1e-6, (j, err)
        assert infos[j]["block"] == 2


def test_block_tuned_many_columns(gpu_lib):
    prob = synth.make_raster(cfg_id=63, n_dets=2, side=12, dwell=8, lam=96, n_rhs=40)
    ref = O.plan_from_problem(prob)
    plan = gpu_lib.Plan.from_problem(prob)
    x, infos = plan.pcg_solve(_dev(prob.d), tol=1e-8, block=-1)
    m = x.cpu().numpy()
    # tuning order: 8 columns alone (t = 1), 8 with t = 8, 16 with t = 16, the last 8 with t = 32
    assert [i["block"] for i in infos] == [1] * 8 + [8] * 8 + [16] * 16 + [32] * 8
    for j in range(40):
        assert infos[j]["converged"] == 1
        want = O.pcg(ref, O.rhs(ref, prob.d[j]), tol=1e-8).x
        err = float(_rel(m[j], want))
        assert err <= 1e-6, (j, err)
    # the plan keeps the tuned size: a second tuned solve uses it for every group
    x2, infos2 = plan.pcg_solve(_dev(prob.d[:20]), tol=1e-8, block=-1)
    sizes = {i["block"] for i in infos2}
    assert len(sizes) == 1 and sizes <= {1, 8, 16}, sizes
    err = float(_rel(x2.cpu().numpy(), m[:20]))
    assert err <= 1e-6, err


def test_block_zero_and_repeated_columns(gpu_lib):
    # a zero column leaves at once (x = 0); two equal columns make the search block rank
    # deficient, which the pseudo-inverse absorbs: both still reach the same map
    prob, ref = case("raster_rhs6")
    d = np.stack([prob.d[0], np.zeros_like(prob.d[0]), prob.d[0], prob.d[1]])
    plan = gpu_lib.Plan.from_problem(prob)
    x, infos = plan.pcg_solve(_dev(d), tol=1e-8, block=4)
    m = x.cpu().numpy()
    assert infos[1]["iterations"] == 0 and infos[1]["converged"] == 1
    assert np.all(m[1] == 0.0)
    for j, src in ((0, 0), (2, 0), (3, 1)):
        assert infos[j]["converged"] == 1
        want = O.pcg(ref, O.rhs(ref, prob.d[src]), tol=1e-8).x
        err = float(_rel(m[j], want))
        assert err <= 1e-6, (j, err)


def test_block_white_noise_one_iteration(gpu_lib):
    prob = synth.make_raster(cfg_id=64, n_dets=3, side=16, dwell=4, lam=0, noise="white",
                             n_rhs=3)
    ref = O.plan_from_problem(prob)
    plan = gpu_lib.Plan.from_problem(prob)
    x, infos = plan.pcg_solve(_dev(prob.d), block=3)
    m = x.cpu().numpy()
    for j in range(3):
        assert infos[j]["iterations"] == 1
        err = float(_rel(m[j], O.binned_map(ref, prob.d[j])))
        assert err <= 1e-7, (j, err)


def test_block_rejects_restart(gpu_lib):
    prob, ref = case("raster_rhs6")
    plan = gpu_lib.Plan.from_problem(prob)
    x = plan.pcg_solve(_dev(prob.d[:2]), block=2)[0]
    with pytest.raises(RuntimeError):
        plan.pcg_solve(_dev(prob.d[:2]), x=x, use_x0=True, block=2)
