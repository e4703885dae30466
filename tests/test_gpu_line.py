"""GPU parity of the one-dimensional workloads (Sec. 4.1 continuous random wave
speed, Sec. 4.2 random jump): u(T) of every node against the oracle, the
device-pointer path, and Algorithm 1 for the L^2(D)-valued QoI."""
import numpy as np
import pytest

import paper_2106_11117_amd as P
from oracle import oned

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx():
    _torch()
    c = P.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("kind", ["kl", "jump"])
def test_line_solutions_match_oracle(ctx, kind):
    """u(T) at T = 11 (continuous field) and T = 6 (jump) on levels 0-4 (p = 16 .. 1
    and 32 .. 2): max-norm error <= 1e-11 of max |u|, for two samples each."""
    mk = oned.kl_level if kind == "kl" else oned.jump_level
    rule = P.line_sample_rule(kind)
    orule = oned.Rule1D(kind=kind, T=rule.T, cfl=rule.cfl)
    worst = 0.0
    for l in range(5):
        lid = ctx.add_line_level(P.line_rule(kind, l))
        lv = mk(l)
        s = P.gen_line_samples(0, l, 0, 4, rule, P.line_rule(kind, l))
        U = ctx.line_forward(lid, s["kappa"], s["n_steps"], s["dt"], rule, lv.n)
        for i in (0, 3):
            u = oned.solve_sample(lv, orule, 0, l, i)
            e = np.max(np.abs(U[i] - u)) / np.max(np.abs(u))
            worst = max(worst, e)
            assert e <= 1e-11, (l, i, e)
    print(f"{kind}: worst max-norm error {worst:.2e}")


def test_line_device_pointers(ctx):
    torch = _torch()
    rule = P.line_sample_rule("jump")
    lid = ctx.add_line_level(P.line_rule("jump", 1))
    n = P.line_level_host(P.line_rule("jump", 1))["n_nodes"]
    s = P.gen_line_samples(0, 1, 0, 5, rule, P.line_rule("jump", 1))
    Uh = ctx.line_forward(lid, s["kappa"], s["n_steps"], s["dt"], rule, n)
    d = torch.device("cuda:0")
    Ud = ctx.line_forward(lid, torch.tensor(s["kappa"], device=d), torch.tensor(s["n_steps"], device=d),
                          torch.tensor(s["dt"], device=d), rule, n)
    assert np.array_equal(Uh, Ud.cpu().numpy())


def test_line_mlmc_matches_oracle(ctx):
    """Algorithm 1 for Q = u(T) in L^2(D) on three levels of the random-jump
    workload (T = 2): the same L and N_l as the oracle, V_l and |mean|_V to
    1e-9, and the estimate (a function on the finest mesh) to 1e-11."""
    rule = P.line_sample_rule("jump", T=2.0)
    ids = [ctx.add_line_level(P.line_rule("jump", l)) for l in range(3)]
    res = ctx.line_mlmc(ids, rule, eps=2e-3, N_init=(16, 8, 4), L_start=1)
    levels = [oned.jump_level(l) for l in range(3)]
    ores = oned.mlmc_vec(levels, oned.Rule1D(kind="jump", T=2.0), eps=2e-3, N_init=(16, 8, 4), L_start=1)
    print(f"GPU L={res['L']} N={res['N']}; oracle L={ores.L} N={ores.N}")
    assert res["L"] == ores.L and res["N"] == ores.N
    for l in range(res["L"] + 1):
        assert abs(res["var"][l] - ores.var[l]) <= 1e-9 * ores.var[l]
        assert abs(res["mean_norm"][l] - ores.mean_norm[l]) <= 1e-9 * ores.mean_norm[l]
        assert res["cost"][l] == ores.cost[l]
    est = res["estimate"]
    assert est.size == ores.estimate.size
    assert np.max(np.abs(est - ores.estimate)) <= 1e-11 * np.max(np.abs(ores.estimate))
    assert abs(res["bias"] - ores.bias) <= 1e-9 * ores.bias


def test_line_leapfrog_twin_matches_oracle(ctx):
    """The standard leapfrog twin of a refined level (P empty, the step of the
    refined cells everywhere) against the oracle."""
    rule = P.line_sample_rule("kl")
    lid = ctx.add_line_level(P.line_rule("kl", 1, lf=True))
    lv = oned.kl_level(1, lf=True)
    s = P.gen_line_samples(0, 1, 0, 2, rule, P.line_rule("kl", 1, lf=True))
    U = ctx.line_forward(lid, s["kappa"], s["n_steps"], s["dt"], rule, lv.n)
    u = oned.solve_sample(lv, oned.Rule1D(kind="kl", T=11.0), 0, 1, 1)
    assert np.max(np.abs(U[1] - u)) <= 1e-11 * np.max(np.abs(u))
