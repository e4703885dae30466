"""The library's host build of multi-level LTS tiers (lts_mlts_host) against
the oracle's tier sets: node tiers of the halving rule and of given cell
tiers bit for bit, sizes, the update count, rejected descriptions."""
import numpy as np
import pytest

import paper_2106_11117_amd as P
from oracle import mesh, mlts


def _node_tiers(lv, ct, T):
    """Largest j with the node in P_j (0 off P_1), on the node grid."""
    out = np.zeros(lv.nyn * lv.nxn, dtype=np.uint8)
    ids = lv.dof_ids
    for j, Pj in enumerate(mlts.tier_projectors(lv, ct, T), start=1):
        out[ids[Pj > 0]] = j
    return out.reshape(lv.nyn, lv.nxn)


@pytest.mark.parametrize("n_base,T,ps", [(32, 5, [2, 2, 2, 2, 2]), (64, 3, [4, 2, 8]), (32, 1, [16])])
def test_halving_rule_matches_oracle(n_base, T, ps):
    lv = mesh.graded_L_level(n_base)
    ct = mlts.tiers_by_leg(lv, T)
    h = P.mlts_host(P.graded_L_rule(n_base), ps)
    want = _node_tiers(lv, ct, T)
    assert np.array_equal(h["node_tier"], want)
    nP = [int((want >= j).sum()) for j in range(1, T + 1)]
    assert h["n_P"] == nP and h["p"] == ps and h["n_tiers"] == T
    K, span = 0, 1
    for p in ps:
        K += span * (p - 1)
        span *= p
    assert h["phases"] == K
    upd, rate = lv.n_dof - nP[0], 1
    for j in range(T):
        rate *= ps[j]
        upd += rate * (nP[j] - (nP[j + 1] if j + 1 < T else 0))
    assert h["updates_per_step"] == upd
    assert h["n_tiles"] >= 1 and h["max_region"] <= 2048 and h["threads"] in (256, 512, 1024)


def test_given_cell_tiers_match_oracle():
    """Caller-given tiers on the box-refined C0 level: tier 2 the fine cells
    whose midpoint lies in the inner half of the refined box."""
    lv = mesh.box_refined_level(32, box=(0.4375, 0.5625))
    mx = 0.5 * (lv.xs[:-1] + lv.xs[1:])
    MX, MY = np.meshgrid(mx, mx)
    inner = (abs(MX - 0.5) < 0.03) & (abs(MY - 0.5) < 0.03)
    ct = np.where(lv.cell_active & lv.cell_fine, np.where(inner, 2, 1), 0).astype(np.uint8)
    h = P.mlts_host(P.box_rule(32, box=(0.4375, 0.5625)), [2, 2], ct)
    assert np.array_equal(h["node_tier"], _node_tiers(lv, ct, 2))
    assert 0 < h["n_P"][1] < h["n_P"][0]


def test_region_cap():
    """Smaller region caps give more, smaller tiles on smaller workgroups."""
    rule = P.box_rule(32, box=(0.4375, 0.5625))
    big = P.mlts_host(rule, [2, 2])
    small = P.mlts_host(rule, [2, 2], max_region=512)
    assert small["max_region"] <= 512 and small["threads"] == 256
    assert small["n_tiles"] > big["n_tiles"] and np.array_equal(small["node_tier"], big["node_tier"])


def test_rejected_descriptions():
    rule = P.graded_L_rule(32)
    with pytest.raises(P.LtsError):
        P.mlts_host(rule, [])
    with pytest.raises(P.LtsError):
        P.mlts_host(rule, [2] * 6)
    with pytest.raises(P.LtsError):
        P.mlts_host(rule, [2, 17])
    with pytest.raises(P.LtsError):
        P.mlts_host(P.graded_L_rule(512), [16, 16, 16])   # regions of radius 4095 do not fit
    with pytest.raises(P.LtsError):
        P.mlts_host(rule, [2, 2], max_region=300)
    with pytest.raises(P.LtsError):                       # radius 31 at the band crossing: above 1024 nodes
        P.mlts_host(P.graded_L_rule(128), [2] * 5, max_region=1024)
    lv = mesh.graded_L_level(32)
    ct = mlts.tiers_by_leg(lv, 2).astype(np.uint8)
    bad = ct.copy()
    bad[~(lv.cell_active & lv.cell_fine)] = 1          # a coarse cell in a tier
    with pytest.raises(P.LtsError):
        P.mlts_host(rule, [2, 2], bad)
    bad = ct.copy()
    bad[ct == 2] = 3                                   # beyond n_tiers
    with pytest.raises(P.LtsError):
        P.mlts_host(rule, [2, 2], bad)
    bad = ct.copy()
    bad[ct >= 1] = 0                                   # a fine cell in no tier
    with pytest.raises(P.LtsError):
        P.mlts_host(rule, [2, 2], bad)
