"""GPU tests of the C ABI boundary: levels described by the caller
(lts_add_level / lts_level_arrays), device-resident sample arrays (gathered and
checked on the device), the log-wave-speed input, and ordering against the
caller's torch stream."""
import numpy as np
import pytest

import paper_2106_11117_amd as P
from oracle import fem, lts, mesh

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


def _graded_rule(T):
    return P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), T=T)


def _c0_rule():
    return P.sample_rule(n_blocks=16, sigma=0.25, pulse=(0.2, 0.4, 0.2, 0.4), width=0.05, T=1.0)


@pytest.mark.parametrize("graded", [True, False])
def test_add_level_from_oracle_arrays(ctx, graded):
    """A level passed in as the oracle's own grid and cell arrays: the library's
    derived arrays (flags, lumped mass, QoI weights, blocks) equal the oracle's
    bit for bit, and a solve on it matches the oracle and the generated level."""
    lv = mesh.graded_L_level(32) if graded else mesh.box_refined_level(32)
    ops = fem.operators(lv)
    lid = ctx.add_level(lv.xs, lv.ys, np.where(lv.cell_active, lv.cell_block, 0), lv.cell_fine, lv.cell_qoi,
                        lv.n_blocks, lv.h, lv.p, lv.nu, cell_active=lv.cell_active)
    arr = ctx.level_arrays(lid)
    assert np.array_equal(arr["x"], lv.xs) and np.array_equal(arr["y"], lv.ys)
    flags = arr["flags"]
    assert np.array_equal((flags & P.LTS_NODE_DOF) != 0, lv.dof)
    assert np.array_equal((flags & P.LTS_NODE_P) != 0, lv.Pmask)
    assert np.array_equal((flags & P.LTS_NODE_FPLUS) != 0, lv.Fplus)
    assert np.array_equal(arr["mass"], lv.mass)
    assert np.array_equal(arr["qoi_w"], lv.qoi_w)
    assert np.array_equal(arr["cell_block"], np.where(lv.cell_active, lv.cell_block, -1))
    info = ctx.level_info(lid)
    assert (info["n_dof"], info["n_P"], info["n_Fplus"], info["p"]) == (
        lv.n_dof, int(lv.Pmask.sum()), int(lv.Fplus.sum()), lv.p)
    rule = _graded_rule(2.0) if graded else _c0_rule()
    s = P.gen_samples(0, 0, 0, 4, rule, lv.h)
    q = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    gen = ctx.add_rect_level(P.graded_L_rule(32) if graded else P.box_rule(32))
    assert np.array_equal(q, ctx.forward(gen, s["kappa"], s["x0"], s["n_steps"], s["dt"]))
    for i in range(4):
        u = lts.Solver(ops, s["kappa"][i]).run(lts.pulse(ops, s["x0"][i]), s["dt"][i], int(s["n_steps"][i]))
        qo, sc = float(lts.qoi(ops, u)), float(ops.qoi_w @ np.abs(u))
        assert abs(q[i] - qo) <= 1e-11 * sc, (i, q[i], qo)


def test_device_samples_and_log_wave_speed(ctx):
    """Device-resident inputs give the host path's QoIs bit for bit; g = log c in
    place of kappa gives the same QoIs from host and device arrays (kappa =
    exp(2 g) is formed on the device), within rounding of the host's kappa."""
    torch = _torch()
    lid = ctx.add_rect_level(P.box_rule(32))
    s = P.gen_samples(0, 0, 0, 9, _c0_rule(), 1 / 32)
    dev = torch.device("cuda:0")
    t = {k: torch.tensor(v, device=dev) for k, v in s.items()}
    qh = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    qd = ctx.forward(lid, t["kappa"], t["x0"], t["n_steps"], t["dt"]).cpu().numpy()
    assert np.array_equal(qh, qd)
    qgh = ctx.forward(lid, None, s["x0"], s["n_steps"], s["dt"], g=s["g"])
    qgd = ctx.forward(lid, None, t["x0"], t["n_steps"], t["dt"], g=t["g"]).cpu().numpy()
    assert np.array_equal(qgh, qgd)
    assert np.max(np.abs(qgh - qh)) <= 1e-12 * np.max(np.abs(qh))
    # coupled differences and the adjoint: device outputs equal host outputs
    lc = ctx.add_rect_level(P.box_rule(16))
    sc = P.gen_samples(0, 1, 0, 9, _c0_rule(), 1 / 16)
    fh = ctx.forward_coupled(lid, lc, s["kappa"], s["x0"], s["n_steps"], s["dt"], sc["n_steps"], sc["dt"])
    fd = ctx.forward_coupled(lid, lc, t["kappa"], t["x0"], t["n_steps"], t["dt"],
                             torch.tensor(sc["n_steps"], device=dev), torch.tensor(sc["dt"], device=dev))
    for a, b in zip(fh, fd):
        assert np.array_equal(a, b.cpu().numpy())
    assert np.array_equal(fh[2], fh[0] - fh[1])
    dl = np.linspace(-1.0, 1.0, 9)
    lb = ctx.add_rect_level(P.box_rule(16))
    sb = P.gen_samples(0, 0, 0, 9, P.sample_rule(T=0.3), 1 / 16)
    qbh, gbh = ctx.backward(lb, sb["kappa"], sb["x0"], sb["n_steps"], sb["dt"], dl, K=8)
    tb = {k: torch.tensor(v, device=dev) for k, v in sb.items()}
    qbd, gbd = ctx.backward(lb, tb["kappa"], tb["x0"], tb["n_steps"], tb["dt"], torch.tensor(dl, device=dev), K=8)
    assert np.array_equal(qbh, qbd.cpu().numpy()) and np.array_equal(gbh, gbd.cpu().numpy())


def test_device_inputs_checked_on_device(ctx):
    """Invalid device-resident values are found by the gathering kernel: LTS_ERR_ARG
    before any step, for kappa <= 0, non-finite g and non-finite x0."""
    torch = _torch()
    lid = ctx.add_rect_level(P.box_rule(32))
    s = P.gen_samples(0, 0, 0, 4, _c0_rule(), 1 / 32)
    dev = torch.device("cuda:0")
    t = {k: torch.tensor(v, device=dev) for k, v in s.items()}
    bad_k = t["kappa"].clone()
    bad_k[2, 5] = 0.0
    bad_g = t["g"].clone()
    bad_g[1, 0] = float("inf")
    bad_x = t["x0"].clone()
    bad_x[3, 1] = float("nan")
    for kw, msg in ((dict(kappa=bad_k), "kappa"), (dict(kappa=None, g=bad_g), "g must"),
                    (dict(kappa=t["kappa"], x0=bad_x), "x0")):
        args = dict(kappa=t["kappa"], x0=t["x0"])
        args.update(kw)
        with pytest.raises(P.LtsError) as e:
            ctx.forward(lid, args.pop("kappa"), args.pop("x0"), t["n_steps"], t["dt"], **args)
        assert e.value.code == -1 and msg in str(e.value), str(e.value)
    # the context is usable afterwards
    q = ctx.forward(lid, t["kappa"], t["x0"], t["n_steps"], t["dt"])
    assert torch.isfinite(q).all()


def test_moments_of_tensor_from_another_stream(ctx):
    """A tensor still being computed on the caller's (non-default) torch stream is
    read only after that work: the binding waits for the caller's stream."""
    torch = _torch()
    dev = torch.device("cuda:0")
    side = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(side):
        a = torch.randn(2048, 2048, dtype=torch.float64, device=dev)
        for _ in range(4):
            a = (a @ a) / 2048.0                      # long-running producer on `side`
        x = a[:, 0] - a[:, 1]                          # fresh difference, like Q_f - Q_c
        out = ctx.moments(x)
    ref = x.cpu().numpy()
    assert out[0] == ref.size
    assert abs(out[1] - ref.mean()) <= 1e-12 * np.abs(ref).max()
    assert abs(out[2] / (ref.size - 1) - ref.var(ddof=1)) <= 1e-10 * ref.var(ddof=1)
