"""The device-pointer path captured in a HIP graph (through torch.cuda.graph): with the plan's
list kept by the caller (reann_plan_set_list_policy(0) + reann_plan_update_list), a forward +
backward makes no host synchronisation or allocation, so it can be captured and replayed.
Every replay is checked against an eager evaluation of the same positions (bitwise: the same
kernels on the same list) and, in FP64, against the oracle; eager work and synchronisations
run between the replays."""
import numpy as np
import pytest

from synth import models, systems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_06711_amd as rn
    return rn


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_forward_backward_replayed_from_a_graph(rn, oracle_lib, prec):
    import torch
    s = systems.water_box(seed=90)
    m = models.water_model(T_max=3, seed=90)
    ctx = rn.Context(0)
    model = rn.Model(m)
    skin = 0.6
    plan = rn.Plan(ctx, model, s, T=3, precision=prec, skin=skin)
    plan.set_list_policy(False)
    pos = torch.tensor(s["pos"], dtype=torch.float64, device="cuda")
    E = torch.zeros((), dtype=torch.float64, device="cuda")
    F = torch.zeros_like(pos)
    W = torch.zeros((3, 3), dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        assert plan.update_list(pos) is True          # the first build
        for _ in range(2):                            # warm-up on the capture stream
            plan.forward(pos, E)
            plan.backward(F, virial=W)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        plan.forward(pos, E)
        plan.backward(F, virial=W)
    rng = np.random.default_rng(0)
    E2 = torch.zeros_like(E); F2 = torch.zeros_like(F); W2 = torch.zeros_like(W)
    for k in range(4):
        # displacements below skin/2 in total: the list stays valid
        x = s["pos"] + rng.uniform(-0.1, 0.1, s["pos"].shape)
        pos.copy_(torch.tensor(x, dtype=torch.float64))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        Eg, Fg, Wg = float(E), F.cpu().numpy(), W.cpu().numpy()
        assert plan.update_list(pos) is False          # still within the skin
        plan.forward(pos, E2)                          # eager, same list
        plan.backward(F2, virial=W2)
        torch.cuda.synchronize()
        assert Eg == float(E2)
        np.testing.assert_array_equal(Fg, F2.cpu().numpy())
        np.testing.assert_array_equal(Wg, W2.cpu().numpy())
        if prec == "fp64":
            ref = oracle_lib.evaluate(m, dict(s, pos=x), T=3)
            assert abs(Eg - ref["energy"]) <= 1e-12 * np.abs(ref["atom_energy"]).sum()
            np.testing.assert_allclose(Fg, ref["forces"], rtol=0, atol=1e-10 * np.abs(ref["forces"]).max())
    # beyond the skin: the caller's update rebuilds, and the graph is captured again
    x = s["pos"] + rng.uniform(-0.6, 0.6, s["pos"].shape)
    pos.copy_(torch.tensor(x, dtype=torch.float64))
    with torch.cuda.stream(side):
        assert plan.update_list(pos) is True
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2, stream=side):
        plan.forward(pos, E)
        plan.backward(F, virial=W)
    g2.replay()
    torch.cuda.synchronize()
    ref_plan = rn.Plan(ctx, model, dict(s, pos=x), T=3, precision=prec, skin=skin)
    ref_plan.forward(pos, E2)
    ref_plan.backward(F2, virial=W2)
    torch.cuda.synchronize()
    scale = np.abs(F2.cpu().numpy()).max()
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert abs(float(E) - float(E2)) <= tol * max(1.0, abs(float(E2)))
    assert np.abs(F.cpu().numpy() - F2.cpu().numpy()).max() <= tol * scale


def test_forward_without_a_list_is_refused(rn):
    import torch
    s = systems.water_box(seed=91)
    ctx = rn.Context(0)
    plan = rn.Plan(ctx, rn.Model(models.water_model(T_max=2, seed=91)), s, T=2, precision="fp32")
    plan.set_list_policy(False)
    pos = torch.tensor(s["pos"], dtype=torch.float64, device="cuda")
    E = torch.zeros((), dtype=torch.float64, device="cuda")
    with pytest.raises(rn.ReannError):
        plan.forward(pos, E)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_automatic_list_policy_keeps_and_rebuilds(rn, oracle_lib, prec):
    """The plan's default policy: each forward checks the skin rule on the device, with the
    forward on the checked list queued behind the check, and rebuilds and repeats the forward
    when the list is stale.  Positions move below and beyond skin/2 in turn; every step is
    checked against the FP64 oracle at the same positions (FP64: 1e-10; FP32: the path's
    bounds), and the rebuilds happen exactly when an atom has moved more than skin/2 since the
    last build."""
    import torch
    s = systems.water_box(seed=91)
    m = models.water_model(T_max=3, seed=91)
    ctx = rn.Context(0)
    model = rn.Model(m)
    skin = 0.6
    plan = rn.Plan(ctx, model, s, T=3, precision=prec, skin=skin)
    plan.set_timing(True)         # its per-phase counts include the list builds
    E = torch.zeros((), dtype=torch.float64, device="cuda")
    F = torch.zeros((len(s["pos"]), 3), dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(3)
    ref_pos = s["pos"].copy()     # positions of the last build
    x = s["pos"].copy()
    builds = 0
    for k in range(8):
        if k > 0:
            x = x + rng.uniform(-1, 1, x.shape) * (0.02 if k % 3 else 0.4)   # every third step jumps
        moved = np.sqrt(((x - ref_pos) ** 2).sum(1)).max()
        stale = k == 0 or moved > 0.5 * skin
        if stale:
            ref_pos = x.copy()
            builds += 1
        pos = torch.tensor(x, dtype=torch.float64, device="cuda")
        g0 = plan.generation()
        plan.forward(pos, E)
        plan.backward(F)
        torch.cuda.synchronize()
        ref = oracle_lib.evaluate(m, dict(s, pos=x), T=3, skin=skin)
        Ek, Fk = float(E), F.cpu().numpy()
        if prec == "fp64":
            assert abs(Ek - ref["energy"]) <= 1e-10 * abs(ref["energy"]), k
            np.testing.assert_allclose(Fk, ref["forces"], rtol=0, atol=1e-10 * np.abs(ref["forces"]).max())
        else:
            assert abs(Ek - ref["energy"]) <= 1e-6 * abs(ref["energy"]), k
            np.testing.assert_allclose(Fk, ref["forces"], rtol=0, atol=1e-5 * np.abs(ref["forces"]).max())
        assert plan.generation() > g0
    assert plan.timing()["launches"]["nlist"] == builds >= 3
