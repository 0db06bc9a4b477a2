"""A model written by Model.save and read back by reann_model_load evaluates bit for bit
like the model it was saved from (GPU)."""
import pytest

from synth import models, systems

pytestmark = pytest.mark.gpu


def test_loaded_model_evaluates_identically(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_06711_amd as rn
    p = models.water_model(T_max=3, seed=2)
    s = systems.water_box()
    ctx = rn.Context()
    m0 = rn.Model(p)
    spec = str(tmp_path / "m.json")
    m0.save(spec)
    m1 = rn.Model.load(spec)
    for prec in ("fp64", "fp32"):
        E0, F0, W0 = rn.energy_forces(ctx, m0, s, T=3, precision=prec)
        E1, F1, W1 = rn.energy_forces(ctx, m1, s, T=3, precision=prec)
        assert E0 == E1
        assert (F0 == F1).all() and (W0 == W1).all()


def test_forward_backward_dev_match_plan_calls():
    # reann_forward_dev / reann_backward_dev are the plan's forward and backward under the
    # boundary's names: same results, bit for bit
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_06711_amd as rn
    from paper_2505_06711_amd._binding import check, load
    p = models.water_model(T_max=2, seed=6)
    s = systems.water_box()
    ctx = rn.Context()
    plan = rn.Plan(ctx, rn.Model(p), s, T=2, precision="fp32", skin=0.5)
    pos = torch.tensor(s["pos"], dtype=torch.float64, device="cuda")
    E0, E1 = (torch.zeros((), dtype=torch.float64, device="cuda") for _ in range(2))
    F0, F1 = (torch.zeros((len(s["pos"]), 3), dtype=torch.float64, device="cuda") for _ in range(2))
    W0, W1 = (torch.zeros((3, 3), dtype=torch.float64, device="cuda") for _ in range(2))
    st = torch.cuda.current_stream().cuda_stream
    plan.forward(pos, E0)
    plan.backward(F0, virial=W0)
    check(load().reann_forward_dev(plan.handle, pos.data_ptr(), E1.data_ptr(), st))
    check(load().reann_backward_dev(plan.handle, None, F1.data_ptr(), W1.data_ptr(), st))
    torch.cuda.synchronize()
    assert E0.item() == E1.item()
    assert torch.equal(F0, F1) and torch.equal(W0, W1)
