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
