"""The extended-halo scheme on the GPU (paper_2505_06711_amd.halo: one open-cluster plan per
subdomain with a T (r_c + skin) halo, copies' atomic energies weighted 0): it gives the whole-
system result of the oracle, and the oracle's own halo-scheme evaluation, in FP64 and FP32."""
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


@pytest.mark.parametrize("T,prec", [(1, "fp64"), (2, "fp64"), (3, "fp64"), (3, "fp32")])
def test_halo_scheme_matches_oracle(rn, oracle_lib, T, prec):
    import torch
    from paper_2505_06711_amd.halo import HaloEvaluator
    s = systems.water_box(grid=(6, 6, 6), spacing=systems.WATER_BOX_L / 4, seed=85)
    m = models.water_model(T_max=3, seed=85)
    ctx = rn.Context(0)
    h = HaloEvaluator(ctx, rn.Model(m), m, s, T=T, precision=prec, decomp=(2, 2, 2), skin=0.5)
    h.device_inputs(torch)
    E, F, W = h.step(torch)
    torch.cuda.synchronize()
    E, F, W = float(E), F.cpu().numpy(), W.cpu().numpy()
    ref = oracle_lib.evaluate(m, s, T=T, skin=0.5)
    href = oracle_lib.evaluate_halo(m, s, T=T, skin=0.5, decomp=(2, 2, 2), forces=False)
    den = max(abs(ref["energy"]), np.abs(ref["atom_energy"]).sum())
    print("halo %s T=%d: %d cluster atoms for %d (%.2fx); rel E %.2e, max force %.2e, virial %.2e; oracle halo "
          "rows per layer %s" % (prec, T, h.cluster_atoms(), len(s["pos"]), h.cluster_atoms() / len(s["pos"]),
                                  abs(E - ref["energy"]) / den,
                                  np.abs(F - ref["forces"]).max() / np.abs(ref["forces"]).max(),
                                  np.abs(W - ref["virial"]).max() / np.abs(ref["virial"]).max(),
                                  href["work"][:, 0].tolist()), flush=True)
    tol_e, tol_f, tol_w = (1e-12, 1e-10, 1e-10) if prec == "fp64" else (1e-6, 1e-5, 1e-4)
    assert abs(E - ref["energy"]) <= tol_e * den
    assert abs(href["energy"] - ref["energy"]) <= 1e-12 * den
    assert np.abs(F - ref["forces"]).max() <= tol_f * np.abs(ref["forces"]).max()
    assert np.abs(W - ref["virial"]).max() <= tol_w * np.abs(ref["virial"]).max()
