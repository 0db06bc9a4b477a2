"""GPU parity of the second message form (the radial form: L = 0, the orbital sums as
features, residual message updates) against the FP64 oracle, through the C ABI.

Tolerances are those of the REANN form's parity tests: FP64 |dE| <= 1e-12 (relative to
max(|E|, sum|E_i|)), forces and virial <= 1e-10 of their maxima; FP32 |dE| <= 1e-6, force
RMSE <= 1e-5 of the RMS and every component within 1e-5 * max|F|, virial <= 1e-4 * max|W|;
BF16 within 1% energy and 2% force RMSE per NN layer (a check of operand layouts, not of a
precision).
"""
import numpy as np
import pytest

import synth
from synth import models, systems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_06711_amd as rn
    return rn


@pytest.fixture(scope="module")
def ctx(rn):
    return rn.Context(0)


def rel_energy(E, ref):
    return abs(E - ref["energy"]) / max(abs(ref["energy"]), np.abs(ref["atom_energy"]).sum())


def rel_force_rmse(F, ref):
    return np.sqrt(((F - ref["forces"]) ** 2).mean()) / np.sqrt((ref["forces"] ** 2).mean())


def check_fp64(E, F, W, ref):
    assert rel_energy(E, ref) <= 1e-12
    assert np.abs(F - ref["forces"]).max() <= 1e-10 * np.abs(ref["forces"]).max()
    assert np.abs(W - ref["virial"]).max() <= 1e-10 * np.abs(ref["virial"]).max()


def check_fp32(E, F, W, ref, tag):
    re, rf = rel_energy(E, ref), rel_force_rmse(F, ref)
    fmax, wmax = np.abs(ref["forces"]).max(), np.abs(ref["virial"]).max()
    print("fp32 %s: rel E %.2e, force rel-RMSE %.2e, max component %.2e, virial %.2e" %
          (tag, re, rf, np.abs(F - ref["forces"]).max() / fmax, np.abs(W - ref["virial"]).max() / wmax), flush=True)
    assert re <= 1e-6
    assert rf <= 1e-5
    assert np.abs(F - ref["forces"]).max() <= 1e-5 * fmax
    assert np.abs(W - ref["virial"]).max() <= 1e-4 * wmax


def _eval(rn, ctx, m, s, T, prec, skin=0.0, decomp=(1, 1, 1)):
    return rn.energy_forces(ctx, rn.Model(m), s, T=T, precision=prec, skin=skin, decomp=decomp)


@pytest.mark.parametrize("T", [1, 2, 3])
@pytest.mark.parametrize("decomp", [(1, 1, 1), (2, 2, 2)])
def test_radial_fp64_water(rn, ctx, oracle_lib, T, decomp):
    s = systems.water_box(seed=70)
    m = models.water_model_radial(T_max=3, seed=70, energy_scale=1.2)
    ref = oracle_lib.evaluate(m, s, T=T, skin=0.5)
    check_fp64(*_eval(rn, ctx, m, s, T, "fp64", skin=0.5, decomp=decomp), ref)


@pytest.mark.parametrize("T", [1, 2, 3])
def test_radial_fp32_water(rn, ctx, oracle_lib, T):
    s = systems.water_box(seed=71)
    m = models.water_model_radial(T_max=3, seed=71)
    ref = oracle_lib.evaluate(m, s, T=T, skin=0.5)
    check_fp32(*_eval(rn, ctx, m, s, T, "fp32", skin=0.5, decomp=(2, 1, 1)), ref, "water T=%d" % T)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_radial_cu_with_skin(rn, ctx, oracle_lib, prec):
    s = systems.fcc_crystal((5, 5, 4), seed=72)
    m = models.cu_model_radial(T_max=3, seed=72)
    ref = oracle_lib.evaluate(m, s, T=3, skin=1.0)
    out = _eval(rn, ctx, m, s, 3, prec, skin=1.0)
    if prec == "fp64":
        check_fp64(*out, ref)
    else:
        check_fp32(*out, ref, "cu 5x5x4")


# the fused NN kernels (hidden 64 and 128) and the per-layer path (hidden 96)
SHAPES = {"K8_2x64": dict(K=8, n_hidden=2, hidden=64), "K12_3x128": dict(K=12, n_hidden=3, hidden=128),
          "K12_2x96_per_layer": dict(K=12, n_hidden=2, hidden=96)}


@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_radial_shapes(rn, ctx, oracle_lib, shape, prec):
    s = systems.water_box(seed=73)
    m = models.make_model(["H", "O"], L=0, r_c=5.0, width=0.5, T_max=3, seed=74, bias_std=1.0, form="radial",
                          **SHAPES[shape])
    ref = oracle_lib.evaluate(m, s, T=3, skin=0.5)
    out = _eval(rn, ctx, m, s, 3, prec, skin=0.5, decomp=(1, 2, 1))
    if prec == "fp64":
        check_fp64(*out, ref)
    elif prec == "fp32":
        check_fp32(*out, ref, shape)
    else:
        E, F, W = out
        re, rf = rel_energy(E, ref), rel_force_rmse(F, ref)
        print("radial bf16 %s: rel E %.2e, force rel-RMSE %.2e" % (shape, re, rf), flush=True)
        depth = SHAPES[shape]["n_hidden"] + 1
        assert re <= 1e-2 * depth
        assert rf <= 2e-2 * depth


def test_radial_device_plan_matches_host_call(rn, ctx, oracle_lib):
    """The device-pointer plan (forward, backward) gives the host entry point's results."""
    import torch
    s = systems.water_box(seed=75)
    m = models.water_model_radial(T_max=3, seed=75)
    model = rn.Model(m)
    E0, F0, W0 = rn.energy_forces(ctx, model, s, T=3, precision="fp32", skin=0.5)
    plan = rn.Plan(ctx, model, s, T=3, precision="fp32", skin=0.5)
    pos = torch.tensor(s["pos"], dtype=torch.float64, device="cuda")
    E = torch.zeros((), dtype=torch.float64, device="cuda")
    F = torch.zeros_like(pos)
    W = torch.zeros((3, 3), dtype=torch.float64, device="cuda")
    for _ in range(2):
        plan.forward(pos, E)
        plan.backward(F, virial=W)
    torch.cuda.synchronize()
    assert float(E) == E0
    np.testing.assert_array_equal(F.cpu().numpy(), F0)
    np.testing.assert_array_equal(W.cpu().numpy(), W0)


def test_radial_fp8_is_refused(rn, ctx):
    s = systems.water_box(seed=76)
    m = models.water_model_radial(T_max=2, seed=76)
    with pytest.raises(rn.ReannError):
        _eval(rn, ctx, m, s, 2, "fp8")


def test_radial_cu100800_fp32_against_oracle(rn, ctx, oracle_lib):
    """The 100,800-atom Cu crystal in the radial form (T = 3, the workload's skin), against the
    oracle on the full system."""
    w = synth.workload("cu100800")
    m = models.cu_model_radial(T_max=3, seed=0)
    ref = oracle_lib.evaluate(m, w["system"], T=3, skin=w["skin"])
    check_fp32(*_eval(rn, ctx, m, w["system"], 3, "fp32", skin=w["skin"]), ref, "cu100800")


def test_radial_md_decomposed_equals_whole_fp64(rn):
    """The MD driver with the radial form: 20 velocity-Verlet steps (1 fs, skin 0.3 A, so the
    list is rebuilt on the way) of a 648-atom water box split 2x2x2 equal the whole-system run
    in FP64."""
    import time
    s = systems.water_box(grid=(6, 6, 6), spacing=systems.WATER_BOX_L / 4, seed=81)
    m = models.water_model_radial(T_max=3, seed=81)
    v0 = systems.maxwell_boltzmann(s["species"], ["H", "O"], 300.0, seed=10)
    runs = {}
    for dec in ((1, 1, 1), (2, 2, 2)):
        srv = rn.Server(rn.Model(m), T=3, precision="fp64", skin=0.3, use_graph=True, decomp=dec)
        srv.set_masses([systems.MASS_AMU[e] for e in ("H", "O")])
        sid = srv.add_system(s, v0)
        traj = []
        for _ in range(20):
            t = srv.submit_vv(sid, 1.0)
            t0 = time.time()
            while (r := srv.poll(t, sid, positions=True, velocities=True)) is None:
                assert time.time() - t0 < 60.0
                time.sleep(0.0002)
            traj.append((r["energy"], r["positions"], r["velocities"]))
        runs[dec] = (traj, srv.stats()["list_builds"])
        srv.close()
    L = np.diag(s["cell"]).max()
    for x, y in zip(runs[(1, 1, 1)][0], runs[(2, 2, 2)][0]):
        assert abs(x[0] - y[0]) <= 1e-12 * abs(x[0])
        assert np.abs(x[1] - y[1]).max() <= 1e-12 * L
        assert np.abs(x[2] - y[2]).max() <= 1e-12 * np.abs(x[2]).max()
    assert runs[(2, 2, 2)][1] >= 2


# ---- the literal reading of Eq. (1): only the squares (the "diag" form), on the per-layer path --

@pytest.mark.parametrize("T", [1, 2, 3])
@pytest.mark.parametrize("decomp", [(1, 1, 1), (2, 2, 1)])
def test_diag_fp64_water(rn, ctx, oracle_lib, T, decomp):
    s = systems.water_box(seed=110)
    m = models.water_model_diag(T_max=3, seed=110)
    ref = oracle_lib.evaluate(m, s, T=T, skin=0.5)
    check_fp64(*_eval(rn, ctx, m, s, T, "fp64", skin=0.5, decomp=decomp), ref)


@pytest.mark.parametrize("case", ["water", "cu"])
def test_diag_fp32(rn, ctx, oracle_lib, case):
    if case == "water":
        s, m, skin = systems.water_box(seed=111), models.water_model_diag(T_max=3, seed=111), 0.5
    else:
        s, m, skin = systems.fcc_crystal((5, 5, 4), seed=112), models.cu_model_diag(T_max=3, seed=112), 1.0
    ref = oracle_lib.evaluate(m, s, T=3, skin=skin)
    check_fp32(*_eval(rn, ctx, m, s, 3, "fp32", skin=skin, decomp=(2, 1, 1)), ref, "diag " + case)


def test_diag_bf16(rn, ctx, oracle_lib):
    s = systems.water_box(seed=113)
    m = models.water_model_diag(T_max=3, seed=113)
    ref = oracle_lib.evaluate(m, s, T=3, skin=0.5)
    E, F, W = _eval(rn, ctx, m, s, 3, "bf16", skin=0.5)
    re, rf = rel_energy(E, ref), rel_force_rmse(F, ref)
    print("diag bf16: rel E %.2e, force rel-RMSE %.2e" % (re, rf), flush=True)
    assert re <= 3e-2 and rf <= 6e-2


def test_diag_fp8_is_refused(rn, ctx):
    with pytest.raises(rn.ReannError):
        _eval(rn, ctx, models.water_model_diag(T_max=2, seed=114), systems.water_box(seed=114), 2, "fp8")
