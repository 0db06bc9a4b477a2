"""Molecular dynamics on the device through the server (the MD driver's role, Sec. 2.2: atoms are
reassigned to subdomains as they move; Sec. 4.1: NVT runs at 300 K): velocity-Verlet steps on a
system split into subdomains equal those of the whole-system evaluation, one step equals a host
FP64 velocity-Verlet step driven by the oracle's forces, and the stochastic velocity-rescaling
thermostat samples the canonical kinetic-energy distribution (Berendsen does not)."""
import time

import numpy as np
import pytest

from synth import models, systems

pytestmark = pytest.mark.gpu

ELEMENTS = ["H", "O", "Cu"]
MASSES = [systems.MASS_AMU[e] for e in ELEMENTS]
KACCEL = 9.648533212e-3     # (eV/A) / amu in A/fs^2
KB = 8.617333262e-5         # eV/K


@pytest.fixture(scope="module")
def rn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_06711_amd as rn
    return rn


def wait(srv, ticket, sid, timeout=60.0, **kw):
    t0 = time.time()
    while True:
        r = srv.poll(ticket, sid, **kw)
        if r is not None:
            return r
        if time.time() - t0 > timeout:
            raise TimeoutError("request %d did not complete" % ticket)
        time.sleep(0.0002)


def subdomain(pos, L, P):
    w = pos - np.floor(pos / L) * L
    return np.minimum((w / (L / np.array(P))).astype(int), np.array(P) - 1)


def test_md_decomposed_equals_whole_fp64(rn):
    """30 velocity-Verlet steps (1 fs, skin 0.3 A, so the list is rebuilt several times) of a
    648-atom water box: split 2x2x2 equals the whole-system run step by step in FP64, while atoms
    migrate between subdomains at the rebuilds."""
    s = systems.remap_species(systems.water_box(grid=(6, 6, 6), spacing=systems.WATER_BOX_L / 4, seed=80), ELEMENTS)
    m = models.serving_model(T_max=3, seed=3)
    v0 = systems.maxwell_boltzmann(s["species"], ELEMENTS, 300.0, seed=9)
    L = np.diag(s["cell"])
    runs = {}
    for dec in ((1, 1, 1), (2, 2, 2)):
        srv = rn.Server(rn.Model(m), T=3, precision="fp64", skin=0.3, use_graph=True, decomp=dec)
        srv.set_masses(MASSES)
        sid = srv.add_system(s, v0)
        traj = []
        for _ in range(30):
            r = wait(srv, srv.submit_vv(sid, 1.0), sid, positions=True, velocities=True)
            traj.append((r["energy"], r["kinetic"], r["positions"], r["velocities"], r["forces"]))
        runs[dec] = (traj, srv.stats()["list_builds"])
        srv.close()
    a, b = runs[(1, 1, 1)][0], runs[(2, 2, 2)][0]
    worst = [0.0] * 4
    for k, (x, y) in enumerate(zip(a, b)):
        worst[0] = max(worst[0], abs(x[0] - y[0]) / abs(x[0]))
        worst[1] = max(worst[1], np.abs(x[2] - y[2]).max() / L.max())
        worst[2] = max(worst[2], np.abs(x[3] - y[3]).max() / np.abs(x[3]).max())
        worst[3] = max(worst[3], np.abs(x[4] - y[4]).max() / np.abs(x[4]).max())
    moved = int((subdomain(a[-1][2], L, (2, 2, 2)) != subdomain(s["pos"], L, (2, 2, 2))).any(axis=1).sum())
    print("MD split vs whole over 30 steps: rel E %.2e, positions %.2e (of L), velocities %.2e, forces %.2e; "
          "list builds %d / %d; atoms that changed subdomain: %d" % (*worst, runs[(1, 1, 1)][1], runs[(2, 2, 2)][1],
                                                                       moved), flush=True)
    assert worst[0] <= 1e-12
    assert worst[1] <= 1e-12 and worst[2] <= 1e-12 and worst[3] <= 1e-10
    assert runs[(2, 2, 2)][1] >= 3       # the first build and at least two skin-rule rebuilds
    assert moved > 0                     # atoms migrated between subdomains


def test_vv_step_matches_host_fp64_with_oracle_forces(rn, oracle_lib):
    """One velocity-Verlet step on the device (FP64, split 2x2x1) against the same step on the
    host: x1 = x0 + v0 dt + a0 dt^2 / 2, v1 = v0 + (a0 + a1) dt / 2, with a = F / m from the
    oracle's forces at x0 and at x1."""
    s = systems.remap_species(systems.water_box(seed=81), ELEMENTS)
    m = models.serving_model(T_max=3, seed=3)
    v0 = systems.maxwell_boltzmann(s["species"], ELEMENTS, 300.0, seed=10)
    dt = 0.5
    srv = rn.Server(rn.Model(m), T=3, precision="fp64", skin=0.5, use_graph=True, decomp=(2, 2, 1))
    srv.set_masses(MASSES)
    sid = srv.add_system(s, v0)
    r = wait(srv, srv.submit_vv(sid, dt), sid, positions=True, velocities=True)
    srv.close()
    minv = 1.0 / np.array([MASSES[k] for k in s["species"]])[:, None]
    ref0 = oracle_lib.evaluate(m, s, T=3)
    a0 = ref0["forces"] * minv * KACCEL
    x1 = s["pos"] + v0 * dt + 0.5 * a0 * dt * dt
    ref1 = oracle_lib.evaluate(m, dict(s, pos=x1), T=3)
    a1 = ref1["forces"] * minv * KACCEL
    v1 = v0 + 0.5 * (a0 + a1) * dt
    K1 = 0.5 * (v1 * v1 / minv).sum() / KACCEL
    ex = np.abs(r["positions"] - x1).max()
    ev = np.abs(r["velocities"] - v1).max() / np.abs(v1).max()
    ef = np.abs(r["forces"] - ref1["forces"]).max() / np.abs(ref1["forces"]).max()
    print("VV step vs host FP64: positions %.2e A, velocities %.2e, forces %.2e, E %.2e, K %.2e" % (
        ex, ev, ef, abs(r["energy"] - ref1["energy"]) / abs(ref1["energy"]), abs(r["kinetic"] - K1) / K1), flush=True)
    assert ex <= 1e-12 * np.diag(s["cell"]).max()
    assert ev <= 1e-12
    assert ef <= 1e-10
    assert abs(r["energy"] - ref1["energy"]) <= 1e-12 * np.abs(ref1["atom_energy"]).sum()
    assert abs(r["kinetic"] - K1) <= 1e-12 * K1


def test_md_cu100800_fp32_against_host_steps_with_oracle_forces(rn, oracle_lib):
    """The full 100,800-atom Cu workload as the MD-amortised bench runs it (FP32, T = 3,
    r_c = 6 A + 1 A skin, 1 fs, 300 K, through the server): three velocity-Verlet steps against
    the same steps on the host in FP64, driven by the oracle's forces at each host position.
    FP32 forces hold to 1e-5 of the largest component, so after three steps the positions
    agree to far below 1e-6 A, the velocities to 1e-5 of the largest, the energy at the last
    positions to 1e-6 relative."""
    import synth
    w = synth.workload("cu100800")
    m, s = w["model"], w["system"]
    dt, steps = 1.0, 3
    v0 = systems.maxwell_boltzmann(s["species"], m.elements, 300.0, seed=7)
    srv = rn.Server(rn.Model(m), T=3, precision="fp32", skin=w["skin"], use_graph=True)
    srv.set_masses([systems.MASS_AMU[e] for e in m.elements])
    sid = srv.add_system(s, v0)
    for k in range(steps):
        last = k == steps - 1
        r = wait(srv, srv.submit_vv(sid, dt), sid, forces=last, positions=last, velocities=last)
    srv.close()
    minv = 1.0 / np.array([systems.MASS_AMU[m.elements[k]] for k in s["species"]])[:, None]
    x, v = s["pos"].copy(), v0.copy()
    ref = oracle_lib.evaluate(m, s, T=3, skin=w["skin"])
    a = ref["forces"] * minv * KACCEL
    for k in range(steps):
        x = x + v * dt + 0.5 * a * dt * dt
        ref = oracle_lib.evaluate(m, dict(s, pos=x), T=3, skin=w["skin"])
        a1 = ref["forces"] * minv * KACCEL
        v = v + 0.5 * (a + a1) * dt
        a = a1
    ex = np.abs(r["positions"] - x).max()
    ev = np.abs(r["velocities"] - v).max() / np.abs(v).max()
    fmax = np.abs(ref["forces"]).max()
    ef = np.abs(r["forces"] - ref["forces"]).max() / fmax
    den = max(abs(ref["energy"]), np.abs(ref["atom_energy"]).sum())
    print("cu100800 MD, %d FP32 steps vs host FP64 with oracle forces: positions %.2e A, velocities %.2e, "
          "forces %.2e, E %.2e" % (steps, ex, ev, ef, abs(r["energy"] - ref["energy"]) / den), flush=True)
    assert ex <= 1e-6
    assert ev <= 1e-5
    assert ef <= 1e-5
    assert abs(r["energy"] - ref["energy"]) <= 1e-6 * den


def _kinetic_series(rn, thermostat, steps, warm, seed=0):
    s = systems.remap_species(systems.fcc_crystal((4, 4, 4), seed=82), ELEMENTS)
    # a nearly free crystal (energy scale 1e-4): the kinetic energy is then set by the
    # thermostat alone, whose stationary distribution can be checked against the canonical one
    m = models.serving_model(T_max=3, seed=3, energy_scale=1e-4)
    srv = rn.Server(rn.Model(m), T=2, precision="fp32", skin=1.0, use_graph=True, thermostat_K=300.0,
                    thermostat_tau_fs=10.0, thermostat=thermostat, seed=seed)
    srv.set_masses(MASSES)
    sid = srv.add_system(s, systems.maxwell_boltzmann(s["species"], ELEMENTS, 600.0, seed=11))
    K = []
    for k in range(warm + steps):
        r = wait(srv, srv.submit_vv(sid, 1.0), sid, forces=False)
        if k >= warm:
            K.append(r["kinetic"])
    srv.close()
    return np.array(K), len(s["pos"])


def test_csvr_samples_canonical_kinetic_energy(rn):
    """Stochastic velocity rescaling (300 K, tau = 10 fs) from a 600 K start: the kinetic energy's
    mean and variance over 2000 steps match the canonical values N_f k T / 2 and N_f (k T)^2 / 2
    (N_f = 3 n); Berendsen at the same settings reaches the mean with far smaller fluctuations."""
    K, n = _kinetic_series(rn, "csvr", 2000, 200, seed=5)
    nf = 3 * n
    mean_c, var_c = 0.5 * nf * KB * 300.0, 0.5 * nf * (KB * 300.0) ** 2
    Kb, _ = _kinetic_series(rn, "berendsen", 2000, 200)
    print("CSVR: <K>/K0 %.4f, var/var_canonical %.3f; Berendsen: <K>/K0 %.4f, var/var_canonical %.4f" % (
        K.mean() / mean_c, K.var() / var_c, Kb.mean() / mean_c, Kb.var() / var_c), flush=True)
    assert abs(K.mean() / mean_c - 1) < 0.03
    assert 0.7 < K.var() / var_c < 1.4
    assert abs(Kb.mean() / mean_c - 1) < 0.03
    assert Kb.var() / var_c < 0.3
