"""GPU tests of the continuous-batching server (reann_server_* / reann_submit / reann_poll)."""
import time

import numpy as np
import pytest

from synth import models, systems

pytestmark = pytest.mark.gpu

MASSES = [1.008, 15.999, 63.546]


@pytest.fixture(scope="module")
def rn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_06711_amd as rn
    return rn


@pytest.fixture(scope="module")
def model_params():
    return models.serving_model(T_max=3, seed=3)


def mix(seed, sizes):
    out = []
    for k, n in enumerate(sizes):
        s = systems.water_box_n(n, seed=seed + k) if k % 2 == 0 else systems.fcc_n(n, seed=seed + k)
        out.append(systems.remap_species(s, ["H", "O", "Cu"]))
    return out


def wait(srv, ticket, sid, timeout=60.0, **kw):
    t0 = time.time()
    while True:
        r = srv.poll(ticket, sid, **kw)
        if r is not None:
            return r
        if time.time() - t0 > timeout:
            raise TimeoutError("request %d did not complete" % ticket)
        time.sleep(0.0005)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("use_graph", [True, False])
def test_result_alone_equals_result_in_mix(rn, model_params, use_graph, prec):
    sys_list = mix(100, [300, 500, 2000, 96, 4000, 864, 1500, 200, 3000, 108])
    model = rn.Model(model_params)
    srv = rn.Server(model, T=3, precision=prec, skin=1.0, use_graph=use_graph)
    ids = [srv.add_system(s) for s in sys_list]
    alone = wait(srv, srv.submit_eval(ids[2], sys_list[2]["pos"]), ids[2])
    tickets = [(srv.submit_eval(i, s["pos"]), i) for i, s in zip(ids, sys_list)]
    tickets += [(srv.submit_eval(i, s["pos"]), i) for i, s in zip(ids, sys_list)]
    res = {}
    for t, i in tickets:
        res.setdefault(i, []).append(wait(srv, t, i))
    for r in res[ids[2]]:
        assert r["energy"] == alone["energy"]
        np.testing.assert_array_equal(r["forces"], alone["forces"])
        np.testing.assert_array_equal(r["virial"], alone["virial"])
    st = srv.stats()
    assert st["completed"] == len(tickets) + 1
    if use_graph:
        assert st["graph_replays"] > 0
    srv.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_server_matches_plan_path(rn, model_params, prec):
    sys_list = mix(200, [600, 1372])
    model = rn.Model(model_params)
    ctx = rn.Context(0)
    srv = rn.Server(model, T=3, precision=prec, skin=1.0, use_graph=True)
    for s in sys_list:
        sid = srv.add_system(s)
        # several replays of the same graph with eager work in between
        for rep in range(3):
            r = wait(srv, srv.submit_eval(sid, s["pos"]), sid)
            E, F, W = rn.energy_forces(ctx, model, s, T=3, precision=prec, skin=1.0)
            assert r["energy"] == pytest.approx(E, rel=1e-12, abs=1e-12), rep
            np.testing.assert_allclose(r["forces"], F, rtol=0, atol=1e-9 * np.abs(F).max())


def test_bf16_server_against_fp64_oracle(rn, model_params, oracle_lib):
    """The serving precision (BF16 atomic-NN products) on a water box and an FCC crystal of the
    serving mix, through the server's captured graphs, against the FP64 oracle: errors in
    meV/atom and meV/A.  The bounds are sanity limits (a layout mistake gives errors of the
    order of the energies themselves); the printed values are the measurement."""
    sys_list = mix(250, [600, 1372])
    srv = rn.Server(rn.Model(model_params), T=3, precision="bf16", skin=1.0, use_graph=True)
    for s in sys_list:
        sid = srv.add_system(s)
        r = wait(srv, srv.submit_eval(sid, s["pos"]), sid)
        ref = oracle_lib.evaluate(model_params, s, T=3, skin=1.0)
        n = len(s["pos"])
        de = abs(r["energy"] - ref["energy"]) / n * 1e3
        frmse = np.sqrt(((r["forces"] - ref["forces"]) ** 2).mean()) * 1e3
        frms = np.sqrt((ref["forces"] ** 2).mean())
        print("serving bf16, %d atoms: |dE| = %.3f meV/atom (E/N = %.3f eV), force RMSE = %.2f meV/A "
              "(force RMS %.3f eV/A)" % (n, de, ref["energy"] / n, frmse, frms), flush=True)
        assert de / 1e3 <= 2e-2 * np.abs(ref["atom_energy"]).mean()
        assert frmse / 1e3 <= 5e-2 * frms
    srv.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_serving_mix_systems_against_fp64_oracle(rn, oracle_lib, prec):
    """Systems of the serving workload itself (its model, its 256-system mix with seed 0: the
    smallest, the largest, and quartiles, water boxes and FCC crystals), evaluated together in
    one server, against the FP64 oracle.  FP32: the path's bounds (energy 1e-6 relative, every
    force component 1e-5 of the largest); BF16: the sanity limits of the BF16 test above, with
    the errors printed in meV/atom and meV/A."""
    m = models.serving_model(T_max=3, seed=0)
    mix = systems.serving_mix(256, seed=0, elements=m.elements)
    order = np.argsort([len(x["pos"]) for x in mix])
    pick = sorted(set(int(order[q]) for q in (0, 1, 64, 128, 192, 254, 255)))
    srv = rn.Server(rn.Model(m), T=3, precision=prec, skin=1.0, use_graph=True)
    ids = {k: srv.add_system(mix[k]) for k in pick}
    tickets = {k: srv.submit_eval(ids[k], mix[k]["pos"]) for k in pick}   # all in flight together
    for k in pick:
        r = wait(srv, tickets[k], ids[k])
        ref = oracle_lib.evaluate(m, mix[k], T=3, skin=1.0)
        n = len(mix[k]["pos"])
        de = abs(r["energy"] - ref["energy"])
        den = max(abs(ref["energy"]), np.abs(ref["atom_energy"]).sum())
        fmax = np.abs(ref["forces"]).max()
        frms = np.sqrt((ref["forces"] ** 2).mean())
        frmse = np.sqrt(((r["forces"] - ref["forces"]) ** 2).mean())
        print("serving mix system %d (%d atoms, %s) %s: |dE| = %.3g meV/atom (rel %.2e), force RMSE = %.3g meV/A "
              "(max component %.2e of the largest)" % (k, n, "water" if k % 2 == 0 else "fcc", prec, de / n * 1e3,
                                                       de / den, frmse * 1e3, np.abs(r["forces"] - ref["forces"]).max() / fmax),
              flush=True)
        if prec == "fp32":
            assert de <= 1e-6 * den
            assert np.abs(r["forces"] - ref["forces"]).max() <= 1e-5 * fmax
        else:
            assert de / n <= 2e-2 * np.abs(ref["atom_energy"]).mean()
            assert frmse <= 5e-2 * frms
    srv.close()


# Other model shapes through the server (its graphs capture the same kernels as the plan
# path): K = 8 and K = 4 edge passes, one and two hidden layers, and a hidden width that the
# fused NN kernels do not take (the per-layer path).
SERVE_SHAPES = {
    "L2_K8_2x64": dict(L=2, K=8, n_hidden=2, hidden=64),
    "L1_K4_1x64": dict(L=1, K=4, n_hidden=1, hidden=64),
    "L2_K12_2x96_per_layer": dict(L=2, K=12, n_hidden=2, hidden=96),
}


@pytest.mark.parametrize("shape", list(SERVE_SHAPES))
def test_server_matches_plan_path_other_models(rn, shape):
    m = models.make_model(["H", "O"], r_c=5.0, width=0.5, T_max=3, seed=7, **SERVE_SHAPES[shape])
    model = rn.Model(m)
    ctx = rn.Context(0)
    srv = rn.Server(model, T=3, precision="fp32", skin=1.0, use_graph=True)
    for k, n in enumerate([300, 1200]):
        s = systems.remap_species(systems.water_box_n(n, seed=40 + k), ["H", "O"])
        sid = srv.add_system(s)
        for rep in range(2):
            r = wait(srv, srv.submit_eval(sid, s["pos"]), sid)
            E, F, W = rn.energy_forces(ctx, model, s, T=3, precision="fp32", skin=1.0)
            assert r["energy"] == pytest.approx(E, rel=1e-12, abs=1e-12), rep
            np.testing.assert_allclose(r["forces"], F, rtol=0, atol=1e-9 * np.abs(F).max())
    srv.close()


def test_velocity_verlet_steps_and_rebuilds(rn, model_params):
    s = mix(300, [1500])[0]
    model = rn.Model(model_params)
    srv = rn.Server(model, T=3, precision="fp32", skin=0.4, use_graph=True)
    srv.set_masses(MASSES)
    vel = systems.maxwell_boltzmann(s["species"], ["H", "O", "Cu"], 300.0, seed=1)
    sid = srv.add_system(s, vel)
    energies = []
    for k in range(40):
        r = wait(srv, srv.submit_vv(sid, 0.5), sid, positions=True)
        energies.append(r["energy"])
    assert np.all(np.isfinite(energies))
    # positions moved, so the list was rebuilt at least once with a 0.4 A skin
    assert not np.allclose(r["positions"], s["pos"])
    srv.close()


def test_admission_under_a_tiny_budget(rn, model_params):
    sys_list = mix(400, [3000, 3000, 3000, 3000])
    sys_list = [sys_list[0], sys_list[2], dict(sys_list[0], pos=sys_list[0]["pos"] + 0.05),
                dict(sys_list[2], pos=sys_list[2]["pos"] - 0.05)]
    model = rn.Model(model_params)
    probe = rn.Server(model, T=3, precision="fp32", skin=1.0, hbm_budget_bytes=1 << 20)
    with pytest.raises(rn.ReannError) as e:
        probe.add_system(sys_list[0])
    assert e.value.status == -4
    probe.close()
    # room for about two of these four systems at a time: requests complete through eviction
    big = rn.Server(model, T=3, precision="fp32", skin=1.0, hbm_budget_bytes=1 << 40)
    one = big.add_system(sys_list[0])
    wait(big, big.submit_eval(one, sys_list[0]["pos"]), one)
    per_sys = big.stats()["resident_bytes"]
    big.close()
    budget = int(per_sys * 2.5)
    srv = rn.Server(model, T=3, precision="fp32", skin=1.0, hbm_budget_bytes=budget)
    ids = [srv.add_system(s) for s in sys_list]
    ref = {}
    for rep in range(2):
        ts = [(srv.submit_eval(i, s["pos"]), i) for i, s in zip(ids, sys_list)]
        for t, i in ts:
            r = wait(srv, t, i)
            if rep == 0:
                ref[i] = r["energy"]
            else:
                assert r["energy"] == ref[i]
    st = srv.stats()
    print("tiny budget:", budget, st, flush=True)
    assert st["resident_bytes"] <= budget
    assert st["completed"] == 8
    srv.close()


def test_bad_requests_do_not_stop_the_server(rn, model_params):
    s = mix(500, [400])[0]
    model = rn.Model(model_params)
    srv = rn.Server(model, T=3, precision="bf16", skin=1.0)
    sid = srv.add_system(s)
    with pytest.raises(rn.ReannError):
        srv.submit_eval(sid + 99, s["pos"])               # unknown system
    with pytest.raises(rn.ReannError) as e:
        srv.submit_vv(sid, 1.0)                           # no masses yet
    assert e.value.status == -7
    bad = s["pos"].copy()
    bad[3, 1] = np.nan
    with pytest.raises(rn.ReannError):
        srv.submit_eval(sid, bad)
    r = wait(srv, srv.submit_eval(sid, s["pos"]), sid)
    assert np.isfinite(r["energy"])
    from paper_2505_06711_amd._binding import _Result, load
    import ctypes as C
    assert load().reann_poll(srv.handle, C.c_uint64(123456), C.byref(_Result())) == -6   # unknown ticket
    srv.close()


def _vv_run(rn, model_params, s, dt, steps, prec, T0=0.0, tau=0.0, temp=300.0):
    srv = rn.Server(rn.Model(model_params), T=3, precision=prec, skin=1.0, use_graph=True, thermostat_K=T0,
                    thermostat_tau_fs=tau)
    srv.set_masses(MASSES)
    v = systems.maxwell_boltzmann(s["species"], ["H", "O", "Cu"], temp, seed=5)
    sid = srv.add_system(s, v)
    Ep, K = [], []
    for _ in range(steps):
        r = wait(srv, srv.submit_vv(sid, dt), sid, forces=False)
        Ep.append(r["energy"])
        K.append(r["kinetic"])
    srv.close()
    return np.array(Ep), np.array(K)


def test_vv_conserves_energy_to_second_order(rn, model_params):
    # constant-energy velocity Verlet (FP64 forces) over the same 20 fs at two time steps: the
    # total energy stays within a small fraction of the potential energy it exchanges, and its
    # deviation shrinks ~4x when the step halves (the method is second order)
    s = systems.remap_species(systems.fcc_n(400, seed=1), ["H", "O", "Cu"])
    dev = {}
    for dt in (0.5, 0.25):
        Ep, K = _vv_run(rn, model_params, s, dt, int(round(20 / dt)), "fp64")
        Et = Ep + K
        dev[dt] = np.abs(Et - Et[0]).max()
        assert dev[dt] < 1e-3 * (Ep.max() - Ep.min())
        assert K.min() > 0
    assert 3.0 < dev[0.5] / dev[0.25] < 5.0, dev


def test_berendsen_thermostat_pulls_toward_target(rn, model_params):
    # from a 3000 K start the random-weight potential keeps heating the crystal at constant
    # energy; the thermostat (300 K, tau = 10 fs) brings it down instead
    s = systems.remap_species(systems.fcc_n(400, seed=1), ["H", "O", "Cu"])
    kB, n = 8.617333262e-5, len(s["pos"])
    _, K_nve = _vv_run(rn, model_params, s, 0.5, 200, "fp32", temp=3000.0)
    _, K_th = _vv_run(rn, model_params, s, 0.5, 200, "fp32", T0=300.0, tau=10.0, temp=3000.0)
    T_nve, T_th = 2 * K_nve / (3 * n * kB), 2 * K_th / (3 * n * kB)
    assert T_nve[-1] > T_nve[0]
    assert T_th[-1] < 0.5 * T_th[0]
    assert T_th[-1] < 0.25 * T_nve[-1]


@pytest.mark.parametrize("use_graph", [True, False])
def test_skipped_outputs_change_nothing_but_the_copy(rn, model_params, use_graph):
    # two copies of one system at constant energy follow the same trajectory whether or not the
    # steps bring their vectors back; a poll that asks for a skipped vector is refused and the
    # result stays for a poll that does not
    from paper_2505_06711_amd._binding import ReannError
    s = mix(11, [900])[0]
    srv = rn.Server(rn.Model(model_params), T=3, precision="fp32", skin=0.5, use_graph=use_graph)
    srv.set_masses(MASSES)
    v = systems.maxwell_boltzmann(s["species"], ["H", "O", "Cu"], 600.0, seed=2)
    a, b = srv.add_system(s, v), srv.add_system(s, v)
    full = dict(forces=True, positions=True, velocities=True)
    for k in range(24):
        skip = () if k % 8 == 7 else (("forces", "positions", "velocities") if k % 2 else ("positions",))
        ta, tb = srv.submit_vv(a, 0.5, skip=skip), srv.submit_vv(b, 0.5)
        rb = wait(srv, tb, b, **full)
        want = {n: n not in skip for n in ("forces", "positions", "velocities")}
        if skip:
            with pytest.raises(ReannError):
                wait(srv, ta, a, **full)
        ra = wait(srv, ta, a, **want)
        assert ra["energy"] == rb["energy"] and ra["kinetic"] == rb["kinetic"]
        np.testing.assert_array_equal(ra["virial"], rb["virial"])
        for n, w in want.items():
            if w:
                np.testing.assert_array_equal(ra[n], rb[n])
    assert srv.stats()["list_builds"] > 2          # rebuilds happened along the way
    import ctypes as C
    from paper_2505_06711_amd._binding import _Request, load
    r = _Request(sys_id=a, kind=1, dt_fs=0.5, skip_outputs=8)
    assert load().reann_submit(srv.handle, C.byref(r), C.byref(C.c_uint64())) == -1   # unknown bit
    srv.close()


def test_lists_stay_valid_when_the_previous_step_decides_them(rn, model_params):
    # velocity Verlet at a constant dt with a thin skin, so that lists are rebuilt often and
    # each step's list is decided by the displacement the previous step predicted for it: every
    # step's energy and forces (FP64) equal a fresh evaluation at the same positions with a
    # list built for them, to rounding.  A list kept one step too long would miss pairs that
    # came within the cutoff.
    s = mix(21, [700])[0]
    model = rn.Model(model_params)
    ctx = rn.Context(0)
    srv = rn.Server(model, T=3, precision="fp64", skin=0.3, use_graph=True)
    srv.set_masses(MASSES)
    v = systems.maxwell_boltzmann(s["species"], ["H", "O", "Cu"], 1500.0, seed=4)
    sid = srv.add_system(s, v)
    for k in range(40):
        r = wait(srv, srv.submit_vv(sid, 1.0), sid, forces=True, positions=True)
        E, F, W = rn.energy_forces(ctx, model, dict(s, pos=r["positions"]), T=3, precision="fp64", skin=0.3)
        assert r["energy"] == pytest.approx(E, rel=1e-11, abs=1e-11), k
        np.testing.assert_allclose(r["forces"], F, rtol=0, atol=1e-10 * np.abs(F).max())
    st = srv.stats()
    assert st["list_builds"] >= 4, st
    assert st["predicted_list_decisions"] >= 38, st
    assert st["skin_checks"] <= 2, st
    srv.close()


def test_eval_request_reports_no_kinetic_energy(rn, model_params):
    s = mix(7, [200])[0]
    srv = rn.Server(rn.Model(model_params), T=2, precision="fp32", skin=1.0)
    sid = srv.add_system(s)
    r = wait(srv, srv.submit_eval(sid, s["pos"]), sid)
    assert r["kinetic"] == 0.0
    srv.close()


def test_injected_fault_fails_one_request_and_the_server_keeps_serving(rn, monkeypatch):
    """A request refused for its inputs fails alone (here forced through the server's test hook
    REANN_SERVER_FAULT_TICKET): its system is set aside (later requests get REANN_E_STATE), and
    the other systems' requests complete and match a server without the fault."""
    import time
    m = rn.Model(models.serving_model(T_max=3, seed=7))
    systems_ = mix(90, [120, 256, 180])

    def run(fault):
        if fault:
            monkeypatch.setenv("REANN_SERVER_FAULT_TICKET", "2")
        srv = rn.Server(m, T=3, precision="fp32", skin=0.5, use_graph=True)
        monkeypatch.delenv("REANN_SERVER_FAULT_TICKET", raising=False)
        ids = [srv.add_system(s) for s in systems_]
        tickets = [(srv.submit_eval(sid, s["pos"]), sid) for sid, s in zip(ids, systems_)]   # tickets 1, 2, 3
        out = {}
        for t, sid in tickets:
            t0 = time.time()
            while True:
                try:
                    r = srv.poll(t, sid)
                except rn.ReannError as e:
                    r = e
                if r is not None:
                    break
                assert time.time() - t0 < 60
                time.sleep(0.0005)
            out[t] = r
        # a second round: the failed system is refused, the others still serve
        again = {}
        for sid, s in zip(ids, systems_):
            t = srv.submit_eval(sid, s["pos"])
            t0 = time.time()
            while True:
                try:
                    r = srv.poll(t, sid)
                except rn.ReannError as e:
                    r = e
                if r is not None:
                    break
                assert time.time() - t0 < 60
                time.sleep(0.0005)
            again[sid] = r
        srv.close()
        return ids, out, again

    ids, ok, ok2 = run(False)
    ids_f, bad, bad2 = run(True)
    assert isinstance(bad[2], rn.ReannError) and bad[2].status == -1 and "injected" in str(bad[2])
    for t in (1, 3):
        assert not isinstance(bad[t], Exception)
        assert bad[t]["energy"] == ok[t]["energy"]
        np.testing.assert_array_equal(bad[t]["forces"], ok[t]["forces"])
    failed_sid = ids_f[1]
    assert isinstance(bad2[failed_sid], rn.ReannError) and bad2[failed_sid].status == -7
    for k in (0, 2):
        assert not isinstance(bad2[ids_f[k]], Exception)
        assert bad2[ids_f[k]]["energy"] == ok2[ids[k]]["energy"]
