"""Throughput benchmark: REANN energy + force + virial evaluations on one MI355X.

One step = one full evaluation of the workload (neighbour-list reuse check, T message-
passing layers forward, the hand-written backward for forces and virial) with the
positions already resident in HBM.  Default workload: the 100,800-atom FCC Cu-like
crystal, r_c = 6 A with a 1 A skin, T = 3, L = 2, K = 12, 3x128 SiLU atomic NNs, FP32.

Prints ONE JSON line (rank 0).  Per-kernel durations come from HIP events recorded by
the library on the evaluation stream during the timed steps; the roofline entry is
for the kernel phase with the largest share of the step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "energy+force atom-steps/s at T=3 on 1 MI355X vs FP64 oracle; serve p50/p99"
HBM_PEAK_GBS = 8000.0
# MI355X published peaks.  The FP32 vector figure (256 CUs x 2.4 GHz x 256 flop/clk/CU) needs
# packed FP32 instructions, which every kernel here is built without; the unpacked rate, half
# of it, is the reachable ceiling and also sets the ridge point used to classify a kernel.
PEAK_TFLOPS = {"fp32_vector": 157.3, "fp64_vector": 78.6, "fp32_mfma": 157.3, "bf16_mfma": 2500.0,
               "fp8_mfma": 5000.0, "fp64_mfma": 78.6}
UNPACKED_TFLOPS = {"fp32_vector": 78.6, "fp64_vector": 78.6}


def describe(name, w):
    m = w["model"]
    return ("%s: %d atoms, r_c=%g A + %g A skin, T=%d, L=%d, K=%d, %dx%d SiLU atomic NNs, decomp %s"
            % (name, len(w["system"]["pos"]), m.r_c, w["skin"], w["T"], m.L, m.K, m.n_hidden, m.hidden,
               "x".join(map(str, w["decomp"]))))


def work_model(w, n_pairs_local, n_in_cutoff, prec):
    """Algorithmic work of one launch of each single-kernel phase (one MP layer, all atoms).

    Per atom and layer, with n_l list entries (r_c + skin) and n_c in-cutoff edges per atom,
    Lam = (L+1)(L+2)(L+3)/6 angular components and rs bytes per working value:
      edge forward  bytes 4 n_l + 24 + rs K + rs Lam K;   VALU n_c (2 Lam K + 7 K + 40)
      edge adjoint, centre role  bytes 4 n_l + 24 + 2 rs K + rs Lam K + 3 rs;
                    VALU n_c (4 Lam K + 12 K + 80) (the adjoint-message terms reuse the
                    sums the gradient forms, so every launch counts the same work)
      edge adjoint, neighbour role  bytes per in-cutoff local edge: one slot index and one
                    record (rs (4 + K), or 4 rs without message terms); + rs (3 + K) out
      atomic NN     2 (F H + (h - 1) H^2 + H K_out) flop (forward; the adjoint the same)
    (an exp counts as 4 VALU slots; bytes count each atom's own data once and exclude cache
    re-reads of gathered neighbours)."""
    m, n = w["model"], len(w["system"]["pos"])
    K, L = m.K, m.L
    lam = (L + 1) * (L + 2) * (L + 3) // 6
    F, H, nh = m.F, m.hidden, m.n_hidden
    rs = 8 if prec == "fp64" else 4
    n_l, n_c = n_pairs_local / n, n_in_cutoff / n
    out = {}
    out["edge_fwd"] = dict(bytes=n * (4 * n_l + 24 + rs * K + rs * lam * K), flops=n * n_c * (2 * lam * K + 7 * K + 40))
    out["adj_centre"] = dict(bytes=n * (4 * n_l + 24 + 2 * rs * K + rs * lam * K + 3 * rs),
                             flops=n * n_c * (4 * lam * K + 12 * K + 80))
    out["adj_gather"] = dict(bytes=n_in_cutoff * (4 + rs * (4 + K)) + n * rs * (3 + K),
                             bytes_nocbar=n_in_cutoff * (4 + 4 * rs) + n * rs * 3)
    out["nn"] = dict(flops_msg=2 * n * (F * H + (nh - 1) * H * H + H * K),
                     flops_en=2 * n * (F * H + (nh - 1) * H * H + H))
    return out


def load_traffic(kernel, workload, precision):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3 counter summary, or
    None when there is none or the kernel's source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s_%s.md" % (kernel, workload, precision))
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    src = os.path.join(ROOT, "paper_2505_06711_amd", "csrc", fields.get("source", ""))
    if not os.path.isfile(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != fields.get("source_sha256"):
        return None
    return float(fields["traffic_bytes_per_dispatch"])


KERNEL_OF_PHASE = {"edge_fwd": "k_edge_fwd", "adj_centre": "k_adj_centre", "adj_gather": "k_adj_gather",
                   "nn_fwd": "k_mlp_fwd", "nn_bwd": "k_mlp_bwd", "density": "k_density",
                   "density_adj": "k_density_vjp"}


def kernel_work(wk, tim, T, prec, phase):
    """(algorithmic flops, algorithmic bytes, peak key) of one launch of a single-kernel phase."""
    nla = tim["launches"][phase]
    steps = max(1, tim["steps"])
    vec = "fp64_vector" if prec == "fp64" else "fp32_vector"
    if phase == "edge_fwd":
        return wk["edge_fwd"]["flops"], wk["edge_fwd"]["bytes"], vec
    if phase == "adj_centre":
        return wk["adj_centre"]["flops"], wk["adj_centre"]["bytes"], vec
    if phase == "adj_gather":   # T - 1 launches gather message terms, one does not
        return 0.0, ((T - 1) * wk["adj_gather"]["bytes"] + wk["adj_gather"]["bytes_nocbar"]) / T, None
    # atomic NNs: T - 1 message NNs and one energy NN per step (the adjoint the same work)
    flops = ((T - 1) * wk["nn"]["flops_msg"] + wk["nn"]["flops_en"]) / (nla / steps)
    return flops, None, {"fp64": "fp64_mfma", "fp32": "fp32_mfma", "bf16": "bf16_mfma", "fp8": "fp8_mfma"}[prec]


def kernel_entry(wk, tim, T, prec, phase):
    """Achieved rate of one kernel against its roofline: algorithmic work per launch over the
    average launch time (library HIP events on the evaluation stream)."""
    nla = tim["launches"][phase]
    per_launch_ms = tim["ms"][phase] / nla
    flops, byts, kind = kernel_work(wk, tim, T, prec, phase)
    sec = per_launch_ms * 1e-3
    e = dict(kernel=KERNEL_OF_PHASE[phase], per_launch_ms=round(per_launch_ms, 4), launches=nla,
             algorithmic_flops_per_launch=round(flops), algorithmic_bytes_per_launch=None if byts is None else round(byts))
    if byts is not None:
        e["hbm_gbs"] = round(byts / sec / 1e9, 1)
        e["hbm_frac"] = round(byts / sec / 1e9 / HBM_PEAK_GBS, 4)
    if kind is not None and flops > 0:
        tf = flops / sec / 1e12
        e["tflops"] = round(tf, 3)
        e["peak_tflops"] = PEAK_TFLOPS[kind]
        e["tflops_frac"] = round(tf / PEAK_TFLOPS[kind], 4)
        if kind in UNPACKED_TFLOPS:
            e["peak_tflops_unpacked"] = UNPACKED_TFLOPS[kind]
            e["tflops_frac_unpacked"] = round(tf / UNPACKED_TFLOPS[kind], 4)
    return e


def roofline(wk, tim, T, prec, workload):
    """Roofline entry of the single-kernel phase with the largest share of the step.  A vector
    kernel is HBM-bound when its bytes at 8 TB/s take longer than its flops at the reachable
    (unpacked) vector rate, ALU-bound otherwise; `peak` is the published figure, and the
    unpacked one is reported beside it."""
    phases = [p for p in ("edge_fwd", "adj_centre", "adj_gather", "nn_fwd", "nn_bwd")
              if tim["launches"].get(p, 0) > 0]
    dom = max(phases, key=lambda p: tim["ms"][p])
    e = kernel_entry(wk, tim, T, prec, dom)
    flops, byts, kind = kernel_work(wk, tim, T, prec, dom)
    reach = UNPACKED_TFLOPS.get(kind, PEAK_TFLOPS.get(kind)) if kind else None
    if kind is None or (byts is not None and kind.endswith("vector")
                        and flops / (reach * 1e12) < byts / (HBM_PEAK_GBS * 1e9)):
        roof = dict(bound="hbm", achieved=e["hbm_gbs"], peak=HBM_PEAK_GBS, unit="GB/s", frac=e["hbm_frac"])
    else:
        roof = dict(bound="alu" if kind.endswith("vector") else "mfma", achieved=e["tflops"],
                    peak=PEAK_TFLOPS[kind], unit="TFLOP/s", frac=e["tflops_frac"])
        if kind in UNPACKED_TFLOPS:
            roof.update(peak_unpacked=UNPACKED_TFLOPS[kind], frac_unpacked=e["tflops_frac_unpacked"])
    roof["traffic"] = load_traffic(KERNEL_OF_PHASE[dom], workload, prec)
    roof.update({k: e[k] for k in ("kernel", "per_launch_ms", "launches", "algorithmic_flops_per_launch",
                                   "algorithmic_bytes_per_launch")})
    return roof


def cpu_baseline(workload_name, T, max_seconds=30.0):
    """The FP64 oracle timed on this host on the same workload (one full evaluation)."""
    import oracle
    import synth
    oracle.build(force=False)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = int(min(cores, 16))
    w = synth.workload(workload_name)
    s = w["system"]
    n = len(s["pos"])
    sample = "full %s system, one energy+force+virial evaluation (its neighbour search included)" % workload_name
    # bound the CPU work: on hosts far slower than expected fall back to an FCC sub-box of
    # the same lattice, density and model
    if workload_name == "cu100800" and threads < 4:
        s = synth.systems.fcc_crystal((12, 12, 12))
        n = len(s["pos"])
        sample = "12x12x12-cell sub-box (6,912 atoms) of the same crystal and model"
    t0 = time.perf_counter()
    oracle.evaluate(w["model"], s, T=T, skin=w["skin"], threads=threads)
    dt = time.perf_counter() - t0
    out = dict(value=n / dt, unit="atom-steps/s", cores=threads, kind="oracle", sample=sample,
               seconds=round(dt, 3), nproc=os.cpu_count(), cpu_model=_cpu_model())
    # one core, on a sub-box of the same crystal and model (a few seconds of work)
    if workload_name == "cu100800":
        s1 = synth.systems.fcc_crystal((12, 12, 12))
        t0 = time.perf_counter()
        oracle.evaluate(w["model"], s1, T=T, skin=w["skin"], threads=1)
        dt1 = time.perf_counter() - t0
        out["single_core"] = dict(value=len(s1["pos"]) / dt1, unit="atom-steps/s", cores=1,
                                  sample="12x12x12-cell sub-box (6,912 atoms) of the same crystal and model",
                                  seconds=round(dt1, 3))
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def md_amortised(rn, w, precision, steps=100, dt_fs=1.0, temperature=300.0):
    """The workload run as molecular dynamics: `steps` velocity-Verlet steps of dt_fs on the
    device (one request each, through the server), the list rebuilt by the skin rule when
    needed, the vectors left on the device (energies come back every step).  Reports the rate
    including rebuilds and the number of builds; then as many more steps that bring forces,
    positions and velocities back every step, for their cost."""
    import synth
    m, s = w["model"], w["system"]
    srv = rn.Server(rn.Model(m), T=w["T"], precision=precision, skin=w["skin"], use_graph=True)
    srv.set_masses([synth.systems.MASS_AMU[e] for e in m.elements])
    vel = synth.systems.maxwell_boltzmann(s["species"], m.elements, temperature, seed=7)
    sid = srv.add_system(s, vel)

    everything = ("forces", "positions", "velocities")

    def run_one(skip):
        t = srv.submit_vv(sid, dt_fs, skip=skip)
        want = {k: k not in skip for k in everything}
        while True:
            r = srv.poll(t, sid, **want)
            if r is not None:
                return r
            time.sleep(0.0001)

    run_one(everything)                 # first build, graph capture
    b0 = srv.stats()["list_builds"]
    t0 = time.perf_counter()
    for _ in range(steps):
        r = run_one(everything)
    el = time.perf_counter() - t0
    builds = srv.stats()["list_builds"] - b0
    final_energy = r["energy"]
    run_one(())                         # graph capture for the full copy
    t0 = time.perf_counter()
    for _ in range(steps):
        run_one(())
    el_vec = time.perf_counter() - t0
    srv.close()
    n = len(s["pos"])
    return dict(steps=steps, dt_fs=dt_fs, temperature_K=temperature, ms_per_step=round(el / steps * 1e3, 4),
                atom_steps_per_s=round(n * steps / el, 1), list_rebuilds=int(builds),
                final_energy=final_energy, ms_per_step_vectors_every_step=round(el_vec / steps * 1e3, 4),
                note="host submit/poll per step included; vectors stay on the device except in the second figure")


def serve_bench(rn, seconds=4.0, n_systems=256, seed=0):
    """Serving: 1 fs velocity-Verlet requests over independent systems (sizes log-uniform
    64-20,000 atoms, half water boxes, half FCC crystals), r_c = 5 A, T = 3, BF16 atomic NNs,
    constant energy.  A system has at most one request in flight (a step needs the previous
    forces).  The random-weight potentials do not hold the atoms near their start: the share
    of steps that rebuild a list grows from ~15% to ~40% over tens of seconds of serving.  So
    every phase below starts from the same freshly added systems (after one warm-up step
    each), and all phases serve the same workload.  Closed loop first, keeping c requests in
    flight on random idle systems for c = 1 .. all, to find the saturation rate (the best of
    them); then open-loop Poisson arrivals at 0.5, 0.8 and 0.95 of it, each arrival served by
    a random idle system; the front end keeps at most as many requests in flight as the best
    closed-loop point and queues the rest FIFO.  Latency is submit -> result ready on the
    library's clock in the closed loop, and arrival -> result seen by this driver in the open
    loop."""
    import synth
    m = synth.models.serving_model(T_max=3, seed=seed)
    model = rn.Model(m)
    mix = synth.systems.serving_mix(n_systems, seed=seed, elements=m.elements)
    vels = [synth.systems.maxwell_boltzmann(s["species"], m.elements, 300.0, seed=seed + k) for k, s in enumerate(mix)]
    rng = np.random.default_rng(seed)

    def fresh():
        srv = rn.Server(model, T=3, precision="bf16", skin=1.0, use_graph=True)
        srv.set_masses([synth.systems.MASS_AMU[e] for e in m.elements])
        ids = [srv.add_system(s, v) for s, v in zip(mix, vels)]
        sizes = {sid: len(s["pos"]) for sid, s in zip(ids, mix)}
        inflight = {sid: srv.submit_vv(sid, 1.0) for sid in ids}   # residency, lists, graph capture
        t0 = time.perf_counter()
        while inflight:
            for sid, t in list(inflight.items()):
                if srv.poll(t, sid, forces=False) is not None:
                    del inflight[sid]
        return srv, ids, sizes, time.perf_counter() - t0

    def drain(srv, sizes, inflight, idle, lat, done, clock):
        for sid, (t, t_arr) in list(inflight.items()):
            r = srv.poll(t, sid, forces=False)
            if r is not None:
                del inflight[sid]
                idle.append(sid)
                lat.append(r["latency_s"] if clock == "library" else time.perf_counter() - t_arr)
                done[0] += sizes[sid]

    curve, warm = [], None
    for c in (1, 2, 4, 8, 16, 64, n_systems):
        srv, ids, sizes, w = fresh()
        warm = w if warm is None else warm
        lat, done, inflight, idle = [], [0], {}, list(ids)
        b0 = srv.stats()["list_builds"]
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            while len(inflight) < c and idle:
                sid = idle.pop(int(rng.integers(len(idle))))
                inflight[sid] = (srv.submit_vv(sid, 1.0), None)
            drain(srv, sizes, inflight, idle, lat, done, "library")
        el = time.perf_counter() - t0
        builds = srv.stats()["list_builds"] - b0
        srv.close()
        curve.append(dict(in_flight=c, requests_per_s=round(len(lat) / el, 1), atom_steps_per_s=round(done[0] / el, 1),
                          p50_ms=round(1e3 * float(np.percentile(lat, 50)), 3),
                          p99_ms=round(1e3 * float(np.percentile(lat, 99)), 3),
                          rebuild_fraction=round(builds / max(len(lat), 1), 3)))
    best = max(curve, key=lambda d: d["requests_per_s"])
    out = dict(systems=n_systems, atoms_resident=int(sum(len(s["pos"]) for s in mix)), warmup_s=round(warm, 2),
               phase_s=seconds, saturation=dict(best), closed_loop=curve)
    sat_rate, cap = best["requests_per_s"], best["in_flight"]
    levels = []
    for frac in (0.5, 0.8, 0.95):
        srv, ids, sizes, _ = fresh()
        rate = frac * sat_rate
        lat, done, inflight, idle, queue = [], [0], {}, list(ids), []
        b0 = srv.stats()["list_builds"]
        t_next = time.perf_counter()
        t0 = t_next
        while time.perf_counter() - t0 < seconds:
            now = time.perf_counter()
            while t_next <= now:      # arrivals
                queue.append(t_next)
                t_next += rng.exponential(1.0 / rate)
            drain(srv, sizes, inflight, idle, lat, done, "driver")
            while queue and idle and len(inflight) < cap:
                sid = idle.pop(int(rng.integers(len(idle))))
                inflight[sid] = (srv.submit_vv(sid, 1.0), queue.pop(0))
        el = time.perf_counter() - t0
        while inflight:
            drain(srv, sizes, inflight, idle, [], [0], "driver")
        builds = srv.stats()["list_builds"] - b0
        stats = srv.stats()
        srv.close()
        levels.append(dict(load=frac, offered_requests_per_s=round(rate, 1), atom_steps_per_s=round(done[0] / el, 1),
                           p50_ms=round(1e3 * float(np.percentile(lat, 50)), 3) if lat else None,
                           p99_ms=round(1e3 * float(np.percentile(lat, 99)), 3) if lat else None,
                           completed=len(lat), queued_at_end=len(queue), max_in_flight=cap,
                           rebuild_fraction=round(builds / max(len(lat), 1), 3)))
    out["open_loop"] = levels
    out["stats_last_phase"] = stats
    return out


def time_steps(rn, torch, ctx, model, w, T, precision, steps, warmup, want_forces=False, exchange="messages"):
    """ms per energy+force step of `w` at T (device-resident positions), and optionally the
    energy and forces of the last step (caller atom order)."""
    s = w["system"]
    pos = torch.tensor(s["pos"], dtype=torch.float64, device="cuda")
    E = torch.zeros((), dtype=torch.float64, device="cuda")
    F = torch.zeros_like(pos)
    plan = rn.Plan(ctx, model, s, T=T, precision=precision, decomp=w["decomp"], skin=w["skin"], exchange=exchange)
    for _ in range(1 + warmup):
        plan.forward(pos, E)
        plan.backward(F)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        plan.forward(pos, E)
        plan.backward(F)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    out = (ms, float(E), F.cpu().numpy()) if want_forces else (ms,)
    del plan
    return out


def fit_linear_T(rows):
    t = np.array([r["T"] for r in rows], float)
    y = np.array([r["ms_per_step"] for r in rows])
    A = np.stack([np.ones_like(t), t], 1)
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    fit = A @ coef
    r2 = 1 - ((y - fit) ** 2).sum() / max(1e-30, ((y - y.mean()) ** 2).sum())
    return dict(a=round(float(coef[0]), 4), b_per_layer=round(float(coef[1]), 4), r2=round(float(r2), 6),
                residuals_ms=[round(float(v), 4) for v in (y - fit)])


def tsweep(rn, torch, ctx, model, w, name, precision, Ts, steps, warmup):
    """Cost of one energy+force step against the number of MP layers T (Sec. 2.2: the
    same neighbour list and ghost shell serve every layer, so the cost is linear in T)."""
    n = len(w["system"]["pos"])
    rows = []
    for T in Ts:
        ms = time_steps(rn, torch, ctx, model, w, T, precision, steps, warmup)[0]
        rows.append(dict(T=T, ms_per_step=round(ms, 4), atom_steps_per_s=round(n / (ms * 1e-3), 1)))
        print("tsweep %s T=%d %.3f ms" % (name, T, ms), file=sys.stderr, flush=True)
    return dict(metric="cost vs number of MP layers T", workload=describe(name, w), precision=precision,
                n_atoms=n, rows=rows, fit_ms=fit_linear_T(rows))


def decomposed_water(rn, torch, ctx, steps=10, warmup=2, Ts=(1, 2, 3, 4, 6)):
    """The 1,207,296-atom water box split 2x2x2 with the per-layer ghost exchange, FP32: the
    step time at T = 3 and the cost against T (fit a + b T, R^2, residuals)."""
    import synth
    w = synth.workload("water1207296")
    n = len(w["system"]["pos"])
    model = rn.Model(w["model"])
    info = rn.build_neighbors(ctx, w["system"], w["model"].r_c, w["skin"], w["decomp"]).info()
    sw = tsweep(rn, torch, ctx, model, w, "water1207296", "fp32", Ts, steps, warmup)
    t3 = [r for r in sw["rows"] if r["T"] == 3][0]
    return dict(workload=describe("water1207296", w), precision="fp32", n_atoms=n, ghosts=info["n_ghosts"],
                list_pairs=info["n_local_pairs"], ms_per_step_T3=t3["ms_per_step"],
                atom_steps_per_s_T3=t3["atom_steps_per_s"], steps_per_T=steps, tsweep=sw)


def halo_ablation(rn, torch, ctx, exchange_rows, Ts=(1, 2, 3, 4), steps=3, warmup=1):
    """The redundancy the per-layer exchange avoids (Sec. 2.2, Fig. 2): the 1,207,296-atom
    water box split 2x2x2 evaluated by the extended-halo scheme (each subdomain an open cluster
    of every copy within T (r_c + skin) of its box, recomputed at every layer, no exchange
    between layers; paper_2505_06711_amd.halo) against the per-layer exchange at the same
    split (`exchange_rows`, the decomposed_water sweep).  FP32, ms per energy+force+virial step."""
    import synth
    from paper_2505_06711_amd.halo import HaloEvaluator
    w = synth.workload("water1207296")
    s, m = w["system"], w["model"]
    n = len(s["pos"])
    model = rn.Model(m)
    ex = {r["T"]: r["ms_per_step"] for r in exchange_rows}
    rows = []
    for T in Ts:
        h = HaloEvaluator(ctx, model, m, s, T=T, precision="fp32", decomp=w["decomp"], skin=w["skin"])
        h.device_inputs(torch)
        for _ in range(1 + warmup):
            h.step(torch)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(steps):
            h.step(torch)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        rows.append(dict(T=T, halo_ms_per_step=round(ms, 3), exchange_ms_per_step=ex.get(T),
                         halo_over_exchange=round(ms / ex[T], 3) if T in ex else None,
                         cluster_atoms=h.cluster_atoms(), cluster_atoms_per_atom=round(h.cluster_atoms() / n, 3)))
        print("halo ablation T=%d %.2f ms (%d cluster atoms)" % (T, ms, h.cluster_atoms()), file=sys.stderr, flush=True)
        del h
    return dict(workload=describe("water1207296", w), precision="fp32", scheme="extended halo T (r_c + skin), "
                "every layer over the whole cluster, vs per-layer ghost exchange", rows=rows)


def precision_ladder(rn, torch, ctx, w, name, steps=20, warmup=3):
    """The Cu workload with the atomic-NN products in FP32, BF16 and FP8 e4m3 (FP32
    accumulation): atom-steps/s and the errors against the FP64 oracle's stored energy and 256
    sampled forces (tests/golden/<workload>_T3.json, written by a script that calls only the
    oracle), in meV/atom and meV/A."""
    import hashlib
    path = os.path.join(ROOT, "tests", "golden", "%s_T%d.json" % (name, w["T"]))
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    s = w["system"]
    if hashlib.sha256(np.ascontiguousarray(s["pos"], dtype=np.float64).tobytes()).hexdigest() != g["positions_sha256"]:
        return None
    n = len(s["pos"])
    idx = np.array(g["sample_index"])
    Fref = np.array(g["sample_forces"]).reshape(-1, 3)
    model = rn.Model(w["model"])
    rungs = []
    for prec in ("fp32", "bf16", "fp8"):
        ms, E, F = time_steps(rn, torch, ctx, model, w, w["T"], prec, steps, warmup, want_forces=True)
        rungs.append(dict(precision=prec, ms_per_step=round(ms, 4), atom_steps_per_s=round(n / (ms * 1e-3), 1),
                          energy_error_mev_per_atom=float("%.4g" % (abs(E - g["energy"]) / n * 1e3)),
                          rel_energy_error=float("%.3g" % (abs(E - g["energy"]) / max(abs(g["energy"]),
                                                                                    g["sum_abs_atom_energy"]))),
                          force_rmse_mev_per_a=float("%.4g" % (np.sqrt(((F[idx] - Fref) ** 2).mean()) * 1e3))))
        print("ladder %s %.3f ms" % (prec, ms), file=sys.stderr, flush=True)
    return dict(workload=describe(name, w), reference="FP64 oracle: stored energy and 256 sampled forces",
                energy_per_atom_ev=round(g["energy"] / n, 5), force_rms_ev_per_a=round(g["force_rms"], 5),
                rungs=rungs)


def message_forms(rn, torch, ctx, w, name, reann_ms, steps=10, warmup=2, Ts=(1, 2, 3, 4)):
    """The second message form on the same exchange (the radial form: L = 0, the K orbital sums
    as features, residual message updates) on the same system, list and skin: ms per
    energy+force step at T = 3 in FP32 and BF16, and its cost against T in FP32."""
    import synth
    m = synth.models.cu_model_radial(T_max=max(Ts), seed=0) if name == "cu100800" else None
    if m is None:
        return None
    n = len(w["system"]["pos"])
    model = rn.Model(m)
    rows = []
    for prec in ("fp32", "bf16"):
        ms = time_steps(rn, torch, ctx, model, w, 3, prec, steps, warmup)[0]
        rows.append(dict(precision=prec, T=3, ms_per_step=round(ms, 4), atom_steps_per_s=round(n / (ms * 1e-3), 1)))
        print("forms radial %s %.3f ms" % (prec, ms), file=sys.stderr, flush=True)
    wr = dict(w, model=m)
    sw = tsweep(rn, torch, ctx, model, wr, name + " (radial form)", "fp32", Ts, steps, warmup)
    return dict(workload=describe(name, wr), form="radial: L = 0, F = K = %d features, residual updates" % m.K,
                model=dict(K=m.K, n_hidden=m.n_hidden, hidden=m.hidden, r_c=m.r_c), rows=rows,
                reann_form_fp32_ms_per_step=round(reann_ms, 4), tsweep=sw)


def node_feature_exchange(rn, torch, ctx, w, name, steps=10, warmup=2, Ts=(1, 2, 3)):
    """The communication the paper contrasts its scheme with (end of Sec. 2.2): exchanging node
    features (here each ghost's orbital sums S^t, NL K values) and running the message NNs for
    every ghost in every subdomain, against exchanging messages (K values) and running the NNs
    for locals only.  Same results; ms per energy+force step on the Cu crystal against T, and
    on the 1.2M-atom water box split 2x2x2 at T = 3, FP32."""
    import synth
    out = {}
    cases = [(name, w, Ts)]
    if name == "cu100800":
        cases.append(("water1207296", synth.workload("water1207296"), (3,)))
    for wname, ww, ts in cases:
        m = ww["model"]
        model = rn.Model(m)
        n = len(ww["system"]["pos"])
        info = rn.build_neighbors(ctx, ww["system"], m.r_c, ww["skin"], ww["decomp"]).info()
        nl_ = (m.L + 1) * (m.L + 2) * (m.L + 3) // 6
        rows = []
        for T in ts:
            r = dict(T=T)
            for ex in ("messages", "node_features"):
                ms = time_steps(rn, torch, ctx, model, ww, T, "fp32", steps, warmup, exchange=ex)[0]
                r[ex + "_ms_per_step"] = round(ms, 4)
                print("exchange %s %s T=%d %.3f ms" % (wname, ex, T, ms), file=sys.stderr, flush=True)
            r["node_over_messages"] = round(r["node_features_ms_per_step"] / r["messages_ms_per_step"], 3)
            rows.append(r)
        out[wname] = dict(workload=describe(wname, ww), n_atoms=n, ghosts=info["n_ghosts"],
                          message_nn_rows_per_layer=dict(messages=n, node_features=n + info["n_ghosts"]),
                          values_exchanged_per_ghost_per_layer=dict(messages=m.K, node_features=nl_ * m.K),
                          rows=rows)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cu100800")
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16", "fp8"])
    ap.add_argument("--T", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the precision ladder and the decomposed 1.2M-atom water run")
    ap.add_argument("--serve-seconds", type=float, default=4.0)
    ap.add_argument("--tsweep", default=None,
                    help="comma list of T values: time each T on the workload instead of the headline run")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (the known-size "
                         "kernel that scales rocprofv3's FETCH_SIZE / WRITE_SIZE readings)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the subdomain exchange is "
              "emulated inside one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if a.copy_calibration:
        nbytes = a.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_calibration_bytes=nbytes, repeats=3)), flush=True)
        return
    import synth
    import paper_2505_06711_amd as rn

    w = synth.workload(a.workload)
    if a.T is not None:
        w["T"] = a.T
    s, m, T = w["system"], w["model"], w["T"]
    n = len(s["pos"])
    print("bench: %s precision=%s steps=%d warmup=%d" % (describe(a.workload, w), a.precision, a.steps, a.warmup),
          file=sys.stderr, flush=True)
    ctx = rn.Context(0, torch.cuda.current_stream())
    model = rn.Model(m)
    if a.tsweep:
        print(json.dumps(tsweep(rn, torch, ctx, model, w, a.workload, a.precision,
                                [int(x) for x in a.tsweep.split(",")], a.steps, a.warmup)), flush=True)
        return
    plan = rn.Plan(ctx, model, s, T=T, precision=a.precision, decomp=w["decomp"], skin=w["skin"])
    pos = torch.tensor(s["pos"], dtype=torch.float64, device="cuda")
    E = torch.zeros((), dtype=torch.float64, device="cuda")
    F = torch.zeros_like(pos)
    W = torch.zeros((3, 3), dtype=torch.float64, device="cuda")

    def step():
        plan.forward(pos, E)
        plan.backward(F, virial=W)

    t_build = time.perf_counter()
    step()
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t_build
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.timing()                     # reset accumulators
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
    evs[0].record()
    for k in range(a.steps):
        step()
        evs[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = evs[0].elapsed_time(evs[-1])
    per_step = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(a.steps)])
    tim = plan.timing()
    plan.set_timing(False)
    ms_per_step = gpu_ms / a.steps
    value = n * a.steps / (gpu_ms / 1e3)

    nl = rn.build_neighbors(ctx, s, m.r_c, w["skin"], w["decomp"]).info()
    n_local_pairs = nl["n_local_pairs"]
    # in-cutoff directed edges of the locals: the list without skin
    n_in_cutoff = rn.build_neighbors(ctx, s, m.r_c, 0.0, w["decomp"]).info()["n_local_pairs"]
    wk = work_model(w, n_local_pairs, n_in_cutoff, a.precision)

    steps_t = max(1, tim["steps"])
    ms = {k: v / steps_t for k, v in tim["ms"].items()}
    la = tim["launches"]
    roof = roofline(wk, tim, T, a.precision, a.workload)
    kernels = [kernel_entry(wk, tim, T, a.precision, p) for p in ("edge_fwd", "adj_centre", "adj_gather", "nn_fwd",
                                                                   "nn_bwd") if la.get(p, 0) > 0]

    # neighbour-list build on its own (the C-ABI build of the same list), median of three
    tb = []
    for _ in range(3):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rn.build_neighbors(ctx, s, m.r_c, w["skin"], w["decomp"])
        torch.cuda.synchronize()
        tb.append((time.perf_counter() - t1) * 1e3)
    nlist_ms = float(np.median(tb))
    # the plan's own rebuild (its buffers kept): the caller-kept list policy, and a rigid shift
    # of the whole system by 0.6 of the skin and back, so that each update rebuilds
    plan.set_list_policy(False)
    shift = torch.zeros_like(pos)
    shift[:, 0] = 0.6 * w["skin"]
    tr = []
    for k in range(4):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rebuilt = plan.update_list(pos + shift if k % 2 == 0 else pos)
        tr.append((time.perf_counter() - t1) * 1e3)
        assert rebuilt
    plan.set_list_policy(True)
    rebuild_ms = float(np.median(tr))

    # the host-pointer entry point on the same system: positions in and forces / virial out
    # over PCIe each call (reported beside the device-resident rate, never as `value`)
    nh = max(1, min(5, a.steps))
    rn.energy_forces(ctx, model, s, T=T, precision=a.precision, decomp=w["decomp"], skin=w["skin"])
    torch.cuda.synchronize()
    th = time.perf_counter()
    for _ in range(nh):
        rn.energy_forces(ctx, model, s, T=T, precision=a.precision, decomp=w["decomp"], skin=w["skin"])
    host_ms = (time.perf_counter() - th) / nh * 1e3

    out = dict(metric=METRIC, value=round(value, 1), unit="atom-steps/s", n_gpus=1, steps=a.steps,
               warmup=a.warmup, ms_per_step=round(ms_per_step, 4), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype={"fp64": "f64", "fp32": "f32", "bf16": "bf16", "fp8": "fp8"}[a.precision],
               data="synthetic",
               config=dict(workload=describe(a.workload, w), precision=a.precision, n_atoms=n,
                           ghosts=nl["n_ghosts"], list_pairs=n_local_pairs, in_cutoff_edges=n_in_cutoff,
                           first_step_s=round(t_build, 3), wall_s=round(wall, 3)),
               step_ms=dict(median=round(float(np.median(per_step)), 4),
                            iqr=round(float(np.percentile(per_step, 75) - np.percentile(per_step, 25)), 4)),
               nlist_build_ms=round(nlist_ms, 3), nlist_rebuild_ms=round(rebuild_ms, 3),
               phase_ms_per_step={k: round(v, 4) for k, v in ms.items()},
               host_pointer_path=dict(ms_per_call=round(host_ms, 3), atom_steps_per_s=round(n / (host_ms * 1e-3), 1),
                                      note="reann_energy_forces with host buffers: PCIe copies included"),
               roofline=roof, kernels=kernels)
    if not a.no_extra and a.workload == "cu100800":
        print("bench: precision ladder", file=sys.stderr, flush=True)
        out["precision_ladder"] = precision_ladder(rn, torch, ctx, w, a.workload)
        print("bench: decomposed water", file=sys.stderr, flush=True)
        out["decomposed_water"] = decomposed_water(rn, torch, ctx)
        print("bench: halo ablation", file=sys.stderr, flush=True)
        out["halo_ablation"] = halo_ablation(rn, torch, ctx, out["decomposed_water"]["tsweep"]["rows"])
        print("bench: node-feature exchange", file=sys.stderr, flush=True)
        out["node_feature_exchange"] = node_feature_exchange(rn, torch, ctx, w, a.workload)
        print("bench: message forms", file=sys.stderr, flush=True)
        out["message_forms"] = message_forms(rn, torch, ctx, w, a.workload, ms_per_step if a.precision == "fp32"
                                             else float("nan"))
    if not a.no_serve:
        print("bench: MD-amortised run", file=sys.stderr, flush=True)
        out["md_amortised"] = md_amortised(rn, w, a.precision)
        print("bench: serving", file=sys.stderr, flush=True)
        out["serve"] = serve_bench(rn, seconds=a.serve_seconds)
    if not a.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.workload, T)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
