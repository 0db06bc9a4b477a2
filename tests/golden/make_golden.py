"""Write the oracle's expected values for the full-size workloads.

Calls only ``oracle`` (FP64 CPU) and ``synth`` (seeded inputs).  The GPU parity
tests compare against the stored numbers at sizes where running the oracle in the
test itself would take too long.  Each file records a checksum of the generated
positions so that a change of the generator is caught instead of silently
comparing different systems.

Usage:  python tests/golden/make_golden.py cu100800 [water1207296] [--threads N]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_SAMPLE = 256


def positions_digest(pos: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(pos, dtype=np.float64).tobytes()).hexdigest()


def make(name: str, T: int, threads: int) -> str:
    w = synth.workload(name)
    s, m = w["system"], w["model"]
    n = len(s["pos"])
    t0 = time.time()
    out = oracle.evaluate(m, s, T=T, skin=w["skin"], threads=threads)
    dt = time.time() - t0
    idx = np.sort(np.random.default_rng(12345).choice(n, min(N_SAMPLE, n), replace=False))
    rec = dict(workload=name, T=T, skin=w["skin"], n_atoms=n, positions_sha256=positions_digest(s["pos"]),
               energy=out["energy"], sum_abs_atom_energy=float(np.abs(out["atom_energy"]).sum()),
               virial=out["virial"].ravel().tolist(), force_rms=float(np.sqrt((out["forces"] ** 2).mean())),
               force_sum=out["forces"].sum(0).tolist(),
               sample_index=idx.tolist(), sample_atom_energy=out["atom_energy"][idx].tolist(),
               sample_forces=out["forces"][idx].ravel().tolist(),
               oracle_seconds=dt, oracle_threads=threads)
    path = os.path.join(HERE, "%s_T%d.json" % (name, T))
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    return path


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+")
    ap.add_argument("--T", type=int, nargs="*", default=None)
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    for nm in a.names:
        Ts = a.T or [synth.workload(nm)["T"]]
        for T in Ts:
            print(make(nm, T, a.threads), flush=True)
