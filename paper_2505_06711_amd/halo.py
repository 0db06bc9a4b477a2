"""Extended-halo evaluation: the redundant alternative to the per-layer ghost exchange.

The paper's scheme (Sec. 2.2) keeps a ghost shell of r_c + skin for every T and exchanges the
ghosts' messages once per message-passing layer.  The alternative it argues against (Sec. 2.2,
Fig. 2(a): the receptive field of T layers reaches T r_c) avoids the per-layer exchange by
giving every subdomain all atom copies within T (r_c + skin) of its box and recomputing
their messages inside the subdomain: no communication between layers, one reverse sum of the
copies' forces onto their owners at the end, and redundant work on the halo.

Here each subdomain's extended set is evaluated by the library as one open cluster (its own
plan, every layer over the whole cluster), with the atomic energies of the copies weighted 0
(``reann_plan_set_energy_weights``), so the plan's energy is the subdomain's share and its
backward the gradient of that share.  This module only lays out the clusters (which copies
belong to which subdomain) and sums the clusters' results; every evaluation runs in the
library's kernels.
"""
from __future__ import annotations

import numpy as np

from ._binding import Context, Model, Plan


def subdomain_clusters(system: dict, rcut: float, T: int, decomp=(1, 1, 1)):
    """Per subdomain: (owner index [m], positions [m, 3], number of locals).  Locals first (the
    atoms whose wrapped position lies in the subdomain's box), then every other periodic copy
    whose position lies within T rcut + 1e-6 of the box on each periodic axis."""
    pos = np.asarray(system["pos"], dtype=np.float64)
    L = np.diag(np.asarray(system["cell"], dtype=np.float64)).copy()
    per = np.asarray(system["pbc"]) != 0
    P = np.asarray(decomp, dtype=np.int64)
    if np.any(~per & (P != 1)):
        raise ValueError("a non-periodic axis cannot be split")
    w = pos.copy()
    for a in range(3):
        if per[a]:
            q = np.floor(pos[:, a] / L[a])
            w[:, a] = pos[:, a] - q * L[a]
            w[:, a] = np.where(w[:, a] < 0, w[:, a] + L[a], w[:, a])
            w[:, a] = np.where(w[:, a] >= L[a], w[:, a] - L[a], w[:, a])
    h = np.where(per, L / P, np.inf)
    cidx = np.where(per[None, :], np.minimum((w / h[None, :]).astype(np.int64), P[None, :] - 1), 0)
    dom = (cidx[:, 0] * P[1] + cidx[:, 1]) * P[2] + cidx[:, 2]
    shell = T * rcut + 1e-6
    nm = [int(np.floor(shell / L[a])) + 1 if per[a] else 0 for a in range(3)]
    shifts = np.array([(i, j, k) for i in range(-nm[0], nm[0] + 1) for j in range(-nm[1], nm[1] + 1)
                       for k in range(-nm[2], nm[2] + 1)], dtype=np.int64)
    out = []
    for p in range(int(P.prod())):
        pc = np.array([p // (P[1] * P[2]), (p // P[2]) % P[1], p % P[2]])
        lo = np.where(per, pc * h, -np.inf)
        hi = np.where(per, np.where(pc == P - 1, L, (pc + 1) * h), np.inf)
        loc = np.nonzero(dom == p)[0]
        own, xs = [loc], [w[loc]]
        for s in shifts:
            y = w + s[None, :] * np.where(per, L, 0.0)[None, :]
            inside = np.all(~per[None, :] | ((y >= lo - shell) & (y < hi + shell)), axis=1)
            if not s.any():
                inside &= dom != p
            sel = np.nonzero(inside)[0]
            own.append(sel)
            xs.append(y[sel])
        out.append((np.concatenate(own), np.concatenate(xs), len(loc)))
    return out


class HaloEvaluator:
    """E, F, W of `system` by the extended-halo scheme on the GPU: one open-cluster plan per
    subdomain at fixed cluster membership (the clusters follow the positions given here)."""

    def __init__(self, ctx: Context, model: Model, params, system: dict, T: int, precision="fp64",
                 decomp=(1, 1, 1), skin: float = 0.0):
        self.n = len(system["pos"])
        self.T = T
        rcut = params.r_c + skin
        self.parts = []
        spec = np.asarray(system["species"], dtype=np.int32)
        for owner, x, nloc in subdomain_clusters(system, rcut, T, decomp):
            # an open cluster: the box only has to be valid, the non-periodic axes ignore it
            span = np.ptp(x, axis=0) + 2 * rcut + 1.0
            cl = dict(pos=x, species=spec[owner], cell=np.diag(span), pbc=np.zeros(3, np.int32))
            plan = Plan(ctx, model, cl, T=T, precision=precision, skin=skin)
            wts = np.zeros(len(owner))
            wts[:nloc] = 1.0
            plan.set_energy_weights(wts)
            self.parts.append((plan, owner, x, nloc))

    def cluster_atoms(self) -> int:
        return int(sum(len(o) for _, o, _, _ in self.parts))

    def device_inputs(self, torch):
        """Device copies of each cluster's positions, and the owner index (device) for the
        reverse sum."""
        self._dev = [(torch.tensor(x, dtype=torch.float64, device="cuda"),
                      torch.tensor(owner, dtype=torch.int64, device="cuda")) for _, owner, x, _ in self.parts]
        self._E = torch.zeros(len(self.parts), dtype=torch.float64, device="cuda")
        self._W = torch.zeros((len(self.parts), 3, 3), dtype=torch.float64, device="cuda")
        self._F = [torch.zeros((len(owner), 3), dtype=torch.float64, device="cuda") for _, owner, _, _ in self.parts]
        self._Fsum = torch.zeros((self.n, 3), dtype=torch.float64, device="cuda")

    def step(self, torch):
        """One energy + force + virial evaluation, all on the device: every subdomain's plan,
        then the copies' forces summed onto their owners.  Returns device tensors (E, F, W)."""
        for k, (plan, _, _, _) in enumerate(self.parts):
            xd, _ = self._dev[k]
            plan.forward(xd, self._E[k])
            plan.backward(self._F[k], virial=self._W[k])
        self._Fsum.zero_()
        for k in range(len(self.parts)):
            self._Fsum.index_add_(0, self._dev[k][1], self._F[k])
        return self._E.sum(), self._Fsum, self._W.sum(0)
