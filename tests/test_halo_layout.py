"""Host-side layout of the extended-halo clusters (paper_2505_06711_amd.halo): the locals of the
subdomains partition the atoms, and each cluster holds every periodic copy within T (r_c + skin)
of each of its locals, checked by brute force.  No GPU."""
import itertools

import numpy as np
import pytest

from synth import systems


def test_clusters_cover_every_local_receptive_field():
    from paper_2505_06711_amd.halo import subdomain_clusters
    s = systems.water_box(grid=(5, 5, 5), spacing=systems.WATER_BOX_L / 4, seed=84)
    L = np.diag(s["cell"])
    rcut, T = 5.5, 2
    parts = subdomain_clusters(s, rcut, T, (2, 2, 1))
    locs = np.concatenate([o[:k] for o, _, k in parts])
    assert sorted(locs.tolist()) == list(range(len(s["pos"])))
    w = s["pos"] - np.floor(s["pos"] / L) * L
    R = T * rcut
    for owner, x, nloc in parts:
        keys = {(int(o), *np.round((xx - w[o]) / L).astype(int)) for o, xx in zip(owner, x)}
        assert len(keys) == len(owner)                      # no copy twice
        for i in owner[:nloc][::7]:
            for sh in itertools.product(range(-3, 4), repeat=3):
                d = w + np.array(sh) * L - w[i]
                near = np.nonzero(np.sqrt((d * d).sum(1)) < R)[0]
                for j in near:
                    assert (int(j), *sh) in keys
