"""Pins of the oracle's second message form (the radial form: L = 0, the orbital sums
themselves as features, residual message updates; the generality paragraph of Sec. 2.2).

The routes are independent of the oracle's code: a brute-force evaluation of the form's
definition over all pairs of a small open cluster with library (torch) layers for the atomic
networks, central differences of the energy, symmetries, and the equality of the
subdomain-decomposed evaluation with the whole-system one.
"""
import numpy as np
import pytest

from synth import models, systems

pytestmark = pytest.mark.filterwarnings("ignore")


def _cluster(n, seed, spacing=1.5, box=7.0, n_species=2):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        p = rng.uniform(0, box, 3)
        if all(np.linalg.norm(p - q) > spacing for q in pts):
            pts.append(p)
    return dict(pos=np.array(pts), species=rng.integers(0, n_species, n).astype(np.int32),
                cell=np.diag([box, box, box]), pbc=np.zeros(3, np.int32))


def _mlp(params, x):
    import torch
    layers = []
    for k, (W, b) in enumerate(params):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W)); lin.bias.copy_(torch.from_numpy(b))
        layers.append(lin)
        if k < len(params) - 1:
            layers.append(torch.nn.SiLU())
    with torch.no_grad():
        return torch.nn.Sequential(*layers)(torch.from_numpy(np.ascontiguousarray(x))).numpy()


def _brute_radial(m, s, T):
    """The radial form by its definition, every pair of an open cluster."""
    x = s["pos"]; spec = s["species"]; n = len(x)
    d = x[None, :, :] - x[:, None, :]                     # d[i, j] = x_j - x_i
    r = np.linalg.norm(d, axis=-1)
    inside = (r < m.r_c) & ~np.eye(n, dtype=bool)
    fc = np.where(inside, (0.5 * np.cos(np.pi * r / m.r_c) + 0.5) ** 2, 0.0)
    R = np.exp(-m.alphas[None, None, :] * (r[:, :, None] - m.centres[None, None, :]) ** 2)
    filt = R * fc[:, :, None]                             # [i, j, K]
    dims_m = models.mlp_dims(m.K, m.hidden, m.n_hidden, m.K)
    dims_e = models.mlp_dims(m.K, m.hidden, m.n_hidden, 1)
    c = m.c0[spec].copy()
    for t in range(T):
        feat = np.einsum("ijk,jk->ik", filt, c)
        if t == T - 1:
            break
        upd = np.zeros_like(c)
        for sp in range(m.n_species):
            sel = spec == sp
            if sel.any():
                upd[sel] = _mlp(models.unpack_mlp(m.msg_blob, dims_m, t * m.n_species + sp), feat[sel])
        c = c + upd
    e = np.zeros(n)
    for sp in range(m.n_species):
        sel = spec == sp
        if sel.any():
            e[sel] = _mlp(models.unpack_mlp(m.energy_blob, dims_e, sp), feat[sel])[:, 0] * m.energy_scale
    return e


@pytest.mark.parametrize("T", [1, 2, 3])
def test_radial_brute_force_cluster(oracle_lib, T):
    s = _cluster(9, seed=40 + T)
    m = models.water_model_radial(T_max=3, seed=T, energy_scale=1.3)
    out = oracle_lib.evaluate(m, s, T=T, forces=False)
    want = _brute_radial(m, s, T)
    np.testing.assert_allclose(out["atom_energy"], want, rtol=1e-12, atol=1e-12)
    assert abs(out["energy"] - want.sum()) <= 1e-11 * max(1.0, abs(want.sum()))


def test_radial_features_are_the_lambda0_sums(oracle_lib):
    """The features of the radial form are the orbital sums of lambda = 0 (no squaring):
    doubling every layer-0 message doubles S at layer 0."""
    s = _cluster(8, seed=3)
    m = models.water_model_radial(T_max=2, seed=5)
    S1 = oracle_lib.evaluate(m, s, T=1, forces=False, want_S=True)["S"][0]
    m2 = models.water_model_radial(T_max=2, seed=5)
    m2.c0 = 2.0 * m2.c0
    S2 = oracle_lib.evaluate(m2, s, T=1, forces=False, want_S=True)["S"][0]
    assert S1.shape[1] == 1
    np.testing.assert_allclose(S2, 2.0 * S1, rtol=1e-14, atol=1e-15)


def _fd(oracle_lib, m, s, T, skin, i, a, h=1e-4):
    p = s["pos"].copy()
    p[i, a] += h; ep = oracle_lib.evaluate(m, dict(s, pos=p), T=T, skin=skin, forces=False)["energy"]
    p[i, a] -= 2 * h; em = oracle_lib.evaluate(m, dict(s, pos=p), T=T, skin=skin, forces=False)["energy"]
    return -(ep - em) / (2 * h)


@pytest.mark.parametrize("case", ["water_T3", "cu_T3_skin", "cluster_T2"])
def test_radial_forces_central_differences(oracle_lib, case):
    if case == "water_T3":
        s = systems.water_box(seed=21); m = models.water_model_radial(T_max=3, seed=21, energy_scale=0.8)
        T, skin = 3, 0.5
    elif case == "cu_T3_skin":
        s = systems.fcc_crystal((3, 3, 3), seed=22); m = models.cu_model_radial(T_max=3, seed=22)
        T, skin = 3, 1.0
    else:
        s = _cluster(10, seed=23); m = models.water_model_radial(T_max=2, seed=23)
        T, skin = 2, 0.0
    F = oracle_lib.evaluate(m, s, T=T, skin=skin)["forces"]
    rng = np.random.default_rng(1)
    checked = 0
    for i in rng.choice(len(s["pos"]), 4, replace=False):
        for a in range(3):
            fd = _fd(oracle_lib, m, s, T, skin, i, a)
            assert F[i, a] == pytest.approx(fd, rel=1e-6, abs=1e-7 * max(1.0, np.abs(F).max()))
            checked += abs(F[i, a]) > 1e-3
    assert checked >= 4


def test_radial_virial_diagonal_strain(oracle_lib):
    """dE/d(eps_aa) = -W_aa for a homogeneous stretch of cell and positions."""
    s = systems.water_box(seed=24); m = models.water_model_radial(T_max=3, seed=24)
    W = oracle_lib.evaluate(m, s, T=3)["virial"]
    h = 1e-5
    for a in range(3):
        def energy(eps):
            st = np.eye(3); st[a, a] += eps
            return oracle_lib.evaluate(m, dict(s, pos=s["pos"] @ st, cell=s["cell"] @ st), T=3,
                                       forces=False)["energy"]
        dE = (energy(h) - energy(-h)) / (2 * h)
        assert -W[a, a] == pytest.approx(dE, rel=1e-6, abs=1e-7)


def test_radial_rotation_invariance(oracle_lib):
    s = _cluster(12, seed=25)
    m = models.water_model_radial(T_max=3, seed=25)
    out = oracle_lib.evaluate(m, s, T=3)
    th = 0.7
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, np.cos(0.4), -np.sin(0.4)], [0, np.sin(0.4), np.cos(0.4)]])
    Q = Rz @ Rx
    centre = s["pos"].mean(0)
    rot = dict(s, pos=(s["pos"] - centre) @ Q.T + centre + 20.0, cell=np.eye(3) * 60)
    out2 = oracle_lib.evaluate(m, rot, T=3)
    assert out2["energy"] == pytest.approx(out["energy"], rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(out2["forces"], out["forces"] @ Q.T, rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("T,decomp", [(2, (2, 1, 1)), (3, (2, 2, 2)), (3, (1, 3, 2))])
def test_radial_decomposed_equals_whole(oracle_lib, T, decomp):
    """The per-layer exchange (ghost messages copied from their owners, message adjoints and
    ghost forces reduced onto them) carries the residual form exactly."""
    s = systems.water_box(seed=26); m = models.water_model_radial(T_max=3, seed=26)
    whole = oracle_lib.evaluate(m, s, T=T, skin=0.3)
    part = oracle_lib.evaluate(m, s, T=T, skin=0.3, decomp=decomp)
    assert part["energy"] == pytest.approx(whole["energy"], rel=1e-13, abs=1e-12)
    np.testing.assert_allclose(part["forces"], whole["forces"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(part["virial"], whole["virial"], rtol=1e-10, atol=1e-11)


def test_radial_naive_decomposition_fails(oracle_lib):
    """Negative control: ghosts' messages recomputed from the subdomain's incomplete
    neighbourhoods change the energy of the radial form too."""
    s = systems.water_box(seed=27); m = models.water_model_radial(T_max=3, seed=27)
    whole = oracle_lib.evaluate(m, s, T=3, forces=False)["energy"]
    naive = oracle_lib.evaluate(m, s, T=3, forces=False, decomp=(2, 2, 2), naive=True)["energy"]
    assert abs(naive - whole) > 1e-6 * max(1.0, abs(whole))


def test_radial_form_needs_L0(oracle_lib):
    m = models.water_model_radial(T_max=2, seed=1)
    m.L = 1
    with pytest.raises(ValueError):
        oracle_lib.evaluate(m, _cluster(4, seed=1), T=1, forces=False)
