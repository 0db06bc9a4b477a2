"""Pins of the oracle's literal reading of Eq. (1) (the "diag" form: only the squares,
rho[l,a] = sum_{|lambda|=l} l!/lambda! S[lambda,a]^2, F = (L+1) K).

Independent routes: the multinomial theorem in closed form for a dimer and as an all-pairs
identity on a periodic box (with the oracle's own layer-1 messages, so the message indexing is
pinned too), library (torch) layers for the atomic networks, central differences, and the
equality of the decomposed and whole-system evaluations."""
import numpy as np
import pytest

from synth import models, systems

pytestmark = pytest.mark.filterwarnings("ignore")


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


def test_diag_dimer_closed_form(oracle_lib):
    """Dimer at distance r: sum_{|lambda|=l} l!/lambda! (s d)^(2 lambda) = (s r)^(2l), so
    rho[l,m] = (c_j[m] R_m(r) f_c(r))^2 (s r)^(2l) for each atom, and E_i is the energy NN of it."""
    m = models.make_model(["H", "O"], L=2, K=6, r_c=4.5, width=0.6, n_hidden=2, hidden=5, T_max=1, seed=8,
                          ang_scale=0.7, bias_std=0.5, energy_scale=1.4, form="diag")
    r = 2.3
    u = np.array([0.48, 0.6, 0.64])
    s = dict(pos=np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0] + r * u]), species=np.array([0, 1], np.int32),
             cell=np.eye(3) * 30.0, pbc=np.zeros(3, np.int32))
    out = oracle_lib.evaluate(m, s, T=1, forces=False)
    fc = (0.5 * np.cos(np.pi * r / m.r_c) + 0.5) ** 2
    R = np.exp(-m.alphas * (r - m.centres) ** 2)
    dims = models.mlp_dims(m.F, m.hidden, m.n_hidden, 1)
    for i, j in ((0, 1), (1, 0)):
        w = m.c0[s["species"][j]] * R * fc
        rho = np.concatenate([w * w * (m.ang_scale * r) ** (2 * l) for l in range(m.L + 1)])
        e = _mlp(models.unpack_mlp(m.energy_blob, dims, s["species"][i]), rho[None, :])[0, 0] * m.energy_scale
        assert out["atom_energy"][i] == pytest.approx(e, rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("layer", [0, 1])
def test_diag_multinomial_identity(oracle_lib, layer):
    """rho_i[l,a] = sum_{j,k} w_j^a w_k^a (s^2 d_ij . d_ik)^l with w_j^a = c_j[a] R_a(r_ij) f_c(r_ij),
    all pairs of the periodic box with the oracle's messages of that layer; the layer's features
    then give the next layer's messages through library layers."""
    s = systems.water_box(seed=12)
    m = models.water_model(T_max=2, seed=12, form="diag")
    out = oracle_lib.evaluate(m, s, T=2, forces=False, want_S=True, want_c=True)
    cmsg = out["c"][layer]
    L = np.diag(s["cell"])
    pos = s["pos"] - np.floor(s["pos"] / L) * L
    shifts = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)])
    dims_m = models.mlp_dims(m.F, m.hidden, m.n_hidden, m.K)
    for i in [0, 17, 101, 190]:
        d = (pos[None, :, :] - pos[i][None, None, :] + (shifts * L)[:, None, :]).reshape(-1, 3)
        jj = np.tile(np.arange(len(pos)), len(shifts))
        rr = np.linalg.norm(d, axis=1)
        keep = (rr < m.r_c) & (rr > 0)
        d, rr, jj = d[keep], rr[keep], jj[keep]
        fc = (0.5 * np.cos(np.pi * rr / m.r_c) + 0.5) ** 2
        w = cmsg[jj] * np.exp(-m.alphas[None, :] * (rr[:, None] - m.centres[None, :]) ** 2) * fc[:, None]
        G = m.ang_scale ** 2 * (d @ d.T)
        rho = np.concatenate([np.einsum("ja,jk,ka->a", w, G ** l, w) for l in range(m.L + 1)])
        if layer == 0:
            c1 = _mlp(models.unpack_mlp(m.msg_blob, dims_m, s["species"][i]), rho[None, :])[0]
            np.testing.assert_allclose(out["c"][1][i], c1, rtol=1e-10, atol=1e-12)
        else:
            dims_e = models.mlp_dims(m.F, m.hidden, m.n_hidden, 1)
            e = _mlp(models.unpack_mlp(m.energy_blob, dims_e, s["species"][i]), rho[None, :])[0, 0] * m.energy_scale
            assert out["atom_energy"][i] == pytest.approx(e, rel=1e-10, abs=1e-12)


def _fd(oracle_lib, m, s, T, skin, i, a, h=1e-4):
    p = s["pos"].copy()
    p[i, a] += h; ep = oracle_lib.evaluate(m, dict(s, pos=p), T=T, skin=skin, forces=False)["energy"]
    p[i, a] -= 2 * h; em = oracle_lib.evaluate(m, dict(s, pos=p), T=T, skin=skin, forces=False)["energy"]
    return -(ep - em) / (2 * h)


def test_diag_forces_central_differences(oracle_lib):
    s = systems.water_box(seed=13)
    m = models.water_model(T_max=3, seed=13, form="diag")
    F = oracle_lib.evaluate(m, s, T=3, skin=0.5)["forces"]
    rng = np.random.default_rng(2)
    checked = 0
    for i in rng.choice(len(s["pos"]), 4, replace=False):
        for a in range(3):
            fd = _fd(oracle_lib, m, s, 3, 0.5, i, a)
            assert F[i, a] == pytest.approx(fd, rel=1e-6, abs=1e-7 * max(1.0, np.abs(F).max()))
            checked += abs(F[i, a]) > 1e-3
    assert checked >= 4


def test_diag_decomposed_equals_whole(oracle_lib):
    s = systems.water_box(seed=14)
    m = models.water_model(T_max=3, seed=14, form="diag")
    whole = oracle_lib.evaluate(m, s, T=3, skin=0.3)
    part = oracle_lib.evaluate(m, s, T=3, skin=0.3, decomp=(2, 2, 2))
    assert part["energy"] == pytest.approx(whole["energy"], rel=1e-13, abs=1e-12)
    np.testing.assert_allclose(part["forces"], whole["forces"], rtol=1e-10, atol=1e-11)
