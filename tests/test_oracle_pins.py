"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here re-calls the oracle's own formula to check itself.  Each test is a
different route to the same number (brute force, closed forms at special points,
the multinomial identity, library MLP layers, finite differences) or an
invariant (symmetries, locality after T layers, decomposition equivalence).
"""
import math

import numpy as np
import pytest

from synth import models, systems

pytestmark = pytest.mark.filterwarnings("ignore")


# ----------------------------------------------------------------- helpers --

def lambdas(L):
    """Cartesian components in the oracle's documented order: l, lx desc, ly desc."""
    out = []
    for l in range(L + 1):
        for lx in range(l, -1, -1):
            for ly in range(l - lx, -1, -1):
                out.append((lx, ly, l - lx - ly))
    return out


def wrap(x, L):
    q = np.floor(x / L)
    w = x - q * L
    w = np.where(w < 0, w + L, w)
    return np.where(w >= L, w - L, w)


def brute_pairs(system, rcut):
    """Every (i, j, shift) with |x_j + shift*L - x_i| < rcut, (j,shift) != (i,0),
    by exhaustive enumeration over all atoms and lattice shifts."""
    pos = system["pos"]; L = np.diag(system["cell"]); pbc = system["pbc"]
    w = np.where(pbc.astype(bool), wrap(pos, np.where(L > 0, L, 1.0)), pos)
    nmax = [int(math.floor((rcut + 1e-6) / L[a])) + 1 if pbc[a] else 0 for a in range(3)]
    shifts = np.array([(a, b, c) for a in range(-nmax[0], nmax[0] + 1)
                       for b in range(-nmax[1], nmax[1] + 1) for c in range(-nmax[2], nmax[2] + 1)])
    out, near = set(), 0
    for i in range(len(pos)):
        d = (w[None, :, :] + (shifts * L)[:, None, :]) - w[i]
        d2 = (d * d).sum(-1)
        near += int(np.sum(np.abs(np.sqrt(d2) - rcut) < 1e-9))
        for si, j in zip(*np.nonzero(d2 < rcut * rcut)):
            if j == i and not shifts[si].any():
                continue
            out.add((i, int(j), *map(int, shifts[si])))
    assert near == 0, "a pair sits within 1e-9 A of the cutoff: the witness cannot decide it"
    return out


def oracle_pairs(oracle, system, rcut, decomp=(1, 1, 1)):
    row, j, sh = oracle.neighbors(system, rcut, decomp)
    out = set()
    for i in range(len(row) - 1):
        for k in range(row[i], row[i + 1]):
            out.add((i, int(j[k]), *map(int, sh[k])))
    return out, (row, j, sh)


def open_cluster(n, seed, spacing=1.6, box=8.0):
    """Random atoms in a cube with a minimum separation, no periodicity."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        p = rng.uniform(0, box, 3)
        if all(np.linalg.norm(p - q) > spacing for q in pts):
            pts.append(p)
    return dict(pos=np.array(pts), species=rng.integers(0, 2, n).astype(np.int32),
                cell=np.diag([box, box, box]), pbc=np.zeros(3, np.int32), elements=["H", "O"])


def small_water(seed=0, T_max=3):
    return systems.water_box(seed=seed), models.water_model(T_max=T_max, seed=seed)


def small_cu(seed=0, cells=(3, 3, 3), T_max=3):
    return systems.fcc_crystal(cells, seed=seed), models.cu_model(T_max=T_max, seed=seed)


def rho_from_S(S, L, K):
    """Density features from orbital sums with the multinomial weights (Eq. (1))."""
    lam = lambdas(L)
    out = []
    for l in range(L + 1):
        for a in range(K):
            for b in range(a, K):
                s = 0.0
                for k, (lx, ly, lz) in enumerate(lam):
                    if lx + ly + lz == l:
                        wgt = math.factorial(l) / (math.factorial(lx) * math.factorial(ly) * math.factorial(lz))
                        s += wgt * S[..., k, a] * S[..., k, b]
                out.append(s)
    return np.stack(out, axis=-1)


# ------------------------------------------------------------- neighbours --

@pytest.mark.parametrize("case", ["water", "tiny_box", "slab", "cluster", "skinned_cu"])
def test_neighbors_match_brute_force(oracle_lib, case):
    if case == "water":
        s, rcut = systems.water_box(seed=1), 5.0
    elif case == "tiny_box":      # box edge < 2 * rcut: several images of the same atom
        rng = np.random.default_rng(2)
        s = dict(pos=rng.uniform(-1, 5, (7, 3)), species=np.zeros(7, np.int32),
                 cell=np.diag([4.0, 3.3, 5.1]), pbc=np.ones(3, np.int32), elements=["Cu"])
        rcut = 3.7
    elif case == "slab":
        s = systems.water_box(seed=3); s = dict(s, pbc=np.array([1, 1, 0], np.int32)); rcut = 4.5
    elif case == "cluster":
        s, rcut = open_cluster(30, 4), 4.0
    else:
        s, rcut = systems.fcc_crystal((2, 3, 2), seed=5), 7.0
    got, (row, j, sh) = oracle_pairs(oracle_lib, s, rcut)
    assert got == brute_pairs(s, rcut)
    for i in range(len(row) - 1):      # canonical row order (owner, shift)
        keys = [(int(j[k]), *map(int, sh[k])) for k in range(row[i], row[i + 1])]
        assert keys == sorted(keys)


@pytest.mark.parametrize("decomp", [(2, 1, 1), (2, 2, 2), (3, 2, 1), (1, 1, 4)])
def test_neighbors_independent_of_decomposition(oracle_lib, decomp):
    s = systems.water_box(seed=6)
    a = oracle_lib.neighbors(s, 6.0)
    b = oracle_lib.neighbors(s, 6.0, decomp)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


# ------------------------------------------------------- closed forms --

def test_dimer_special_points(oracle_lib):
    """Dimer at r = r_c/2 with a Gaussian centred exactly there: f_c = 1/4, R = 1,
    so S[lambda, m*] = c_j[m*] * A_lambda(d) / 4 with A the scaled monomials."""
    rc = 4.0
    m = models.make_model(["H", "O"], L=2, K=5, r_c=rc, width=0.4, n_hidden=1, hidden=3, T_max=1,
                          seed=3, ang_scale=0.7)
    mstar = 2
    assert m.centres[mstar] == 2.0
    u = np.array([0.36, -0.48, 0.8])          # unit vector
    d = 2.0 * u
    s = dict(pos=np.array([[0.0, 0.0, 0.0], d]), species=np.array([0, 1], np.int32),
             cell=np.eye(3) * 20, pbc=np.zeros(3, np.int32), elements=["H", "O"])
    S = oracle_lib.evaluate(m, s, T=1, forces=False, want_S=True)["S"][0]
    c1 = m.c0[1][mstar]
    sd = 0.7 * d
    for k, (lx, ly, lz) in enumerate(lambdas(2)):
        want = c1 * sd[0] ** lx * sd[1] ** ly * sd[2] ** lz / 4.0
        assert S[0, k, mstar] == pytest.approx(want, rel=1e-13, abs=1e-15)
    # the other atom sees -d: odd l flips sign
    c0 = m.c0[0][mstar]
    for k, (lx, ly, lz) in enumerate(lambdas(2)):
        want = c0 * (-sd[0]) ** lx * (-sd[1]) ** ly * (-sd[2]) ** lz / 4.0
        assert S[1, k, mstar] == pytest.approx(want, rel=1e-13, abs=1e-15)


def test_cutoff_is_smooth_at_rc(oracle_lib):
    """A partner crossing r_c changes neither E nor F discontinuously, and just
    outside r_c the dimer energy is the sum of two isolated atoms (f_c and f_c'
    vanish at r_c)."""
    m = models.water_model(T_max=2, seed=7)
    def dimer(r):
        return dict(pos=np.array([[0.0, 0, 0], [r, 0, 0]]), species=np.array([1, 0], np.int32),
                    cell=np.eye(3) * 30, pbc=np.zeros(3, np.int32), elements=["H", "O"])
    def single(sp):
        return dict(pos=np.zeros((1, 3)), species=np.array([sp], np.int32), cell=np.eye(3) * 30,
                    pbc=np.zeros(3, np.int32), elements=["H", "O"])
    e_iso = sum(oracle_lib.evaluate(m, single(sp), T=2, forces=False)["energy"] for sp in (1, 0))
    inner = oracle_lib.evaluate(m, dimer(m.r_c - 1e-5), T=2)
    outer = oracle_lib.evaluate(m, dimer(m.r_c + 1e-5), T=2)
    assert outer["energy"] == pytest.approx(e_iso, abs=1e-14)
    assert inner["energy"] == pytest.approx(e_iso, abs=1e-12)
    assert np.abs(inner["forces"]).max() < 1e-12
    mid = oracle_lib.evaluate(m, dimer(0.5 * m.r_c), T=2)
    assert abs(mid["energy"] - e_iso) > 1e-3       # the pair does interact inside r_c


@pytest.mark.parametrize("layer", [0, 1])
def test_three_body_identity(oracle_lib, layer):
    """sum_{|lambda|=l} l!/lambda! S[lambda,a] S[lambda,b] = sum_{j,k} w_j^a w_k^b (s^2 d_ij.d_ik)^l
    (multinomial theorem), with w_j^a = c_j[a] R_a(r_ij) f_c(r_ij); layer 1 uses the
    oracle's messages c^1, so the message indexing (c of the neighbour j) is pinned too."""
    s, m = small_water(seed=8, T_max=2)
    out = oracle_lib.evaluate(m, s, T=2, forces=False, want_S=True, want_c=True)
    S, cmsg = out["S"][layer], out["c"][layer]
    rho = rho_from_S(S, m.L, m.K)
    L = np.diag(s["cell"])
    pos = wrap(s["pos"], L)
    for i in [0, 5, 77, 191]:
        d = pos[None, :, :] - pos[i][None, None, :]
        shifts = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)])
        d = (d + (shifts * L)[:, None, :]).reshape(-1, 3)
        jj = np.tile(np.arange(len(pos)), len(shifts))
        r = np.linalg.norm(d, axis=1)
        keep = (r < m.r_c) & (r > 0)
        d, r, jj = d[keep], r[keep], jj[keep]
        fc = (0.5 * np.cos(np.pi * r / m.r_c) + 0.5) ** 2
        R = np.exp(-m.alphas[None, :] * (r[:, None] - m.centres[None, :]) ** 2)
        w = cmsg[jj] * R * fc[:, None]                        # [n_j, K]
        G = (m.ang_scale ** 2) * (d @ d.T)                    # s^2 d_ij . d_ik
        f = 0
        for l in range(m.L + 1):
            Gl = G ** l
            for a in range(m.K):
                for b in range(a, m.K):
                    want = w[:, a] @ Gl @ w[:, b]
                    assert rho[i, f] == pytest.approx(want, rel=1e-11, abs=1e-13)
                    f += 1


def _torch_mlp(params, x):
    import torch
    layers = []
    for k, (W, b) in enumerate(params):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W)); lin.bias.copy_(torch.from_numpy(b))
        layers.append(lin)
        if k < len(params) - 1:
            layers.append(torch.nn.SiLU())
    net = torch.nn.Sequential(*layers)
    with torch.no_grad():
        return net(torch.from_numpy(x)).numpy()


def test_atomic_networks_match_library_layers(oracle_lib):
    """Message NN (Eq. (2)) and energy NN against torch.nn.Linear + SiLU layers."""
    s, m = small_water(seed=9, T_max=2)
    out = oracle_lib.evaluate(m, s, T=2, forces=False, want_S=True, want_c=True)
    dims_m = models.mlp_dims(m.F, m.hidden, m.n_hidden, m.K)
    dims_e = models.mlp_dims(m.F, m.hidden, m.n_hidden, 1)
    rho0 = rho_from_S(out["S"][0], m.L, m.K)
    rho1 = rho_from_S(out["S"][1], m.L, m.K)
    for sp in range(m.n_species):
        sel = s["species"] == sp
        c1 = _torch_mlp(models.unpack_mlp(m.msg_blob, dims_m, sp), rho0[sel])
        np.testing.assert_allclose(out["c"][1][sel], c1, rtol=1e-12, atol=1e-12)
        e = _torch_mlp(models.unpack_mlp(m.energy_blob, dims_e, sp), rho1[sel])[:, 0] * m.energy_scale
        np.testing.assert_allclose(out["atom_energy"][sel], e, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out["c"][0], m.c0[s["species"]], rtol=0, atol=0)   # c^0 per element


# ---------------------------------------------------------------- calculus --

def _fd_force(oracle_lib, m, s, T, skin, i, a, h=1e-4):
    p = s["pos"].copy()
    p[i, a] += h; ep = oracle_lib.evaluate(m, dict(s, pos=p), T=T, skin=skin, forces=False)["energy"]
    p[i, a] -= 2 * h; em = oracle_lib.evaluate(m, dict(s, pos=p), T=T, skin=skin, forces=False)["energy"]
    return -(ep - em) / (2 * h)


@pytest.mark.parametrize("case", ["water_T2", "water_T3", "cu_T3_skin"])
def test_forces_central_differences(oracle_lib, case):
    if case == "water_T2":
        s, m = small_water(seed=10, T_max=2); T, skin = 2, 0.0
    elif case == "water_T3":     # non-unit energy scale: the backward must carry it
        s = systems.water_box(seed=11); m = models.water_model(T_max=3, seed=11, energy_scale=1.7)
        T, skin = 3, 0.5
    else:
        s, m = small_cu(seed=12); T, skin = 3, 1.0
    out = oracle_lib.evaluate(m, s, T=T, skin=skin)
    F = out["forces"]
    rng = np.random.default_rng(0)
    checked = 0
    for i in rng.choice(len(s["pos"]), 4, replace=False):
        for a in range(3):
            fd = _fd_force(oracle_lib, m, s, T, skin, i, a)
            assert F[i, a] == pytest.approx(fd, rel=1e-6, abs=1e-7 * max(1.0, np.abs(F).max()))
            checked += abs(F[i, a]) > 1e-3
    assert checked >= 4


def test_virial_diagonal_strain_periodic(oracle_lib):
    """dE/d(eps_aa) = -W_aa for a homogeneous stretch of cell and positions."""
    s, m = small_water(seed=13, T_max=2)
    W = oracle_lib.evaluate(m, s, T=2)["virial"]
    h = 1e-6
    for a in range(3):
        es = []
        for sgn in (+1, -1):
            M = np.eye(3); M[a, a] += sgn * h
            s2 = dict(s, pos=s["pos"] @ M.T, cell=s["cell"] @ M.T)
            es.append(oracle_lib.evaluate(m, s2, T=2, forces=False)["energy"])
        assert -(es[0] - es[1]) / (2 * h) == pytest.approx(W[a, a], rel=1e-6, abs=1e-6)


def test_virial_full_strain_cluster(oracle_lib):
    """Open cluster: dE/d(eps_ab) = -W_ba for every a,b, and W = sum_i x_i (x) F_i."""
    s = open_cluster(24, 14)
    m = models.water_model(T_max=3, seed=14)
    out = oracle_lib.evaluate(m, s, T=3)
    W, F = out["virial"], out["forces"]
    np.testing.assert_allclose(W, s["pos"].T @ F, rtol=1e-10, atol=1e-10)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            es = []
            for sgn in (+1, -1):
                M = np.eye(3); M[a, b] += sgn * h
                es.append(oracle_lib.evaluate(m, dict(s, pos=s["pos"] @ M.T), T=3, forces=False)["energy"])
            assert -(es[0] - es[1]) / (2 * h) == pytest.approx(W[b, a], rel=1e-6, abs=1e-6)


# -------------------------------------------------------------- symmetries --

def test_rotation_invariance_cluster(oracle_lib):
    s = open_cluster(20, 15)
    m = models.water_model(T_max=3, seed=15)
    a = oracle_lib.evaluate(m, s, T=3)
    th = 0.7
    Q = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    Q = Q @ np.array([[1, 0, 0], [0, math.cos(1.1), -math.sin(1.1)], [0, math.sin(1.1), math.cos(1.1)]])
    b = oracle_lib.evaluate(m, dict(s, pos=s["pos"] @ Q.T + 3.0), T=3)
    assert b["energy"] == pytest.approx(a["energy"], rel=1e-12)
    np.testing.assert_allclose(b["forces"], a["forces"] @ Q.T, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(b["virial"], Q @ a["virial"] @ Q.T, rtol=1e-9, atol=1e-9)
    # torque-free and force-free
    assert np.abs(a["forces"].sum(0)).max() < 1e-10
    assert np.abs(np.cross(s["pos"], a["forces"]).sum(0)).max() < 1e-9


def test_translation_and_permutation_periodic(oracle_lib):
    s, m = small_water(seed=16, T_max=3)
    a = oracle_lib.evaluate(m, s, T=3, skin=0.3)
    assert np.abs(a["forces"].sum(0)).max() < 1e-10
    b = oracle_lib.evaluate(m, dict(s, pos=s["pos"] + np.array([3.3, -7.1, 20.2])), T=3, skin=0.3)
    assert b["energy"] == pytest.approx(a["energy"], rel=1e-12)
    np.testing.assert_allclose(b["forces"], a["forces"], rtol=1e-9, atol=1e-10)
    perm = np.random.default_rng(1).permutation(len(s["pos"]))
    c = oracle_lib.evaluate(m, dict(s, pos=s["pos"][perm], species=s["species"][perm]), T=3, skin=0.3)
    assert c["energy"] == pytest.approx(a["energy"], rel=1e-12)
    np.testing.assert_allclose(c["forces"], a["forces"][perm], rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(c["atom_energy"], a["atom_energy"][perm], rtol=1e-11, atol=1e-12)


def test_cubic_axis_permutation(oracle_lib):
    s, m = small_water(seed=17, T_max=2)
    a = oracle_lib.evaluate(m, s, T=2)
    P = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], float)
    b = oracle_lib.evaluate(m, dict(s, pos=s["pos"] @ P.T), T=2)
    assert b["energy"] == pytest.approx(a["energy"], rel=1e-12)
    np.testing.assert_allclose(b["forces"], a["forces"] @ P.T, rtol=1e-9, atol=1e-10)


# ---------------------------------------------------- message-passing depth --

@pytest.mark.parametrize("T", [1, 2, 3])
def test_receptive_field_is_T_hops(oracle_lib, T):
    """On a chain whose atoms only see their direct neighbours, E_0 depends on atoms
    0..T and on nothing farther (T layers = T hops; T = 1 is the local EANN model)."""
    m = models.water_model(T_max=3, seed=18)
    n = 7
    base = np.zeros((n, 3)); base[:, 0] = np.arange(n) * 0.6 * m.r_c
    base[:, 1] = 0.1 * np.sin(np.arange(n))
    s = dict(pos=base, species=(np.arange(n) % 2).astype(np.int32), cell=np.eye(3) * 100,
             pbc=np.zeros(3, np.int32), elements=["H", "O"])
    e0 = oracle_lib.evaluate(m, s, T=T, forces=False)["atom_energy"][0]
    for k in range(1, n):
        p = base.copy(); p[k, 1] += 0.3
        ek = oracle_lib.evaluate(m, dict(s, pos=p), T=T, forces=False)["atom_energy"][0]
        if k <= T:
            assert ek != e0, k
        else:
            assert ek == e0, k


# -------------------------------------------------- spatial decomposition --

@pytest.mark.parametrize("T", [1, 2, 3, 6])
@pytest.mark.parametrize("decomp", [(2, 1, 1), (2, 2, 2), (3, 2, 1), (1, 1, 3)])
def test_decomposed_equals_whole(oracle_lib, T, decomp):
    """Subdomains that copy ghost messages from their owners every layer and reduce
    ghost adjoints and forces back reproduce the whole-system result (Sec. 2.2)."""
    s = systems.water_box(seed=19)
    m = models.water_model(T_max=6, seed=19)
    skin = 0.5
    a = oracle_lib.evaluate(m, s, T=T, skin=skin)
    b = oracle_lib.evaluate(m, s, T=T, skin=skin, decomp=decomp)
    assert b["energy"] == pytest.approx(a["energy"], rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(b["atom_energy"], a["atom_energy"], rtol=1e-11, atol=1e-12)
    fmax = np.abs(a["forces"]).max()
    assert np.abs(b["forces"] - a["forces"]).max() <= 1e-10 * fmax
    assert np.abs(b["virial"] - a["virial"]).max() <= 1e-10 * np.abs(a["virial"]).max()


def test_decomposed_equals_whole_cu(oracle_lib):
    s, m = small_cu(seed=20, cells=(4, 4, 4))
    a = oracle_lib.evaluate(m, s, T=3, skin=1.0)
    b = oracle_lib.evaluate(m, s, T=3, skin=1.0, decomp=(2, 2, 2))
    assert b["energy"] == pytest.approx(a["energy"], rel=1e-12)
    assert np.abs(b["forces"] - a["forces"]).max() <= 1e-10 * np.abs(a["forces"]).max()


@pytest.mark.parametrize("T", [1, 2, 3])
def test_naive_decomposition_negative_control(oracle_lib, T):
    """Without the per-layer ghost exchange (ghost messages computed from a subdomain's
    incomplete neighbourhood) the energy is wrong for T >= 2 and right for T = 1."""
    s = systems.water_box(seed=21)
    m = models.water_model(T_max=3, seed=21)
    whole = oracle_lib.evaluate(m, s, T=T, forces=False)["energy"]
    naive = oracle_lib.evaluate(m, s, T=T, forces=False, decomp=(2, 2, 2), naive=True)["energy"]
    if T == 1:
        assert naive == pytest.approx(whole, rel=1e-12)
    else:
        assert abs(naive - whole) > 1e-6 * abs(whole)


def test_skin_does_not_change_results(oracle_lib):
    s, m = small_water(seed=22, T_max=3)
    a = oracle_lib.evaluate(m, s, T=3, skin=0.0)
    b = oracle_lib.evaluate(m, s, T=3, skin=1.5)
    assert b["energy"] == pytest.approx(a["energy"], rel=1e-13)
    np.testing.assert_allclose(b["forces"], a["forces"], rtol=1e-10, atol=1e-12)


def test_invalid_arguments(oracle_lib):
    s, m = small_water(seed=23, T_max=2)
    with pytest.raises(ValueError):
        oracle_lib.evaluate(m, dict(s, species=s["species"] + 5), T=2)
    with pytest.raises(ValueError):
        oracle_lib.evaluate(m, s, T=3)
    with pytest.raises(ValueError):
        oracle_lib.evaluate(m, dict(s, pbc=np.array([0, 1, 1], np.int32)), T=2, decomp=(2, 1, 1))
    with pytest.raises(ValueError):
        cell = s["cell"].copy(); cell[0, 1] = 0.5
        oracle_lib.evaluate(m, dict(s, cell=cell), T=2)


# ---- the extended-halo scheme (Sec. 2.2, Fig. 2(a)): no exchange between layers, a T (r_c +
# skin) halo recomputed in every subdomain.  It must give the whole-system result, and its work
# counts show the redundancy the per-layer exchange avoids.

@pytest.mark.parametrize("T", [1, 2, 3])
@pytest.mark.parametrize("decomp", [(1, 1, 1), (2, 2, 2), (3, 2, 1)])
def test_halo_scheme_equals_whole(oracle_lib, T, decomp):
    s = systems.water_box(seed=30)
    m = models.water_model(T_max=3, seed=30)
    ref = oracle_lib.evaluate(m, s, T=T, skin=0.5)
    h = oracle_lib.evaluate_halo(m, s, T=T, skin=0.5, decomp=decomp)
    assert abs(h["energy"] - ref["energy"]) <= 1e-12 * np.abs(ref["atom_energy"]).sum()
    np.testing.assert_allclose(h["atom_energy"], ref["atom_energy"], rtol=0, atol=1e-12 * np.abs(ref["atom_energy"]).max())
    assert np.abs(h["forces"] - ref["forces"]).max() <= 1e-10 * np.abs(ref["forces"]).max()
    assert np.abs(h["virial"] - ref["virial"]).max() <= 1e-10 * np.abs(ref["virial"]).max()


def test_halo_scheme_work_counts(oracle_lib):
    """At T = 1 the halo scheme evaluates exactly the locals and their in-cutoff edges, like the
    per-layer exchange; for T > 1 its layer t evaluates more rows the earlier the layer (the
    halo shrinks by one cutoff per layer), its last layer only the locals, and in total more
    than the T n rows of the exchange."""
    s = systems.water_box(grid=(6, 6, 6), spacing=systems.WATER_BOX_L / 4, seed=83)
    m = models.water_model(T_max=4, seed=83)
    n = len(s["pos"])
    row, _, _ = oracle_lib.neighbors(s, m.r_c)
    n_edges = int(row[-1])
    for T in (1, 2, 3):
        w = oracle_lib.evaluate_halo(m, s, T=T, skin=0.0, decomp=(2, 2, 2), forces=False)["work"]
        assert w[-1, 0] == n and w[-1, 1] == n_edges
        if T == 1:
            continue
        assert all(w[t, 0] > w[t + 1, 0] for t in range(T - 1))
        assert w[:, 0].sum() > T * n and w[:, 1].sum() > T * n_edges
