"""Seeded synthetic REANN model parameters.

No trained weights from the paper exist here, so every model is drawn at random
from a seed.  This module only draws numbers and lays them out in the flat
parameter format that both sides parse on their own; it computes nothing of the
model itself.

Hyper-parameters (Sec. 2.1, Eq. (1)-(2)):
    L          maximum angular order of the Cartesian orbitals
    K          number of primitive Gaussians N_phi (radial channels)
    r_c        cutoff radius in Angstrom
    centres    [K]   Gaussian centres r_m (Angstrom)
    alphas     [K]   Gaussian exponents alpha_m (1/Angstrom^2); a width w maps
                     to alpha = 1/(2 w^2) (the width is read as a standard deviation)
    c0         [n_species, K]  layer-0 orbital coefficients per element
    n_hidden, hidden           hidden layers and their width in every atomic NN
    T_max      number of message-passing layers the parameter set supports; it
               holds T_max - 1 message NNs per element and one energy NN per element
    ang_scale  factor applied to the displacement in the angular part
    energy_scale factor applied to the energy NN output

Message forms: "reann" (Eqs. (1)-(2): paired density features), "diag" (the literal reading of
Eq. (1): only the squares, F = (L+1) K) and "radial" (a second, invariant form on the same
exchange: L = 0, the K orbital sums are the features, and messages are updated with a
residual c^{t+1} = c^t + M(x^t)); F = K for "radial".

Flat parameter layout (float64), shared as a data format only:
    one atomic NN with dims [d0, d1, ..., dn] is, for k = 1..n, the row-major
    weight W_k [d_k, d_{k-1}] followed by the bias b_k [d_k];
    msg blob    = NN(t, s) for t in 0..T_max-2, s in 0..n_species-1, dims [F, H.., K]
    energy blob = NN(s) for s in 0..n_species-1, dims [F, H.., 1]
with F = (L+1) K (K+1) / 2 the number of density features.

Draw order from ``numpy.random.default_rng(seed)``: c0 (row-major), then every
message NN weight/bias in blob order, then every energy NN in blob order.
Weights are N(0, 1/fan_in) except the first layer of every NN, which is
N(0, w1_scale^2/fan_in); biases are N(0, bias_std^2) (0 by default).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def n_features(L: int, K: int, form: str = "reann") -> int:
    if form == "radial":
        return K
    if form == "diag":
        return (L + 1) * K
    return (L + 1) * K * (K + 1) // 2


def mlp_dims(F: int, hidden: int, n_hidden: int, out: int) -> list[int]:
    return [F] + [hidden] * n_hidden + [out]


def mlp_param_count(dims: list[int]) -> int:
    return sum(dims[k] * dims[k - 1] + dims[k] for k in range(1, len(dims)))


@dataclass
class ModelParams:
    elements: list
    L: int
    K: int
    r_c: float
    centres: np.ndarray
    alphas: np.ndarray
    c0: np.ndarray
    n_hidden: int
    hidden: int
    T_max: int
    msg_blob: np.ndarray
    energy_blob: np.ndarray
    ang_scale: float = 1.0
    energy_scale: float = 1.0
    meta: dict = field(default_factory=dict)
    form: str = "reann"

    @property
    def n_species(self) -> int:
        return len(self.elements)

    @property
    def F(self) -> int:
        return n_features(self.L, self.K, self.form)


def make_model(elements, L=2, K=8, r_c=5.0, width=0.5, centre_range=None, n_hidden=2,
               hidden=64, T_max=2, seed=0, bias_std=0.0, c0_std=1.0, ang_scale=1.0,
               energy_scale=1.0, w1_scale=1.0, form="reann") -> ModelParams:
    """Draw a model.  Centres are linspace(lo, hi, K) with (lo, hi) = centre_range
    (default (0, r_c)); every exponent is 1/(2 width^2)."""
    rng = np.random.default_rng(seed)
    ns = len(elements)
    if form not in ("reann", "radial", "diag") or (form == "radial" and L != 0):
        raise ValueError("form 'radial' takes L = 0; forms: 'reann', 'radial', 'diag'")
    F = n_features(L, K, form)
    lo, hi = centre_range if centre_range is not None else (0.0, r_c)
    centres = np.linspace(lo, hi, K)
    alphas = np.full(K, 1.0 / (2.0 * width * width))
    c0 = rng.normal(scale=c0_std, size=(ns, K))

    def draw(dims):
        parts = []
        for k in range(1, len(dims)):
            std = (w1_scale if k == 1 else 1.0) / np.sqrt(dims[k - 1])
            W = rng.normal(scale=std, size=(dims[k], dims[k - 1]))
            b = rng.normal(scale=bias_std, size=dims[k]) if bias_std > 0 else np.zeros(dims[k])
            parts += [W.ravel(), b]
        return np.concatenate(parts)

    mdims = mlp_dims(F, hidden, n_hidden, K)
    edims = mlp_dims(F, hidden, n_hidden, 1)
    msg = [draw(mdims) for _t in range(T_max - 1) for _s in range(ns)]
    en = [draw(edims) for _s in range(ns)]
    msg_blob = np.concatenate(msg) if msg else np.zeros(0)
    return ModelParams(elements=list(elements), L=L, K=K, r_c=float(r_c), centres=centres,
                       alphas=alphas, c0=c0, n_hidden=n_hidden, hidden=hidden, T_max=T_max,
                       msg_blob=np.ascontiguousarray(msg_blob, dtype=np.float64),
                       energy_blob=np.ascontiguousarray(np.concatenate(en), dtype=np.float64),
                       ang_scale=float(ang_scale), energy_scale=float(energy_scale),
                       meta=dict(seed=seed, width=width, bias_std=bias_std, w1_scale=w1_scale), form=form)


def unpack_mlp(blob: np.ndarray, dims: list[int], index: int):
    """Return [(W_k, b_k)] of the ``index``-th NN of ``dims`` in ``blob``."""
    n = mlp_param_count(dims)
    seg = blob[index * n:(index + 1) * n]
    out, o = [], 0
    for k in range(1, len(dims)):
        W = seg[o:o + dims[k] * dims[k - 1]].reshape(dims[k], dims[k - 1]); o += W.size
        b = seg[o:o + dims[k]]; o += dims[k]
        out.append((W, b))
    return out


# ---- the model shapes used by the workloads ------------------------------------------
#
# Every preset draws biases N(0, 1), uses ang_scale = 1/r_c (dimensionless angular
# factors) and a first-layer weight scale w1_scale.  With zero biases the quadratic
# density makes message magnitudes either vanish or square from layer to layer; these
# choices keep every layer's messages and sums O(1) up to T = 6, with atomic energies of
# order 0.5 eV and forces of order 1 eV/A, like a trained potential.

def water_model_plain(T_max=2, seed=0) -> ModelParams:
    """The 64-molecule water configuration's model as stated: L=2, 8 Gaussians centred
    uniformly on [0, 5] A, width 0.5 A, r_c = 5 A, two hidden layers of 64 SiLU units, every
    weight N(0, 1/fan_in), zero biases, c0 ~ N(0, 1), raw Cartesian angular factors (A),
    elements (H, O)."""
    return make_model(["H", "O"], L=2, K=8, r_c=5.0, width=0.5, n_hidden=2, hidden=64, T_max=T_max, seed=seed)


def water_model(T_max=2, seed=0, **kw) -> ModelParams:
    """Water model: L=2, 8 Gaussians centred uniformly on [0, 5] A, width 0.5 A,
    r_c = 5 A, two hidden layers of 64 SiLU units, elements (H, O)."""
    kw = {**dict(bias_std=1.0, w1_scale=2.0, ang_scale=1.0 / 5.0), **kw}
    return make_model(["H", "O"], L=2, K=8, r_c=5.0, width=0.5, n_hidden=2, hidden=64,
                      T_max=T_max, seed=seed, **kw)


def cu_model(T_max=3, seed=0, **kw) -> ModelParams:
    """Cu model: L=2, 12 Gaussians centred uniformly on [0, 6] A, width 0.5 A,
    r_c = 6 A, three hidden layers of 128 SiLU units, element (Cu,)."""
    kw = {**dict(bias_std=1.0, w1_scale=1.0, ang_scale=1.0 / 6.0), **kw}
    return make_model(["Cu"], L=2, K=12, r_c=6.0, width=0.5, n_hidden=3, hidden=128,
                      T_max=T_max, seed=seed, **kw)


def serving_model(T_max=3, seed=0, **kw) -> ModelParams:
    """Serving model: L=2, 12 Gaussians on [0, 5] A, width 0.5 A, r_c = 5 A,
    three hidden layers of 128, elements (H, O, Cu)."""
    kw = {**dict(bias_std=1.0, w1_scale=2.0, ang_scale=1.0 / 5.0), **kw}
    return make_model(["H", "O", "Cu"], L=2, K=12, r_c=5.0, width=0.5, n_hidden=3,
                      hidden=128, T_max=T_max, seed=seed, **kw)


def cu_model_radial(T_max=3, seed=0, **kw) -> ModelParams:
    """The Cu model's sizes in the radial message form: L = 0, 12 Gaussians centred uniformly
    on [0, 6] A, width 0.5 A, r_c = 6 A, three hidden layers of 128 SiLU units, F = K = 12
    features, residual message updates, element (Cu,)."""
    kw = {**dict(bias_std=1.0, w1_scale=1.0), **kw}
    return make_model(["Cu"], L=0, K=12, r_c=6.0, width=0.5, n_hidden=3, hidden=128,
                      T_max=T_max, seed=seed, form="radial", **kw)


def water_model_radial(T_max=3, seed=0, **kw) -> ModelParams:
    """The water model's sizes in the radial message form: L = 0, 8 Gaussians centred
    uniformly on [0, 5] A, width 0.5 A, r_c = 5 A, two hidden layers of 64 SiLU units,
    F = K = 8 features, residual message updates, elements (H, O)."""
    kw = {**dict(bias_std=1.0, w1_scale=1.0), **kw}
    return make_model(["H", "O"], L=0, K=8, r_c=5.0, width=0.5, n_hidden=2, hidden=64,
                      T_max=T_max, seed=seed, form="radial", **kw)


def cu_model_diag(T_max=3, seed=0, **kw) -> ModelParams:
    """The Cu model's sizes with the literal Eq. (1) features (squares only, F = (L+1) K = 36).
    Squares of sums without the cross terms grow faster from layer to layer, so the first
    layer's weight scale is 0.3 (force RMS of order 1 eV/A, like the other presets)."""
    kw = {**dict(bias_std=1.0, w1_scale=0.3, ang_scale=1.0 / 6.0), **kw}
    return make_model(["Cu"], L=2, K=12, r_c=6.0, width=0.5, n_hidden=3, hidden=128,
                      T_max=T_max, seed=seed, form="diag", **kw)


def water_model_diag(T_max=3, seed=0, **kw) -> ModelParams:
    """The water model's sizes with the literal Eq. (1) features (F = (L+1) K = 24); first-layer
    weight scale 1 (force RMS of order 1 eV/A)."""
    kw = {**dict(bias_std=1.0, w1_scale=1.0, ang_scale=1.0 / 5.0), **kw}
    return make_model(["H", "O"], L=2, K=8, r_c=5.0, width=0.5, n_hidden=2, hidden=64,
                      T_max=T_max, seed=seed, form="diag", **kw)
