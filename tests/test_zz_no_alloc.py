"""The allocation-free entry point reann_energy_forces_noalloc (static device scratch) against
reann_energy_forces on the same inputs, through the C ABI: the two share every kernel, so the
results must agree to the FP64 path's bounds (and in practice bit for bit).  Two calls in a
row, the second on a smaller system, so the second runs over the first one's leftover
scratch contents; plus the error paths (too large a system, a model not yet on the GPU)."""
import numpy as np
import pytest

from synth import models, systems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_06711_amd as rn
    return rn


def _agree(a, b, prec):
    tol_e, tol_f = (1e-12, 1e-10) if prec == "fp64" else (1e-6, 1e-5)
    Ea, Fa, Wa = a
    Eb, Fb, Wb = b
    den = max(abs(Ea), 1e-300)
    print("noalloc %s: E %.15g vs %.15g, max |dF| %.3e, max |dW| %.3e" % (prec, Eb, Ea, np.abs(Fa - Fb).max(),
                                                                        np.abs(Wa - Wb).max()), flush=True)
    assert abs(Ea - Eb) <= tol_e * den
    assert np.abs(Fa - Fb).max() <= tol_f * max(np.abs(Fa).max(), 1e-300)
    assert np.abs(Wa - Wb).max() <= tol_f * max(np.abs(Wa).max(), 1e-300)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_allocating_entry_point(rn, prec):
    ctx = rn.Context(0)
    big = systems.water_box(seed=70)                       # 192 atoms
    small = systems.water_box(grid=(3, 3, 3), spacing=systems.WATER_BOX_L / 4, seed=71)   # 81 atoms
    m = models.water_model(T_max=3, seed=70)
    model = rn.Model(m)
    for s in (big, small):   # second call: a smaller system over the first one's scratch contents
        ref = rn.energy_forces(ctx, model, s, T=3, precision=prec, skin=0.5)
        got = rn.energy_forces(ctx, model, s, T=3, precision=prec, skin=0.5, noalloc=True)
        _agree(ref, got, prec)


def test_noalloc_split_system_and_repeat(rn):
    """A 2x2x1 subdomain split (ghost gathers and reductions in the scratch) twice in a row:
    bitwise the same result both times."""
    ctx = rn.Context(0)
    s = systems.fcc_crystal((4, 4, 4), seed=72)
    m = models.cu_model(T_max=3, seed=72)
    model = rn.Model(m)
    ref = rn.energy_forces(ctx, model, s, T=3, precision="fp64", skin=1.0, decomp=(2, 2, 1))
    a = rn.energy_forces(ctx, model, s, T=3, precision="fp64", skin=1.0, decomp=(2, 2, 1), noalloc=True)
    b = rn.energy_forces(ctx, model, s, T=3, precision="fp64", skin=1.0, decomp=(2, 2, 1), noalloc=True)
    _agree(ref, a, "fp64")
    assert a[0] == b[0]
    np.testing.assert_array_equal(a[1], b[1])


def test_noalloc_refuses_too_large_and_unprepared(rn):
    ctx = rn.Context(0)
    m = models.cu_model(T_max=3, seed=73)
    model = rn.Model(m)
    s = systems.fcc_crystal((3, 3, 3), seed=73)
    with pytest.raises(rn.ReannError) as e:   # weights not yet on the GPU at this precision
        rn.energy_forces(ctx, model, s, T=3, precision="fp32", skin=1.0, noalloc=True)
    assert e.value.status == -7
    rn.energy_forces(ctx, model, s, T=3, precision="fp32", skin=1.0)      # puts them there
    big = systems.fcc_crystal((12, 12, 12), seed=74)                       # 6,912 atoms: > 64 MiB
    with pytest.raises(rn.ReannError) as e:
        rn.energy_forces(ctx, model, big, T=3, precision="fp32", skin=1.0, noalloc=True)
    assert e.value.status == -4
    # the entry point still works after a refused call
    ref = rn.energy_forces(ctx, model, s, T=3, precision="fp32", skin=1.0)
    got = rn.energy_forces(ctx, model, s, T=3, precision="fp32", skin=1.0, noalloc=True)
    _agree(ref, got, "fp32")
