"""CPU-side checks of the C ABI: the library loads, exports every declared symbol, and
rejects bad models without touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from synth import models

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2505_06711_amd", "libreann.so")


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "reann.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(reann_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libreann.so not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_header_symbols_exported(lib):
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_model_create_validates(lib):
    from paper_2505_06711_amd import _binding as b
    b.load()
    p = models.water_model(T_max=2, seed=0)
    m = b.Model(p)                    # valid model: no GPU needed
    assert m.handle
    bad = models.make_model(["H"], L=3, K=8, T_max=1)
    with pytest.raises(b.ReannError) as e:
        b.Model(bad)
    assert e.value.status == -2       # unsupported (L, K)
    p2 = models.water_model(T_max=2, seed=0)
    p2.energy_blob = p2.energy_blob.copy()
    p2.energy_blob[3] = np.nan
    with pytest.raises(b.ReannError) as e:
        b.Model(p2)
    assert e.value.status == -1
    assert "non-finite" in b.load().reann_last_error().decode()


def test_null_arguments_rejected(lib):
    from paper_2505_06711_amd import _binding as b
    L = b.load()
    assert L.reann_model_create(None, None) == -1
    assert L.reann_plan_forward(None, None, None, None, None) == -1
    assert L.reann_nlist_info(None, None, None, None, None) == -1
    L.reann_model_free(None)
    L.reann_ctx_free(None)
    L.reann_plan_free(None)
    L.reann_nlist_free(None)
    L.reann_server_destroy(None)
