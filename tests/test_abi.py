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


def test_struct_layouts_and_constants_match_the_header(tmp_path):
    """The binding's ctypes structures and constants against the header, as a C compiler lays
    them out: every field's offset and every struct's size, and the REANN_* values the binding
    mirrors."""
    import shutil
    import subprocess
    from paper_2505_06711_amd import _binding as b
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    structs = {"reann_model_desc": b._ModelDesc, "reann_opts": b._Opts, "reann_server_opts": b._ServerOpts,
               "reann_request": b._Request, "reann_result": b._Result}
    consts = {"REANN_REQ_EVAL": b.REQ_EVAL, "REANN_REQ_VV_STEP": b.REQ_VV_STEP,
              "REANN_OUT_FORCES": b.OUTPUTS["forces"], "REANN_OUT_POSITIONS": b.OUTPUTS["positions"],
              "REANN_OUT_VELOCITIES": b.OUTPUTS["velocities"],
              "REANN_FORM_REANN": b.FORMS["reann"], "REANN_FORM_RADIAL": b.FORMS["radial"],
              "REANN_FORM_DIAG": b.FORMS["diag"], "REANN_EXCHANGE_MESSAGES": b.EXCHANGES["messages"],
              "REANN_EXCHANGE_NODE_FEATURES": b.EXCHANGES["node_features"],
              "REANN_N_SERVER_STATS": len(b.SERVER_STATS)}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "reann.h"', "int main(void) {"]
    for sn, cls in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (sn, sn))
        for f in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (sn, f[0], sn, f[0]))
    for cn in consts:
        lines.append('printf("%s %%lld\\n", (long long)(%s));' % (cn, cn))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                         text=True).stdout.splitlines())
    for sn, cls in structs.items():
        assert int(got["%s size" % sn]) == C.sizeof(cls), sn
        for f in cls._fields_:
            assert int(got["%s.%s" % (sn, f[0])]) == getattr(cls, f[0]).offset, (sn, f[0])
    for cn, v in consts.items():
        assert int(got[cn]) == v, cn
