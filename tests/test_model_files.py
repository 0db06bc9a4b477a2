"""Model files (reann_model_load): a JSON spec plus a raw FP64 weight file, written by
Model.save.  CPU checks of the reader; the GPU check that a loaded model evaluates exactly
like the one it was saved from is in test_gpu_model_files.py."""
import json
import os

import numpy as np
import pytest

from synth import models


@pytest.fixture(scope="module")
def b():
    from paper_2505_06711_amd import _binding as b
    b.load()
    return b


def test_save_then_load(b, tmp_path):
    p = models.water_model(T_max=3, seed=4)
    spec = str(tmp_path / "water.json")
    b.Model(p).save(spec)
    d = json.load(open(spec))
    assert d["format"] == "reann-model" and d["K"] == p.K and d["elements"] == list(p.elements)
    w = np.fromfile(str(tmp_path / d["weights"]), dtype="<f8")
    assert w.size == 2 * p.K + p.c0.size + p.msg_blob.size + p.energy_blob.size
    m = b.Model.load(spec)
    assert (m.K, m.L, m.T_max, m.r_c) == (p.K, p.L, p.T_max, p.r_c)


def _expect_error(b, spec, text):
    with pytest.raises(b.ReannError) as e:
        b.Model.load(spec)
    assert e.value.status == -1 and text in str(e.value)


def test_load_rejects_bad_files(b, tmp_path):
    p = models.cu_model(T_max=2, seed=1)
    spec = str(tmp_path / "cu.json")
    b.Model(p).save(spec)
    good = json.load(open(spec))
    # a missing member
    d = dict(good); del d["hidden"]
    json.dump(d, open(spec, "w")); _expect_error(b, spec, "hidden")
    # a non-numeric value
    d = dict(good); d["r_c"] = "six"
    json.dump(d, open(spec, "w")); _expect_error(b, spec, "r_c")
    # wrong format tag
    d = dict(good); d["format"] = "other"
    json.dump(d, open(spec, "w")); _expect_error(b, spec, "format")
    # weight file one value short
    json.dump(good, open(spec, "w"))
    wpath = str(tmp_path / good["weights"])
    w = np.fromfile(wpath, dtype="<f8")
    w[:-1].tofile(wpath); _expect_error(b, spec, "expected")
    # not JSON at all
    open(spec, "w").write("K = 12\n"); _expect_error(b, spec, "JSON")
    # no such file
    _expect_error(b, str(tmp_path / "missing.json"), "cannot open")


def test_radial_form_save_then_load(b, tmp_path):
    """The second message form's models: F = K features in the weight file, the form kept."""
    p = models.water_model_radial(T_max=3, seed=5)
    spec = str(tmp_path / "radial.json")
    b.Model(p).save(spec)
    d = json.load(open(spec))
    assert d["form"] == "radial" and d["L"] == 0
    w = np.fromfile(str(tmp_path / d["weights"]), dtype="<f8")
    assert w.size == 2 * p.K + p.c0.size + p.msg_blob.size + p.energy_blob.size
    m = b.Model.load(spec)
    assert m.form == "radial" and (m.K, m.L) == (p.K, 0)
    d["form"] = "spherical"
    json.dump(d, open(spec, "w")); _expect_error(b, spec, "form")


def test_form_and_L_must_agree(b):
    p = models.water_model_radial(T_max=2, seed=6)
    p.form = "reann"            # L = 0 is not a REANN model here
    with pytest.raises(b.ReannError):
        b.Model(p)
    q = models.water_model(T_max=2, seed=6)
    q.form = "radial"           # the radial form takes L = 0
    with pytest.raises(b.ReannError):
        b.Model(q)


def test_diag_form_save_then_load(b, tmp_path):
    p = models.water_model(T_max=2, seed=7, form="diag")
    spec = str(tmp_path / "diag.json")
    b.Model(p).save(spec)
    d = json.load(open(spec))
    assert d["form"] == "diag"
    w = np.fromfile(str(tmp_path / d["weights"]), dtype="<f8")
    assert w.size == 2 * p.K + p.c0.size + p.msg_blob.size + p.energy_blob.size
    assert b.Model.load(spec).form == "diag"
