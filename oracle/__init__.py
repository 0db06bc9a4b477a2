"""FP64 CPU oracle for the REANN energy / forces / virial path.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check and
by the benchmark's CPU-baseline leg, never by the GPU library or its binding.
It shares no code with the GPU path; see ``reann_oracle.c`` for what it follows
in the paper and for every reading of points the paper leaves open.

``build()`` compiles ``reann_oracle.c`` with gcc into ``liboracle.so`` next to it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "reann_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (FP64, no floating-point contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Model(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("L", C.c_int32), ("K", C.c_int32), ("T_max", C.c_int32),
                ("n_hidden", C.c_int32), ("hidden", C.c_int32), ("r_c", C.c_double),
                ("ang_scale", C.c_double), ("energy_scale", C.c_double),
                ("centres", C.c_void_p), ("alphas", C.c_void_p), ("c0", C.c_void_p),
                ("msg", C.c_void_p), ("en", C.c_void_p), ("form", C.c_int32)]

FORMS = {"reann": 0, "radial": 1, "diag": 2}   # forms of reann_oracle.c (readings R1-R5, R14, R15)


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB_OVERRIDE")   # e.g. a deliberately mutated build
        if not path:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            path = _LIB
        lib = C.CDLL(path)
        lib.oracle_neighbors.restype = C.c_int64
        lib.oracle_neighbors.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.oracle_eval.restype = C.c_int
        lib.oracle_eval.argtypes = [C.POINTER(_Model), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_double, C.c_int32, C.c_void_p, C.c_int32, C.c_int32,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.oracle_eval_halo.restype = C.c_int
        lib.oracle_eval_halo.argtypes = [C.POINTER(_Model), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_double, C.c_int32, C.c_void_p, C.c_int32,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _sys_arrays(system):
    pos = np.ascontiguousarray(system["pos"], dtype=np.float64)
    cell = np.ascontiguousarray(system["cell"], dtype=np.float64).reshape(9)
    pbc = np.ascontiguousarray(system["pbc"], dtype=np.int32)
    return pos, cell, pbc


def neighbors(system: dict, rcut: float, decomp=(1, 1, 1)):
    """Canonical neighbour list: (row[n+1], j[n_pairs], shift[n_pairs,3]) with each row
    sorted by (owner j, shift); built through the given subdomain split."""
    lib = _load()
    pos, cell, pbc = _sys_arrays(system)
    n = pos.shape[0]
    dec = np.ascontiguousarray(decomp, dtype=np.int32)
    cnt = lib.oracle_neighbors(n, _p(pos), _p(cell), _p(pbc), float(rcut), _p(dec), None, None, None)
    if cnt < 0:
        raise ValueError("oracle_neighbors failed: %d" % cnt)
    row = np.zeros(n + 1, np.int64)
    j = np.zeros(max(cnt, 1), np.int64)
    sh = np.zeros((max(cnt, 1), 3), np.int32)
    cnt2 = lib.oracle_neighbors(n, _p(pos), _p(cell), _p(pbc), float(rcut), _p(dec), _p(row), _p(j), _p(sh))
    assert cnt2 == cnt
    return row, j[:cnt], sh[:cnt]


def n_lambda(L: int) -> int:
    return (L + 1) * (L + 2) * (L + 3) // 6


def _model_struct(model):
    keep = [np.ascontiguousarray(a, dtype=np.float64) for a in
            (model.centres, model.alphas, model.c0, model.msg_blob, model.energy_blob)]
    if keep[3].size == 0:
        keep[3] = np.zeros(1)
    mm = _Model(model.n_species, model.L, model.K, model.T_max, model.n_hidden, model.hidden, model.r_c,
                model.ang_scale, model.energy_scale, *[_p(a) for a in keep],
                FORMS[getattr(model, "form", "reann")])
    return mm, keep


def evaluate_halo(model, system: dict, T: int, skin: float = 0.0, decomp=(1, 1, 1), forces: bool = True,
                  threads: int = 0) -> dict:
    """The extended-halo scheme (every subdomain evaluates all copies within T (r_c + skin) of
    its box, no exchange between layers; see oracle_eval_halo).  Returns energy, atom_energy,
    forces, virial and work [T, 2] (rows and in-cutoff edges evaluated per layer, summed over
    subdomains)."""
    lib = _load()
    pos, cell, pbc = _sys_arrays(system)
    spec = np.ascontiguousarray(system["species"], dtype=np.int32)
    n = pos.shape[0]
    mm, keep = _model_struct(model)
    E = np.zeros(1)
    Ei = np.zeros(n)
    F = np.zeros((n, 3)) if forces else None
    W = np.zeros(9) if forces else None
    work = np.zeros((T, 2), np.int64)
    dec = np.ascontiguousarray(decomp, dtype=np.int32)
    rc = lib.oracle_eval_halo(C.byref(mm), n, _p(pos), _p(spec), _p(cell), _p(pbc), float(skin), int(T), _p(dec),
                              int(threads), _p(E), _p(Ei), _p(F), _p(W), _p(work))
    if rc != 0:
        raise ValueError("oracle_eval_halo failed: %d" % rc)
    out = dict(energy=float(E[0]), atom_energy=Ei, work=work)
    if forces:
        out["forces"] = F
        out["virial"] = W.reshape(3, 3)
    return out


def evaluate(model, system: dict, T: int, skin: float = 0.0, decomp=(1, 1, 1), naive: bool = False,
             forces: bool = True, want_S: bool = False, want_c: bool = False, threads: int = 0) -> dict:
    """Evaluate E (eV), per-atom E_i, F (eV/A), virial W (eV, W = sum_edges d (x) f).

    ``model`` is a ``synth.models.ModelParams``.  Returns a dict with keys
    energy, atom_energy, forces, virial and optionally S [T,n,NL,K], c [T,n,K]."""
    lib = _load()
    pos, cell, pbc = _sys_arrays(system)
    spec = np.ascontiguousarray(system["species"], dtype=np.int32)
    n = pos.shape[0]
    K, NL = model.K, n_lambda(model.L)
    mm, keep = _model_struct(model)
    E = np.zeros(1)
    Ei = np.zeros(n)
    F = np.zeros((n, 3)) if forces else None
    W = np.zeros(9) if forces else None
    S = np.zeros((T, n, NL, K)) if want_S else None
    cc = np.zeros((T, n, K)) if want_c else None
    dec = np.ascontiguousarray(decomp, dtype=np.int32)
    rc = lib.oracle_eval(C.byref(mm), n, _p(pos), _p(spec), _p(cell), _p(pbc), float(skin), int(T), _p(dec),
                         int(bool(naive)), int(threads), _p(E), _p(Ei), _p(F), _p(W), _p(S), _p(cc))
    if rc != 0:
        raise ValueError("oracle_eval failed: %d" % rc)
    out = dict(energy=float(E[0]), atom_energy=Ei)
    if forces:
        out["forces"] = F
        out["virial"] = W.reshape(3, 3)
    if want_S:
        out["S"] = S
    if want_c:
        out["c"] = cc
    return out
