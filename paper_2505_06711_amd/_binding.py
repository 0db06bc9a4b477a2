"""ctypes binding of ``libreann.so`` (declared in include/reann.h).

Argument marshalling only: every step of the evaluation runs in the library's HIP
kernels.  Importing fails loudly when the library has not been built.
"""
from __future__ import annotations

import atexit
import json
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libreann.so")

FP64, FP32, BF16, FP8 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "fp8": FP8}
REQ_EVAL, REQ_VV_STEP = 0, 1
OUTPUTS = {"forces": 1, "positions": 2, "velocities": 4}   # REANN_OUT_*
# reann_server_stats, in order (REANN_N_SERVER_STATS entries)
SERVER_STATS = ("admission_rounds", "completed", "atoms", "graph_replays", "deferred", "resident_bytes",
                "list_builds", "enqueue_ns", "graph_launch_ns", "finish_ns", "list_build_ns", "graph_capture_ns",
                "skin_checks", "skin_check_ns", "predicted_list_decisions")
OK, PENDING = 0, 1


class ReannError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("reann status %d: %s" % (status, msg))
        self.status = status


class _ModelDesc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("L", C.c_int32), ("K", C.c_int32), ("T_max", C.c_int32),
                ("n_hidden", C.c_int32), ("hidden", C.c_int32), ("r_c", C.c_double),
                ("ang_scale", C.c_double), ("energy_scale", C.c_double),
                ("centres", C.c_void_p), ("alphas", C.c_void_p), ("c0", C.c_void_p),
                ("msg", C.c_void_p), ("en", C.c_void_p), ("form", C.c_int32)]


FORMS = {"reann": 0, "radial": 1, "diag": 2}   # REANN_FORM_REANN, REANN_FORM_RADIAL, REANN_FORM_DIAG


class _Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("decomp", C.c_int32 * 3), ("skin", C.c_double), ("exchange", C.c_int32)]


EXCHANGES = {"messages": 0, "node_features": 1}   # REANN_EXCHANGE_MESSAGES, REANN_EXCHANGE_NODE_FEATURES


class _ServerOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_batch_atoms", C.c_int64), ("precision", C.c_int32),
                ("T", C.c_int32), ("skin", C.c_double), ("use_graph", C.c_int32), ("device", C.c_int32),
                ("thermostat_K", C.c_double), ("thermostat_tau_fs", C.c_double), ("decomp", C.c_int32 * 3),
                ("thermostat", C.c_int32), ("seed", C.c_uint64)]


class _Request(C.Structure):
    _fields_ = [("sys_id", C.c_uint64), ("kind", C.c_int32), ("dt_fs", C.c_double), ("pos", C.c_void_p),
                ("skip_outputs", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("energy", C.c_double), ("virial", C.c_double * 9), ("forces", C.c_void_p),
                ("positions", C.c_void_p), ("t_submit_ns", C.c_int64), ("t_done_ns", C.c_int64),
                ("status", C.c_int32), ("kinetic", C.c_double), ("velocities", C.c_void_p)]


_vp, _i32, _i64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
_SIGS = {
    "reann_last_error": (C.c_char_p, []),
    "reann_model_create": (_i32, [C.POINTER(_ModelDesc), C.POINTER(_vp)]),
    "reann_model_free": (None, [_vp]),
    "reann_model_load": (_i32, [C.c_char_p, C.POINTER(_vp)]),
    "reann_forward_dev": (_i32, [_vp, _vp, _vp, _vp]),
    "reann_backward_dev": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "reann_ctx_create": (_i32, [_i32, _vp, C.POINTER(_vp)]),
    "reann_ctx_free": (None, [_vp]),
    "reann_build_neighbors": (_i32, [_vp, _vp, _i64, _vp, _vp, _d, _d, _vp, C.POINTER(_vp)]),
    "reann_nlist_export": (_i32, [_vp, C.POINTER(_i64), _vp, _vp, _vp]),
    "reann_nlist_info": (_i32, [_vp, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64)]),
    "reann_nlist_free": (None, [_vp]),
    "reann_energy_forces": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _d, _i32, C.POINTER(_Opts), _vp, _vp, _vp]),
    "reann_energy_forces_noalloc": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _d, _i32, C.POINTER(_Opts), _vp, _vp,
                                           _vp]),
    "reann_plan_create": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _i32, C.POINTER(_Opts), C.POINTER(_vp)]),
    "reann_plan_forward": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "reann_plan_backward": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "reann_plan_free": (None, [_vp]),
    "reann_plan_get": (_i32, [_vp, _i32, _i32, _vp]),
    "reann_plan_set_timing": (_i32, [_vp, _i32]),
    "reann_plan_generation": (_i32, [_vp, C.POINTER(C.c_uint64)]),
    "reann_plan_set_list_policy": (_i32, [_vp, _i32]),
    "reann_plan_update_list": (_i32, [_vp, _vp, _vp, C.POINTER(C.c_int32)]),
    "reann_plan_set_energy_weights": (_i32, [_vp, _vp]),
    "reann_plan_timing": (_i32, [_vp, _vp, _vp, C.POINTER(_i64)]),
    "reann_server_create": (_i32, [_vp, C.POINTER(_ServerOpts), C.POINTER(_vp)]),
    "reann_server_set_masses": (_i32, [_vp, _vp]),
    "reann_system_add": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp, _vp, C.POINTER(C.c_uint64)]),
    "reann_submit": (_i32, [_vp, C.POINTER(_Request), C.POINTER(C.c_uint64)]),
    "reann_poll": (_i32, [_vp, C.c_uint64, C.POINTER(_Result)]),
    "reann_server_stats": (_i32, [_vp, _vp]),
    "reann_server_destroy": (None, [_vp]),
}

_lib = None

# Handles still alive when the interpreter exits are not freed one by one: teardown order
# is arbitrary and the process exit returns every device allocation anyway, so after this
# point close() makes no library call.
_LIVE = {k: weakref.WeakSet() for k in ("plan", "nlist", "server", "ctx", "model")}
_SHUTDOWN = [False]


def _mark_shutdown():
    _SHUTDOWN[0] = True


atexit.register(_mark_shutdown)


def _can_free(obj) -> bool:
    return bool(getattr(obj, "handle", None)) and _lib is not None and not _SHUTDOWN[0]


def load():
    """Load libreann.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libreann.so is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                              "or `python paper_2505_06711_amd/build.py`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def check(status: int) -> int:
    if status < 0:
        raise ReannError(status, load().reann_last_error().decode())
    return status


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


def _i32a(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _opts(precision="fp32", decomp=(1, 1, 1), skin=0.0, exchange="messages") -> _Opts:
    o = _Opts()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    for a in range(3):
        o.decomp[a] = int(decomp[a])
    o.skin = float(skin)
    o.exchange = EXCHANGES[exchange] if isinstance(exchange, str) else int(exchange)
    return o


class Model:
    """Device-ready model parameters (``reann_model``)."""

    def __init__(self, params):
        """``params``: a synth.models.ModelParams-like object."""
        lib = load()
        self.params = params
        self._keep = [_f64(params.centres), _f64(params.alphas), _f64(params.c0),
                      _f64(params.msg_blob if params.msg_blob.size else np.zeros(1)), _f64(params.energy_blob)]
        self.form = getattr(params, "form", "reann")
        d = _ModelDesc(params.n_species, params.L, params.K, params.T_max, params.n_hidden, params.hidden,
                       params.r_c, params.ang_scale, params.energy_scale, *[_p(a) for a in self._keep],
                       FORMS[self.form])
        h = _vp()
        check(lib.reann_model_create(C.byref(d), C.byref(h)))
        self.handle = h
        self.r_c = params.r_c
        self.T_max = params.T_max
        self.K, self.L = params.K, params.L
        _LIVE["model"].add(self)

    @classmethod
    def load(cls, spec_json_path: str) -> "Model":
        """A model from a spec written by ``save`` (``reann_model_load``); ``params`` is None."""
        self = cls.__new__(cls)
        h = _vp()
        check(load().reann_model_load(os.fsencode(spec_json_path), C.byref(h)))
        self.handle = h
        self.params = None
        self._keep = []
        spec = json.load(open(spec_json_path))
        self.r_c, self.T_max, self.K, self.L = float(spec["r_c"]), int(spec["T_max"]), int(spec["K"]), int(spec["L"])
        self.form = spec.get("form", "reann")
        _LIVE["model"].add(self)
        return self

    def save(self, spec_json_path: str, weights_name: str = None):
        """Write the parameters as a JSON spec plus a raw FP64 weight file (the formats read
        by ``reann_model_load``); the weight file goes next to the spec."""
        p = self.params
        if p is None:
            raise ValueError("model was loaded from files; nothing to save")
        base = os.path.splitext(os.path.basename(spec_json_path))[0]
        weights_name = weights_name or base + ".weights.f64"
        d = os.path.dirname(os.path.abspath(spec_json_path))
        blob = np.concatenate([np.asarray(a, np.float64).ravel() for a in
                               (p.centres, p.alphas, p.c0, p.msg_blob, p.energy_blob)])
        blob.astype("<f8").tofile(os.path.join(d, weights_name))
        spec = dict(format="reann-model", version=1, n_species=int(p.n_species), L=int(p.L), K=int(p.K),
                    T_max=int(p.T_max), n_hidden=int(p.n_hidden), hidden=int(p.hidden), r_c=float(p.r_c),
                    ang_scale=float(p.ang_scale), energy_scale=float(p.energy_scale),
                    form=getattr(p, "form", "reann"), elements=list(getattr(p, "elements", [])), weights=weights_name)
        with open(spec_json_path, "w") as f:
            json.dump(spec, f, indent=1)

    def close(self):
        if _can_free(self):
            _lib.reann_model_free(self.handle)
        self.handle = None

    __del__ = close


class Context:
    """One GPU and one HIP stream (``reann_ctx``).  ``stream``: an int handle, a
    torch.cuda.Stream, or None for a library-created stream."""

    def __init__(self, device: int = 0, stream=None):
        lib = load()
        if stream is not None and hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        h = _vp()
        check(lib.reann_ctx_create(int(device), stream, C.byref(h)))
        self.handle = h
        self.device = device
        _LIVE["ctx"].add(self)

    def close(self):
        if _can_free(self):
            _lib.reann_ctx_free(self.handle)   # the library keeps it until its plans/lists are freed
        self.handle = None

    __del__ = close


class NeighborList:
    def __init__(self, handle, ctx=None):
        self.handle = handle
        self.ctx = ctx
        _LIVE["nlist"].add(self)

    def info(self):
        a, g, p, q = _i64(), _i64(), _i64(), _i64()
        check(load().reann_nlist_info(self.handle, C.byref(a), C.byref(g), C.byref(p), C.byref(q)))
        return dict(n_atoms=a.value, n_ghosts=g.value, n_pairs=p.value, n_local_pairs=q.value)

    def export(self):
        """(row[n+1], j[n_pairs], shift[n_pairs, 3]) in canonical (j, shift) row order."""
        lib = load()
        cnt = _i64()
        check(lib.reann_nlist_export(self.handle, C.byref(cnt), None, None, None))
        n = self.info()["n_atoms"]
        row = np.zeros(n + 1, np.int64)
        j = np.zeros(max(cnt.value, 1), np.int64)
        sh = np.zeros((max(cnt.value, 1), 3), np.int32)
        check(lib.reann_nlist_export(self.handle, C.byref(cnt), _p(row), _p(j), _p(sh)))
        return row, j[:cnt.value], sh[:cnt.value]

    def close(self):
        if _can_free(self):
            _lib.reann_nlist_free(self.handle)
        self.handle = None

    __del__ = close


def build_neighbors(ctx: Context, system: dict, r_c: float, skin: float = 0.0, decomp=(1, 1, 1)) -> NeighborList:
    pos = _f64(system["pos"])
    cell = _f64(system["cell"], (9,))
    pbc = _i32a(system["pbc"])
    dec = _i32a(decomp)
    h = _vp()
    check(load().reann_build_neighbors(ctx.handle, _p(pos), pos.shape[0], _p(cell), _p(pbc), float(r_c), float(skin),
                                       _p(dec), C.byref(h)))
    return NeighborList(h, ctx)


def energy_forces(ctx: Context, model: Model, system: dict, T: int, precision="fp32", decomp=(1, 1, 1),
                  skin: float = 0.0, forces: bool = True, noalloc: bool = False, exchange="messages"):
    """Host-pointer evaluation: returns (E, F[n,3] or None, W[3,3] or None).  noalloc=True
    calls reann_energy_forces_noalloc (no device allocation; bounded system size).  exchange:
    "messages" (the paper's per-layer exchange) or "node_features" (see reann_opts)."""
    pos = _f64(system["pos"])
    spec = _i32a(system["species"])
    cell = _f64(system["cell"], (9,))
    pbc = _i32a(system["pbc"])
    n = pos.shape[0]
    E = np.zeros(1)
    F = np.zeros((n, 3)) if forces else None
    W = np.zeros(9) if forces else None
    o = _opts(precision, decomp, skin, exchange)
    fn = load().reann_energy_forces_noalloc if noalloc else load().reann_energy_forces
    check(fn(ctx.handle, model.handle, _p(pos), _p(spec), n, _p(cell), _p(pbc), float(model.r_c), int(T),
             C.byref(o), _p(E), _p(F), _p(W)))
    return float(E[0]), F, (W.reshape(3, 3) if forces else None)


class Plan:
    """Device-pointer evaluation of one system (``reann_plan``).  Tensors are torch
    tensors on the context's GPU; the stream defaults to torch's current stream."""

    def __init__(self, ctx: Context, model: Model, system: dict, T: int, precision="fp32", decomp=(1, 1, 1),
                 skin: float = 0.0, exchange="messages"):
        lib = load()
        self.ctx, self.model = ctx, model
        spec = _i32a(system["species"])
        cell = _f64(system["cell"], (9,))
        pbc = _i32a(system["pbc"])
        self.n = spec.shape[0]
        self.T = T
        o = _opts(precision, decomp, skin, exchange)
        h = _vp()
        check(lib.reann_plan_create(ctx.handle, model.handle, _p(spec), self.n, _p(cell), _p(pbc), int(T),
                                    C.byref(o), C.byref(h)))
        self.handle = h
        self.L, self.K = model.L, model.K
        _LIVE["plan"].add(self)

    @staticmethod
    def _stream(stream):
        import torch
        if stream is None:
            return torch.cuda.current_stream().cuda_stream
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream

    def forward(self, pos, energy, atom_energy=None, stream=None):
        """pos: float64 [n,3] device tensor; energy: float64 [] device tensor (written)."""
        _require_device_f64(pos, (self.n, 3))
        _require_device_f64(energy, ())
        ae = None
        if atom_energy is not None:
            _require_device_f64(atom_energy, (self.n,))
            ae = atom_energy.data_ptr()
        check(load().reann_plan_forward(self.handle, pos.data_ptr(), energy.data_ptr(), ae, self._stream(stream)))

    def backward(self, forces, grad_energy=None, virial=None, stream=None):
        """forces: float64 [n,3] device tensor receiving -g dE/dx; grad_energy: float64 []
        device tensor g or None (= 1); virial: float64 [3,3] device tensor or None."""
        _require_device_f64(forces, (self.n, 3))
        g = None
        if grad_energy is not None:
            _require_device_f64(grad_energy, ())
            g = grad_energy.data_ptr()
        w = None
        if virial is not None:
            _require_device_f64(virial, (3, 3))
            w = virial.data_ptr()
        check(load().reann_plan_backward(self.handle, g, forces.data_ptr(), w, self._stream(stream)))

    def set_list_policy(self, auto_check: bool):
        """True (the default): every forward checks the skin rule and rebuilds when needed (one
        stream synchronisation).  False: forwards use the list as it is, with no host
        synchronisation or allocation, so forward + backward can be captured in a graph; keep
        the list valid with ``update_list``."""
        check(load().reann_plan_set_list_policy(self.handle, int(bool(auto_check))))

    def update_list(self, pos, stream=None) -> bool:
        """Skin check at ``pos`` (device FP64 [n, 3]) and a rebuild if needed; True if rebuilt
        (a graph captured earlier must then be captured again)."""
        r = C.c_int32(0)
        check(load().reann_plan_update_list(self.handle, pos.data_ptr(), self._stream(stream), C.byref(r)))
        return bool(r.value)

    def set_energy_weights(self, w=None):
        """E = sum_i w_i E_i (w: [n] in caller order; None = all 1); the backward follows."""
        if w is None:
            check(load().reann_plan_set_energy_weights(self.handle, None))
            return
        wa = _f64(w, (self.n,))
        check(load().reann_plan_set_energy_weights(self.handle, _p(wa)))

    def generation(self) -> int:
        """Number of forwards run on this plan (a backward uses the latest one's state)."""
        g = C.c_uint64(0)
        check(load().reann_plan_generation(self.handle, C.byref(g)))
        return g.value

    def get(self, what: str, t: int = 0) -> np.ndarray:
        """Intermediates of the last forward in caller atom order: 'S' [n,NL,K], 'c' [n,K],
        'atom_energy' [n]."""
        NL = (self.L + 1) * (self.L + 2) * (self.L + 3) // 6
        code, shape = {"S": (0, (self.n, NL, self.K)), "c": (1, (self.n, self.K)),
                       "atom_energy": (2, (self.n,))}[what]
        out = np.zeros(shape)
        check(load().reann_plan_get(self.handle, code, int(t), _p(out)))
        return out

    def set_timing(self, on: bool = True):
        check(load().reann_plan_set_timing(self.handle, int(bool(on))))

    PHASES = ("nlist", "edge_fwd", "density", "nn_fwd", "ghost", "nn_bwd", "density_adj", "adj_centre",
              "adj_gather", "other")

    def timing(self) -> dict:
        """Per-phase kernel milliseconds accumulated since the last call (see reann.h)."""
        ms = np.zeros(len(self.PHASES))
        la = np.zeros(len(self.PHASES), np.int64)
        steps = _i64()
        check(load().reann_plan_timing(self.handle, _p(ms), _p(la), C.byref(steps)))
        return dict(ms=dict(zip(self.PHASES, ms.tolist())), launches=dict(zip(self.PHASES, la.tolist())),
                    steps=steps.value)

    def close(self):
        if _can_free(self):
            _lib.reann_plan_free(self.handle)
        self.handle = None

    __del__ = close


def _require_device_f64(t, shape):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 device tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (tuple(shape), tuple(t.shape)))


class Server:
    """Continuous-batching server (``reann_server``): systems stay resident on the device,
    requests are admitted as slots and HBM budget free up (see include/reann.h)."""

    def __init__(self, model: Model, T: int, precision="bf16", skin: float = 1.0, hbm_budget_bytes: int = 0,
                 max_batch_atoms: int = 0, use_graph: bool = True, device: int = 0, thermostat_K: float = 0.0,
                 thermostat_tau_fs: float = 0.0, decomp=(1, 1, 1), thermostat: str = "berendsen", seed: int = 0):
        lib = load()
        o = _ServerOpts()
        o.hbm_budget_bytes = int(hbm_budget_bytes)
        o.max_batch_atoms = int(max_batch_atoms)
        o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        o.T = int(T)
        o.skin = float(skin)
        o.use_graph = int(bool(use_graph))
        o.device = int(device)
        o.thermostat_K = float(thermostat_K)
        o.thermostat_tau_fs = float(thermostat_tau_fs)
        for a in range(3):
            o.decomp[a] = int(decomp[a])
        o.thermostat = {"berendsen": 0, "csvr": 1}[thermostat]
        o.seed = int(seed)
        h = _vp()
        check(lib.reann_server_create(model.handle, C.byref(o), C.byref(h)))
        self.handle = h
        self.model = model
        self.n_atoms = {}
        self._poll_bufs = {}
        _LIVE["server"].add(self)

    def set_masses(self, masses_amu):
        m = _f64(masses_amu)
        check(load().reann_server_set_masses(self.handle, _p(m)))

    def add_system(self, system: dict, vel=None) -> int:
        pos = _f64(system["pos"])
        spec = _i32a(system["species"])
        cell = _f64(system["cell"], (9,))
        pbc = _i32a(system["pbc"])
        v = None if vel is None else _f64(vel)
        sid = C.c_uint64()
        check(load().reann_system_add(self.handle, _p(spec), pos.shape[0], _p(cell), _p(pbc), _p(pos), _p(v),
                                      C.byref(sid)))
        self.n_atoms[sid.value] = pos.shape[0]
        return sid.value

    def _submit(self, sys_id, kind, dt=0.0, pos=None, skip=()) -> int:
        r = _Request()
        r.sys_id = int(sys_id)
        r.kind = int(kind)
        r.dt_fs = float(dt)
        bad = set(skip) - set(OUTPUTS)
        if bad:
            raise ValueError("unknown outputs %s (known: %s)" % (sorted(bad), sorted(OUTPUTS)))
        r.skip_outputs = sum(OUTPUTS[k] for k in set(skip))
        keep = None
        if pos is not None:
            keep = _f64(pos)
            r.pos = keep.ctypes.data
        t = C.c_uint64()
        check(load().reann_submit(self.handle, C.byref(r), C.byref(t)))
        return t.value

    def submit_eval(self, sys_id: int, pos, skip=()) -> int:
        """skip: names in OUTPUTS of result vectors left on the device."""
        return self._submit(sys_id, REQ_EVAL, pos=pos, skip=skip)

    def submit_vv(self, sys_id: int, dt_fs: float, skip=()) -> int:
        """skip: names in OUTPUTS of result vectors left on the device."""
        return self._submit(sys_id, REQ_VV_STEP, dt=dt_fs, skip=skip)

    def poll(self, ticket: int, sys_id: int, forces: bool = True, positions: bool = False, velocities: bool = False):
        """None while pending; else a dict with energy, virial, forces, positions, velocities,
        kinetic (eV, velocity-Verlet steps), latency_s.  A vector asked for here must not have
        been skipped at submit (ReannError otherwise, and the result stays for another poll)."""
        n = self.n_atoms[sys_id]
        res = _Result()
        # the output arrays of a ticket are made once and kept while it is pending
        key = (ticket, forces, positions, velocities)
        bufs = self._poll_bufs.get(ticket)
        if bufs is None or bufs[0] != key:
            bufs = (key,) + tuple(np.empty((n, 3)) if w else None for w in (forces, positions, velocities))
            self._poll_bufs[ticket] = bufs
        _, F, P, V = bufs
        res.forces = None if F is None else F.ctypes.data
        res.positions = None if P is None else P.ctypes.data
        res.velocities = None if V is None else V.ctypes.data
        st = load().reann_poll(self.handle, C.c_uint64(ticket), C.byref(res))
        if st == PENDING:
            return None
        self._poll_bufs.pop(ticket, None)
        check(st)
        return dict(energy=res.energy, virial=np.array(res.virial[:]).reshape(3, 3), forces=F, positions=P,
                    velocities=V, kinetic=res.kinetic, latency_s=(res.t_done_ns - res.t_submit_ns) * 1e-9, t_done_ns=res.t_done_ns)

    def stats(self) -> dict:
        out = np.zeros(len(SERVER_STATS), np.int64)
        check(load().reann_server_stats(self.handle, _p(out)))
        return dict(zip(SERVER_STATS, out.tolist()))

    def close(self):
        if _can_free(self):
            _lib.reann_server_destroy(self.handle)
        self.handle = None

    __del__ = close
