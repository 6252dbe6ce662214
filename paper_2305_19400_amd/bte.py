"""Python binding of the HIP BTE library (``libbte.so``, C ABI in include/bte.h).

Argument marshalling only: every step of the time step runs in the library's
HIP kernels.  PyTorch provides the device workspace (a uint8 tensor owned by
the Solver) and the stream handle; nothing here computes the method.  There is
no CPU fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbte.so")

BTE_OK = 0
BTE_E_INVAL = -1
BTE_E_NOMEM = -2
BTE_E_DEVICE = -3
BTE_E_NUMERIC = -4
BTE_E_NOTCONV = -5
BTE_E_STATE = -6

BTE_WALL_ISOTHERMAL, BTE_WALL_SPECULAR, BTE_WALL_SYMMETRY, BTE_WALL_DIFFUSE = 0, 1, 2, 3
BTE_IMPLICIT_JACOBI, BTE_EXPLICIT_EULER = 0, 1
BTE_FP64, BTE_FP32_MIXED = 0, 1
BTE_T_TAU_WEIGHTED, BTE_T_ENERGY = 0, 1
BTE_WARM_NONE, BTE_WARM_T, BTE_WARM_T_SHIFT = 0, 1, 2

# every symbol include/bte.h declares
EXPORTS = ("bte_workspace_size", "bte_create", "bte_step", "bte_temperature", "bte_intensity",
           "bte_energy", "bte_set_fields", "bte_state_size", "bte_get_state", "bte_set_state",
           "bte_set_wall_temperature", "bte_sweep_time", "bte_sweep_layout",
           "bte_nn_param_count", "bte_nn_params",
           "bte_nn_set_params", "bte_nn_predict", "bte_nn_gradient", "bte_autotune",
           "bte_batch_create", "bte_batch_step", "bte_batch_destroy", "bte_batch_step_static",
           "bte_destroy",
           "bte_last_error")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class bte_mesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double * 3), ("wall", C.c_int * 6),
                ("wall_T", _dp * 6), ("T_init", _dp)]


class bte_dirs(C.Structure):
    _fields_ = [("n", C.c_int), ("s", _dp), ("w", _dp)]


class bte_bands(C.Structure):
    _fields_ = [("n", C.c_int), ("omega", _dp), ("domega", _dp)]


class bte_dispersion(C.Structure):
    _fields_ = [("vg", _dp), ("tau", _dp), ("dos", _dp), ("deg", _dp), ("tau_exp", _dp),
                ("tau_T0", C.c_double)]


class bte_options(C.Structure):
    _fields_ = [("dt", C.c_double), ("tol", C.c_double), ("max_inner", C.c_int),
                ("scheme", C.c_int), ("precision", C.c_int), ("t_definition", C.c_int),
                ("fail_on_notconv", C.c_int), ("timing", C.c_int), ("stream", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("warm_start", C.c_int), ("nn_train_steps", C.c_int), ("nn_epochs", C.c_int),
                ("nn_lr", C.c_float), ("nn_seed", C.c_ulonglong), ("nn_guard", C.c_int)]


class bte_step_stats(C.Structure):
    _fields_ = [("inner", C.c_int), ("converged", C.c_int), ("newton_max", C.c_int),
                ("warm", C.c_int), ("res", C.c_double), ("fallbacks", C.c_int),
                ("trained", C.c_int), ("nn_loss", C.c_double)]


class bte_state_header(C.Structure):
    _fields_ = [("magic", C.c_char * 8), ("version", C.c_int), ("header_bytes", C.c_int),
                ("dim", C.c_int), ("n", C.c_int * 3), ("nd", C.c_int), ("nb", C.c_int),
                ("precision", C.c_int), ("scheme", C.c_int), ("warm_start", C.c_int),
                ("nn_rec", C.c_int), ("layout", C.c_int * 4), ("steps", C.c_longlong),
                ("nn_recorded", C.c_int), ("nn_trained", C.c_int), ("nn_off", C.c_int),
                ("nn_warm_steps", C.c_int), ("nn_warm_sweeps", C.c_int), ("nn_adam_t", C.c_int),
                ("nn_last_batch", C.c_int), ("nn_params", C.c_int),
                ("off", C.c_ulonglong * 11), ("total", C.c_ulonglong)]


class BteError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load the in-tree libbte.so; raises if it has not been built.

    torch is imported first so that the process holds one HIP runtime: the
    library's libamdhip64.so.7 dependency then resolves to the copy torch has
    already loaded (two runtimes in one process do not share the device)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (see docstring)
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with paper_2305_19400_amd.build.build()")
    lib = C.CDLL(path)
    lib.bte_workspace_size.argtypes = [C.POINTER(bte_mesh), C.POINTER(bte_dirs),
                                       C.POINTER(bte_bands), C.POINTER(bte_options),
                                       C.POINTER(C.c_size_t)]
    lib.bte_create.argtypes = [C.POINTER(bte_mesh), C.POINTER(bte_dirs), C.POINTER(bte_bands),
                               C.POINTER(bte_dispersion), C.POINTER(bte_options),
                               C.POINTER(C.c_void_p)]
    lib.bte_step.argtypes = [C.c_void_p, C.c_int, _ip, C.POINTER(bte_step_stats)]
    lib.bte_temperature.argtypes = [C.c_void_p, _dp, C.c_size_t]
    lib.bte_intensity.argtypes = [C.c_void_p, _dp, C.c_size_t]
    lib.bte_energy.argtypes = [C.c_void_p, _dp, C.c_size_t]
    lib.bte_set_fields.argtypes = [C.c_void_p, _dp, C.c_size_t, _dp, C.c_size_t]
    lib.bte_state_size.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
    lib.bte_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    lib.bte_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    lib.bte_set_wall_temperature.argtypes = [C.c_void_p, C.c_int, _dp, C.c_size_t]
    lib.bte_sweep_time.argtypes = [C.c_void_p, _dp, _ip]
    lib.bte_sweep_layout.argtypes = [C.c_void_p, _ip, _ip, _ip, _ip]
    _fp = C.POINTER(C.c_float)
    lib.bte_nn_param_count.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
    lib.bte_nn_params.argtypes = [C.c_void_p, _fp, C.c_size_t]
    lib.bte_nn_set_params.argtypes = [C.c_void_p, _fp, C.c_size_t]
    lib.bte_nn_predict.argtypes = [C.c_void_p, _dp, C.c_size_t]
    lib.bte_nn_gradient.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, C.c_size_t, _fp, C.c_size_t,
                                    _dp, _fp]
    lib.bte_destroy.argtypes = [C.c_void_p]
    lib.bte_autotune.argtypes = [C.c_void_p, C.c_char_p, _ip, _ip, _ip, _dp]
    lib.bte_batch_create.argtypes = [C.c_int, C.POINTER(C.c_void_p), C.c_int,
                                     C.POINTER(C.c_void_p)]
    lib.bte_batch_step.argtypes = [C.c_void_p, C.c_int, C.POINTER(bte_step_stats)]
    lib.bte_batch_destroy.argtypes = [C.c_void_p]
    lib.bte_batch_step_static.argtypes = [C.c_int, C.POINTER(C.c_void_p), C.c_int,
                                          C.POINTER(bte_step_stats)]
    lib.bte_last_error.restype = C.c_char_p
    for name in EXPORTS:
        getattr(lib, name).restype = C.c_char_p if name == "bte_last_error" else C.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != BTE_OK:
        raise BteError(rc, load_library().bte_last_error().decode())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class _Inputs:
    """C structs for one instance; keeps the host arrays alive while in use."""

    def __init__(self, inst, opts: dict):
        self.keep = []

        def ptr(a):
            a = _f64(a)
            self.keep.append(a)
            return a.ctypes.data_as(_dp)

        m = bte_mesh()
        m.dim = int(inst.dim)
        for a in range(3):
            m.n[a] = int(inst.n[a])
            m.h[a] = float(inst.h[a])
        for f in range(6):
            m.wall[f] = int(inst.wall[f])
            m.wall_T[f] = ptr(inst.wall_T[f]) if inst.wall_T[f] is not None else _dp()
        m.T_init = ptr(inst.T_init)
        d = bte_dirs(int(inst.s.shape[0]), ptr(inst.s), ptr(inst.w))
        b = bte_bands(int(inst.omega.shape[0]), ptr(inst.omega), ptr(inst.domega))
        tau_exp = getattr(inst, "tau_exp", None)
        disp = bte_dispersion(ptr(inst.vg), ptr(inst.tau), ptr(inst.dos), ptr(inst.deg),
                              ptr(tau_exp) if tau_exp is not None else _dp(),
                              float(getattr(inst, "tau_T0", 300.0)))
        o = bte_options()
        o.dt = float(opts["dt"])
        o.tol = float(opts["tol"])
        o.max_inner = int(opts["max_inner"])
        o.scheme = int(opts["scheme"])
        o.precision = int(opts["precision"])
        o.t_definition = int(opts["t_definition"])
        o.fail_on_notconv = int(opts.get("fail_on_notconv", 0))
        o.timing = int(bool(opts.get("timing", False)))
        o.warm_start = int(opts.get("warm_start", 0))
        o.nn_train_steps = int(opts.get("nn_train_steps", 0))
        o.nn_epochs = int(opts.get("nn_epochs", 0))
        o.nn_lr = float(opts.get("nn_lr", 0.0))
        o.nn_seed = int(opts.get("nn_seed", 0))
        o.nn_guard = int(opts.get("nn_guard", 0))
        self.mesh, self.dirs, self.bands, self.disp, self.opt = m, d, b, disp, o


def bte_workspace_size(inst, **opts) -> int:
    lib = load_library()
    inp = _Inputs(inst, _resolve(inst, opts))
    n = C.c_size_t(0)
    _check(lib.bte_workspace_size(C.byref(inp.mesh), C.byref(inp.dirs), C.byref(inp.bands),
                                  C.byref(inp.opt), C.byref(n)))
    return int(n.value)


def _resolve(inst, opts: dict) -> dict:
    out = dict(dt=inst.dt, tol=inst.tol, max_inner=inst.max_inner, scheme=inst.scheme,
               precision=inst.precision, t_definition=inst.t_definition)
    out.update({k: v for k, v in opts.items() if v is not None})
    return out


class Solver:
    """One library context for an input instance, on a torch CUDA device."""

    def __init__(self, inst, device: str = "cuda:0", stream=None, **opts):
        import torch

        self.lib = load_library()
        self.inst = inst
        self.opts = _resolve(inst, opts)
        self.nc = int(np.prod(inst.n))
        self.nd = int(inst.s.shape[0])
        self.nb = int(inst.omega.shape[0])
        self.device = torch.device(device)
        inp = _Inputs(inst, self.opts)
        nbytes = C.c_size_t(0)
        _check(self.lib.bte_workspace_size(C.byref(inp.mesh), C.byref(inp.dirs),
                                           C.byref(inp.bands), C.byref(inp.opt),
                                           C.byref(nbytes)))
        self._ws_bytes = int(nbytes.value)
        self.workspace = torch.empty(self._ws_bytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise BteError(BTE_E_INVAL, "torch workspace is not 256-byte aligned")
        # a stream of its own unless one is given: the library captures inner
        # iterations as graphs, which the null stream cannot hold
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        inp.opt.stream = C.c_void_p(int(self.stream.cuda_stream))
        inp.opt.workspace = C.c_void_p(self.workspace.data_ptr())
        inp.opt.workspace_bytes = int(nbytes.value)
        self._ctx = C.c_void_p(0)
        _check(self.lib.bte_create(C.byref(inp.mesh), C.byref(inp.dirs), C.byref(inp.bands),
                                   C.byref(inp.disp), C.byref(inp.opt), C.byref(self._ctx)))

    @property
    def workspace_bytes(self) -> int:
        return self._ws_bytes

    def step(self, nsteps: int = 1, fixed_inner: Optional[List[int]] = None) -> List[dict]:
        st = (bte_step_stats * max(nsteps, 1))()
        fx = None
        if fixed_inner is not None:
            if len(fixed_inner) != nsteps:
                raise ValueError("fixed_inner needs one entry per step")
            fx = (C.c_int * nsteps)(*[int(v) for v in fixed_inner])
        _check(self.lib.bte_step(self._ctx, int(nsteps), fx, st))
        return [dict(inner=s.inner, converged=s.converged, newton_max=s.newton_max, res=s.res,
                     warm=s.warm, fallbacks=s.fallbacks, trained=s.trained, nn_loss=s.nn_loss)
                for s in st[:nsteps]]

    def temperature(self) -> np.ndarray:
        T = np.empty(self.nc)
        _check(self.lib.bte_temperature(self._ctx, T.ctypes.data_as(_dp), self.nc))
        return T

    def energy(self) -> np.ndarray:
        E = np.empty(self.nc)
        _check(self.lib.bte_energy(self._ctx, E.ctypes.data_as(_dp), self.nc))
        return E

    def intensity(self) -> np.ndarray:
        """Intensity at the current time level, FP64, shape [N_b, N_d, N_c]."""
        I = np.empty(self.nb * self.nd * self.nc)
        _check(self.lib.bte_intensity(self._ctx, I.ctypes.data_as(_dp), I.size))
        return I.reshape(self.nb, self.nd, self.nc)

    def set_fields(self, I: np.ndarray, T: np.ndarray):
        """Replaces the intensity [N_b, N_d, N_c] and temperature [N_c] of the
        current time level (T_{n-1} is set to T; E is recomputed)."""
        I = _f64(I).reshape(-1)
        T = _f64(T).reshape(-1)
        _check(self.lib.bte_set_fields(self._ctx, I.ctypes.data_as(_dp), I.size,
                                       T.ctypes.data_as(_dp), T.size))

    def set_wall_temperature(self, side: int, T_face):
        """New face temperatures of an isothermal wall for the next steps."""
        T = _f64(T_face).reshape(-1)
        _check(self.lib.bte_set_wall_temperature(self._ctx, int(side), T.ctypes.data_as(_dp),
                                                 T.size))

    def get_state(self) -> bytearray:
        """Checkpoint of everything the next steps depend on (bte_get_state)."""
        n = C.c_size_t(0)
        _check(self.lib.bte_state_size(self._ctx, C.byref(n)))
        buf = bytearray(n.value)
        cbuf = (C.c_char * len(buf)).from_buffer(buf)
        _check(self.lib.bte_get_state(self._ctx, C.cast(cbuf, C.c_void_p), len(buf)))
        return buf

    def set_state(self, state) -> None:
        """Restores a checkpoint taken by get_state (bte_set_state)."""
        buf = bytearray(state)
        cbuf = (C.c_char * len(buf)).from_buffer(buf)
        _check(self.lib.bte_set_state(self._ctx, C.cast(cbuf, C.c_void_p), len(buf)))

    # ---- learned warm start
    def nn_param_count(self) -> int:
        n = C.c_size_t(0)
        _check(self.lib.bte_nn_param_count(self._ctx, C.byref(n)))
        return int(n.value)

    def nn_params(self) -> np.ndarray:
        out = np.empty(self.nn_param_count(), dtype=np.float32)
        _check(self.lib.bte_nn_params(self._ctx, out.ctypes.data_as(C.POINTER(C.c_float)),
                                      out.size))
        return out

    def nn_set_params(self, vec):
        v = np.ascontiguousarray(vec, dtype=np.float32)
        _check(self.lib.bte_nn_set_params(self._ctx, v.ctypes.data_as(C.POINTER(C.c_float)),
                                          v.size))

    def nn_predict(self) -> np.ndarray:
        out = np.empty(self.nc)
        _check(self.lib.bte_nn_predict(self._ctx, out.ctypes.data_as(_dp), self.nc))
        return out

    def nn_gradient(self, T_n, T_prev, E_n, T_next):
        """(loss, gradient, outputs y) of the current network on one given sample."""
        arrs = [_f64(a).reshape(-1) for a in (T_n, T_prev, E_n, T_next)]
        g = np.empty(self.nn_param_count(), dtype=np.float32)
        y = np.empty(self.nc, dtype=np.float32)
        loss = C.c_double(0.0)
        fp = C.POINTER(C.c_float)
        _check(self.lib.bte_nn_gradient(self._ctx, *[a.ctypes.data_as(_dp) for a in arrs],
                                        self.nc, g.ctypes.data_as(fp), g.size, C.byref(loss),
                                        y.ctypes.data_as(fp)))
        return loss.value, g, y

    def autotune(self, cache_path: Optional[str] = None, ry: int = 0, rz: int = 0,
                 batch: bool = False):
        """Pick the fastest sweep layout for this shape (only layouts with ``ry`` rows
        / ``rz`` planes per wave where these are positive; only layouts a batch
        accepts with ``batch``); returns (ry, rz, direction groups, sweep ms)."""
        ry = -1 if batch else ry
        ry_, rz_, ndg, ms = C.c_int(int(ry)), C.c_int(int(rz)), C.c_int(0), C.c_double(0.0)
        _check(self.lib.bte_autotune(self._ctx, cache_path.encode() if cache_path else None,
                                     C.byref(ry_), C.byref(rz_), C.byref(ndg), C.byref(ms)))
        return ry_.value, rz_.value, ndg.value, ms.value

    def sweep_layout(self) -> dict:
        """The sweep layout in use: kernel family (0 cell per thread, 1 2D column
        walk, 2 3D column walk, 3 3D flattened plane), rows and planes per wave,
        direction groups."""
        v = [C.c_int(0) for _ in range(4)]
        _check(self.lib.bte_sweep_layout(self._ctx, *[C.byref(x) for x in v]))
        return dict(zip(("kind", "ry", "rz", "ndg"), (x.value for x in v)))

    def sweep_time(self):
        """(total ms, count) of sweep kernels timed since the last call."""
        ms = C.c_double(0.0)
        n = C.c_int(0)
        _check(self.lib.bte_sweep_time(self._ctx, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def close(self):
        """Destroys the context (it synchronises its stream) and releases the
        workspace tensor, so the memory can serve the next context at once."""
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self.lib.bte_destroy(self._ctx)
            self._ctx = C.c_void_p(0)
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def parse_state(buf) -> dict:
    """Splits a state written by bte_get_state into its header fields and
    numpy views of its sections (layout as documented in include/bte.h)."""
    h = bte_state_header.from_buffer_copy(bytes(buf[:C.sizeof(bte_state_header)]))
    nc = h.n[0] * h.n[1] * h.n[2]
    out = {name: getattr(h, name) for name, _ in bte_state_header._fields_
           if name not in ("magic", "n", "layout", "off")}
    out["n"] = list(h.n)
    out["layout"] = list(h.layout)
    mv = memoryview(bytes(buf))

    def sec(i, dtype, shape):
        if h.off[i] == 0:
            return None
        cnt = int(np.prod(shape))
        return np.frombuffer(mv, dtype=dtype, count=cnt, offset=h.off[i]).reshape(shape)

    real = np.float64 if h.precision == BTE_FP64 else np.float32
    out["I"] = sec(0, real, (h.nb, h.nd, nc))
    out["T"] = sec(1, np.float64, (nc,))
    out["T_prev"] = sec(2, np.float64, (nc,))
    out["E"] = sec(3, np.float64, (nc,))
    out["I0"] = sec(4, np.float64, (h.nb, nc))
    out["Iref"] = sec(5, np.float64, (h.nb,))
    out["plain_sweeps"] = sec(6, np.int32, (h.nn_rec,))
    out["params"] = sec(7, np.float32, (h.nn_params,))
    out["adam_m"] = sec(8, np.float32, (h.nn_params,))
    out["adam_v"] = sec(9, np.float32, (h.nn_params,))
    out["history"] = sec(10, np.float32, (h.nn_rec, 4, nc))
    return out


def _stats_dict(s) -> dict:
    return dict(inner=s.inner, converged=s.converged, newton_max=s.newton_max, res=s.res,
                warm=s.warm, fallbacks=s.fallbacks, trained=s.trained, nn_loss=s.nn_loss)


def batch_step_static(solvers, nsteps: int = 1):
    """Steps several Solvers (sharing one stream) together through
    bte_batch_step_static, which allocates nothing; returns stats[step][geometry]."""
    lib = load_library()
    n = len(solvers)
    arr = (C.c_void_p * n)(*[s._ctx.value for s in solvers])
    st = (bte_step_stats * max(1, nsteps * n))()
    _check(lib.bte_batch_step_static(n, arr, int(nsteps), st))
    return [[_stats_dict(st[k * n + i]) for i in range(n)] for k in range(nsteps)]


class Batch:
    """Steps several Solvers (sharing one stream) together: persistent sweep over
    all geometries, captured as a HIP graph per inner iteration."""

    def __init__(self, solvers, use_graph: bool = True):
        self.lib = load_library()
        self.solvers = list(solvers)
        n = len(self.solvers)
        arr = (C.c_void_p * n)(*[s._ctx.value for s in self.solvers])
        self._b = C.c_void_p(0)
        _check(self.lib.bte_batch_create(n, arr, int(bool(use_graph)), C.byref(self._b)))

    def step(self, nsteps: int = 1):
        """Returns stats[step][geometry]."""
        n = len(self.solvers)
        st = (bte_step_stats * max(1, nsteps * n))()
        _check(self.lib.bte_batch_step(self._b, int(nsteps), st))
        return [[_stats_dict(st[k * n + i]) for i in range(n)] for k in range(nsteps)]

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            self.lib.bte_batch_destroy(self._b)
            self._b = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
