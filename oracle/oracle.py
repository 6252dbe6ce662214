"""ctypes wrapper around the C oracle (``bte_oracle.c``) -- TEST INFRASTRUCTURE ONLY.

Takes an input instance (any object with the attributes produced by the seeded
input generator: dim, n, h, wall, wall_T, T_init, s, w, omega, domega, vg, tau,
dos, deg, dt, tol, max_inner, scheme, t_definition) and runs the plain FP64
reference time step.  Intensities are returned in the oracle's own storage
order [cell][direction][band].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bte_oracle.c")
_LIB = os.path.join(_HERE, "libbte_oracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class OracleError(RuntimeError):
    pass


class _Stats(C.Structure):
    _fields_ = [("inner", C.c_int), ("res", C.c_double), ("newton_max", C.c_int),
                ("energy", C.c_double)]


def oracle_lib_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, OpenMP, no FMA contraction, no fast-math."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build_oracle()
    lib = C.CDLL(_LIB)
    lib.oracle_create.restype = C.c_void_p
    lib.oracle_create.argtypes = [C.c_int, _ip, _dp, _ip, C.POINTER(_dp), _dp, C.c_int, _dp, _dp,
                                  C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, C.c_double,
                                  C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, C.c_char_p,
                                  C.c_int]
    lib.oracle_destroy.argtypes = [C.c_void_p]
    lib.oracle_step.argtypes = [C.c_void_p, C.c_int, C.POINTER(_Stats)]
    lib.oracle_step_warm.argtypes = [C.c_void_p, C.c_int, _dp, C.c_int, C.POINTER(_Stats)]
    lib.oracle_get_T.argtypes = [C.c_void_p, _dp]
    lib.oracle_get_I.argtypes = [C.c_void_p, _dp]
    lib.oracle_get_E.argtypes = [C.c_void_p, _dp, _dp]
    lib.oracle_set_state.argtypes = [C.c_void_p, _dp, _dp]
    lib.oracle_failed_cell.argtypes = [C.c_void_p]
    lib.oracle_set_wall_temperature.argtypes = [C.c_void_p, C.c_int, _dp]
    lib.oracle_set_threads.argtypes = [C.c_int]
    lib.oracle_get_threads.restype = C.c_int
    lib.oracle_equilibrium.restype = C.c_double
    lib.oracle_equilibrium.argtypes = [C.c_void_p, C.c_int, C.c_double]
    lib.oracle_invert_temperature.argtypes = [C.c_void_p, C.c_double, C.c_double, _dp, _ip]
    lib.oracle_invert_temperature_bands.argtypes = [C.c_void_p, _dp, C.c_double, _dp, _ip]
    lib.oracle_mirror_map.argtypes = [C.c_void_p, C.c_int, _ip]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


class Oracle:
    """One oracle context built from an input instance."""

    def __init__(self, inst, scheme=None, tol=None, max_inner=None, dt=None,
                 t_definition=None):
        lib = _load()
        self.lib = lib
        self.inst = inst
        self.nc = int(np.prod(inst.n))
        self.nd = int(inst.s.shape[0])
        self.nb = int(inst.omega.shape[0])
        keep = []

        def f64(a):
            a = np.ascontiguousarray(a, dtype=np.float64)
            keep.append(a)
            return a

        n = (C.c_int * 3)(*[int(v) for v in inst.n])
        h = (C.c_double * 3)(*[float(v) for v in inst.h])
        wall = (C.c_int * 6)(*[int(v) for v in inst.wall])
        wt = (_dp * 6)()
        for i in range(6):
            a = inst.wall_T[i]
            wt[i] = _ptr(f64(a)) if a is not None else _dp()
        tau_exp = getattr(inst, "tau_exp", None)
        tau_T0 = getattr(inst, "tau_T0", 300.0)
        err = C.create_string_buffer(256)
        self._h = lib.oracle_create(
            int(inst.dim), n, h, wall, wt, _ptr(f64(inst.T_init)), self.nd, _ptr(f64(inst.s)),
            _ptr(f64(inst.w)), self.nb, _ptr(f64(inst.omega)), _ptr(f64(inst.domega)),
            _ptr(f64(inst.vg)), _ptr(f64(inst.tau)), _ptr(f64(inst.dos)), _ptr(f64(inst.deg)),
            _ptr(f64(tau_exp)) if tau_exp is not None else _dp(), float(tau_T0),
            float(inst.dt if dt is None else dt), float(inst.tol if tol is None else tol),
            int(inst.max_inner if max_inner is None else max_inner),
            int(inst.scheme if scheme is None else scheme),
            int(inst.t_definition if t_definition is None else t_definition), err, 256)
        if not self._h:
            raise OracleError(err.value.decode())

    def close(self):
        if getattr(self, "_h", None):
            self.lib.oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def step(self, fixed_inner: int = 0):
        st = _Stats()
        rc = self.lib.oracle_step(self._h, int(fixed_inner), C.byref(st))
        if rc != 0:
            raise OracleError(f"oracle_step failed ({rc}), cell {self.lib.oracle_failed_cell(self._h)}")
        return dict(inner=st.inner, res=st.res, newton_max=st.newton_max, energy=st.energy)

    def step_warm(self, T0, shift: bool = False, fixed_inner: int = 0):
        """One implicit step whose inner iteration starts from temperature T0
        (and, with shift, from I^n moved by I0_b(T0) - I0_b(T_n))."""
        T0 = np.ascontiguousarray(T0, dtype=np.float64).reshape(-1)
        if T0.size != self.nc:
            raise OracleError("T0 size mismatch")
        st = _Stats()
        rc = self.lib.oracle_step_warm(self._h, int(fixed_inner), _ptr(T0), int(bool(shift)),
                                       C.byref(st))
        if rc != 0:
            raise OracleError(f"oracle_step_warm failed ({rc}), cell "
                              f"{self.lib.oracle_failed_cell(self._h)}")
        return dict(inner=st.inner, res=st.res, newton_max=st.newton_max, energy=st.energy)

    def run(self, nsteps: int, schedule=None):
        out = []
        for i in range(nsteps):
            out.append(self.step(0 if schedule is None else schedule[i]))
        return out

    def temperature(self) -> np.ndarray:
        T = np.empty(self.nc)
        self.lib.oracle_get_T(self._h, _ptr(T))
        return T

    def intensity(self) -> np.ndarray:
        """[N_c, N_d, N_b] (the oracle's storage order)."""
        I = np.empty(self.nc * self.nd * self.nb)
        self.lib.oracle_get_I(self._h, _ptr(I))
        return I.reshape(self.nc, self.nd, self.nb)

    def energy(self):
        E = np.empty(self.nc)
        G = np.empty(self.nc)
        self.lib.oracle_get_E(self._h, _ptr(E), _ptr(G))
        return E, G

    def set_state(self, I: np.ndarray, T: np.ndarray):
        I = np.ascontiguousarray(I, dtype=np.float64).reshape(-1)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
        if I.size != self.nc * self.nd * self.nb or T.size != self.nc:
            raise OracleError("state size mismatch")
        if self.lib.oracle_set_state(self._h, _ptr(I), _ptr(T)) != 0:
            raise OracleError("bad state")

    def set_wall_temperature(self, side: int, T_face):
        """New face temperatures of an isothermal wall for the next steps."""
        T_face = np.ascontiguousarray(T_face, dtype=np.float64)
        if self.lib.oracle_set_wall_temperature(self._h, int(side), _ptr(T_face)) != 0:
            raise OracleError("bad wall temperature")

    def equilibrium(self, b: int, T: float) -> float:
        return float(self.lib.oracle_equilibrium(self._h, int(b), float(T)))

    def invert_temperature(self, G: float, T_start: float):
        T = C.c_double(0.0)
        it = C.c_int(0)
        rc = self.lib.oracle_invert_temperature(self._h, float(G), float(T_start), C.byref(T),
                                                C.byref(it))
        if rc != 0:
            raise OracleError("Newton inversion failed")
        return T.value, it.value

    def invert_temperature_bands(self, e, T_start: float):
        """Temperature from per-band direction sums e_b with temperature-
        dependent relaxation times."""
        e = np.ascontiguousarray(e, dtype=np.float64)
        T = C.c_double(0.0)
        it = C.c_int(0)
        rc = self.lib.oracle_invert_temperature_bands(self._h, _ptr(e), float(T_start),
                                                      C.byref(T), C.byref(it))
        if rc != 0:
            raise OracleError("Newton inversion failed")
        return T.value, it.value

    def mirror_map(self, axis: int) -> np.ndarray:
        m = np.empty(self.nd, dtype=np.int32)
        self.lib.oracle_mirror_map(self._h, int(axis), m.ctypes.data_as(_ip))
        return m
