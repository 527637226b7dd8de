"""Python binding of the C ABI in include/mbx.h (ctypes; argument marshalling only).

Every computation runs in the HIP library libmbx.so built in this package
directory.  Loading fails loudly when the library is missing: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbx.so")

MBX_OK, MBX_EINVAL, MBX_ELABEL, MBX_ENEWTON, MBX_ENAN, MBX_ENOMEM, MBX_EBUDGET, MBX_EHIP, MBX_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
MBX_FP64, MBX_MIXED = 0, 1
ERR_NAMES = {0: "MBX_OK", -1: "MBX_EINVAL", -2: "MBX_ELABEL", -3: "MBX_ENEWTON", -4: "MBX_ENAN",
             -5: "MBX_ENOMEM", -6: "MBX_EBUDGET", -7: "MBX_EHIP", -8: "MBX_ESTATE"}

_d = ctypes.c_double
_i = ctypes.c_int
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class Params(ctypes.Structure):
    _fields_ = [("T", _d), ("I_app", _d), ("h", _d), ("c0", _d), ("x0", _d), ("y0", _d),
                ("De", _d), ("kappa", _d), ("tplus", _d), ("thermo", _d),
                ("Ds", _d * 2), ("sigma", _d * 2), ("cmax", _d * 2), ("i00", _d * 2),
                ("U0", _d * 2), ("U1", _d * 2), ("i00_pl", _d), ("n_c", _d),
                ("plating", _i), ("precision", _i), ("newton_tol", _d), ("res_tol", _d),
                ("krylov_rtol", _d), ("newton_max", _i), ("krylov_max", _i), ("V_cut", _d),
                ("graphs", _i), ("i00_ce", _d)]


class StepInfo(ctypes.Structure):
    _fields_ = [("newton_iters", _i), ("krylov_iters", _i), ("res0", _d), ("res_final", _d),
                ("du_final", _d), ("V", _d), ("wall_s", _d), ("substeps", _i)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", _i), ("steps_done", _i), ("V", _d), ("t_submit", _d), ("t_admit", _d),
                ("t_done", _d), ("newton_iters", ctypes.c_int64), ("krylov_iters", ctypes.c_int64),
                ("n_vox", ctypes.c_int64), ("n_an_faces", ctypes.c_int64), ("cutoff", _i), ("retried", _i),
                ("s_ac", _d * 2)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["s_ac"] = (self.s_ac[0], self.s_ac[1])
        return d


class ServerInfo(ctypes.Structure):
    _fields_ = [("steps_run", ctypes.c_int64), ("batches", ctypes.c_int64), ("busy_s", _d),
                ("bytes_in_use", ctypes.c_int64), ("running", _i), ("queued", _i)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


MBX_REQ_DONE, MBX_REQ_QUEUED, MBX_REQ_RUNNING = 0, 1, 2


class MbxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

# exported entry points: name -> (restype, argtypes)
SIGNATURES = {
    "mbx_params_default": (_i, [ctypes.POINTER(Params)]),
    "mbx_cell_create": (_i, [_vp, _i, _i, _i, ctypes.POINTER(Params), _vp, ctypes.POINTER(_vp)]),
    "mbx_cell_destroy": (None, [_vp]),
    "mbx_cell_step": (_i, [_vp, _d, ctypes.POINTER(StepInfo)]),
    "mbx_cell_set_current": (_i, [_vp, _d]),
    "mbx_cell_counts": (_i, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                             ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "mbx_cell_get_state": (_i, [_vp, _vp, _vp, _vp, _i]),
    "mbx_cell_set_state": (_i, [_vp, _vp, _vp, _vp, _i]),
    "mbx_cell_voltage": (_i, [_vp, _dp]),
    "mbx_cell_inventory": (_i, [_vp, _dp]),
    "mbx_cell_mean_solid": (_i, [_vp, _dp]),
    "mbx_cell_launch_shape": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "mbx_cell_run": (_i, [_vp, _d, _i, _dp, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "mbx_cell_run_adaptive": (_i, [_vp, _d, _d, _d, _d, _d, _i, _dp, _dp, ctypes.POINTER(_i), ctypes.POINTER(_i),
                                   ctypes.POINTER(_i)]),
    "mbx_cell_residual": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _d, _vp, _vp, _vp]),
    "mbx_cell_jvp": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _d, _vp, _vp]),
    "mbx_cell_precond": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _d, _vp, _vp]),
    "mbx_cell_solve": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _d, _vp, _d, _vp, ctypes.POINTER(_i)]),
    "mbx_batch_step": (_i, [ctypes.POINTER(_vp), _i, _d, ctypes.POINTER(_i), ctypes.POINTER(StepInfo)]),
    "mbx_cell_footprint": (ctypes.c_int64, [_i, _i, _i, _i, _i, _i]),
    "mbx_cell_capture": (_i, [_vp, _vp, _vp, ctypes.c_int64, _i]),
    "mbx_cell_captured": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "mbx_pod": (_i, [_vp, ctypes.c_int64, _i, ctypes.c_int64, _vp, _d, _i, _vp, ctypes.c_int64, _dp,
                     ctypes.POINTER(_i), _vp]),
    "mbx_pod_noalloc": (_i, [_vp, ctypes.c_int64, _i, ctypes.c_int64, _vp, _d, _i, _vp, ctypes.c_int64, _dp,
                             ctypes.POINTER(_i), _vp]),
    "mbx_sym_eig": (_i, [_i, _dp, _dp, _dp]),
    "mbx_last_error": (ctypes.c_char_p, []),
    "mbx_profile": (_i, [_i]),
    "mbx_profile_read": (_i, [ctypes.POINTER(ctypes.c_int64), _dp, _dp]),
    "mbx_server_create": (_i, [ctypes.c_int64, _i, _d, _i, _vp, ctypes.POINTER(_vp)]),
    "mbx_server_submit": (_i, [_vp, _vp, _i, _i, _i, ctypes.POINTER(Params), _i, ctypes.POINTER(ctypes.c_int64)]),
    "mbx_server_poll": (_i, [_vp, ctypes.c_int64, ctypes.POINTER(RequestInfo)]),
    "mbx_server_result": (_i, [_vp, ctypes.c_int64, _vp, _vp, _vp]),
    "mbx_server_error": (_i, [_vp, ctypes.c_int64, ctypes.c_char_p, _i]),
    "mbx_server_drain": (_i, [_vp, _d]),
    "mbx_server_clock": (_d, [_vp]),
    "mbx_server_stats": (_i, [_vp, ctypes.POINTER(ServerInfo)]),
    "mbx_server_destroy": (None, [_vp]),
}


def load(path: str = LIB_PATH):
    """Load libmbx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: run python -m paper_1704_04139_amd.build")
    # The library and PyTorch exchange device pointers and streams, so the
    # process must hold one HIP runtime.  PyTorch's wheel carries its own
    # libamdhip64 with the SONAME the library needs: importing torch first
    # binds the library to that copy.  Loaded the other way round, torch would
    # map a second runtime, and whichever initialises the GPU second fails.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code):
    if code != MBX_OK:
        raise MbxError(code, load().mbx_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_vp)


def make_params(cp, precision: str = "fp64", **knobs) -> Params:
    """Params from an inputs.CellParams (physical values) plus solver knobs."""
    lib = load()
    p = Params()
    _check(lib.mbx_params_default(ctypes.byref(p)))
    p.T, p.I_app, p.h, p.c0, p.x0, p.y0 = cp.T, cp.I_app, cp.h, cp.c0, cp.x0, cp.y0
    p.De, p.kappa, p.tplus, p.thermo = cp.De, cp.kappa, cp.tplus, cp.thermo
    p.Ds[0], p.Ds[1] = cp.Ds_an, cp.Ds_ca
    p.sigma[0], p.sigma[1] = cp.sigma_an, cp.sigma_ca
    p.cmax[0], p.cmax[1] = cp.cmax_an, cp.cmax_ca
    p.i00[0], p.i00[1] = cp.i00_an, cp.i00_ca
    p.U0[0], p.U1[0] = cp.U_an
    p.U0[1], p.U1[1] = cp.U_ca
    p.i00_pl, p.n_c, p.plating = cp.i00_pl, cp.n_c, int(cp.plating)
    p.i00_ce = getattr(cp, "i00_ce", 0.0)
    p.precision = MBX_MIXED if precision == "mixed" else MBX_FP64
    for k, v in knobs.items():
        setattr(p, k, v)
    return p


@dataclass
class Counts:
    n_vox: int
    n_an_faces: int
    n_ca_faces: int
    n_top: int


class Cell:
    """One cell on the GPU (owns its device memory)."""

    def __init__(self, labels: np.ndarray, params, precision: str = "fp64", stream=None, **knobs):
        lib = load()
        lab = np.ascontiguousarray(labels, dtype=np.uint8)
        nz, ny, nx = lab.shape
        self.shape = (nx, ny, nz)
        self.params = params if isinstance(params, Params) else make_params(params, precision, **knobs)
        h = _vp()
        s = _vp(stream) if stream else None
        _check(lib.mbx_cell_create(_ptr(lab), nx, ny, nz, ctypes.byref(self.params), s, ctypes.byref(h)))
        self._h = h
        self.counts = self._counts()

    def _counts(self) -> Counts:
        a, b, c, d = (ctypes.c_int64() for _ in range(4))
        _check(load().mbx_cell_counts(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        return Counts(a.value, b.value, c.value, d.value)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().mbx_cell_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, dt: float) -> dict:
        info = StepInfo()
        _check(load().mbx_cell_step(self._h, float(dt), ctypes.byref(info)))
        return info.as_dict()

    def try_step(self, dt: float):
        """Step without raising: returns (code, info dict)."""
        info = StepInfo()
        code = load().mbx_cell_step(self._h, float(dt), ctypes.byref(info))
        return code, info.as_dict()

    def set_current(self, I_app: float):
        _check(load().mbx_cell_set_current(self._h, float(I_app)))

    def get_state(self):
        c = np.empty(self.counts.n_vox)
        p = np.empty(self.counts.n_vox)
        n = np.empty(self.counts.n_an_faces)
        _check(load().mbx_cell_get_state(self._h, _ptr(c), _ptr(p), _ptr(n), 0))
        return c, p, n

    def get_state_device(self, c_ptr: int, p_ptr: int, n_ptr: int):
        _check(load().mbx_cell_get_state(self._h, _vp(c_ptr), _vp(p_ptr), _vp(n_ptr), 1))

    def capture(self, c_ptr: int, p_ptr: int, ld: int, capacity: int):
        """Snapshot capture into caller-owned device columns (0 pointers skip a field)."""
        _check(load().mbx_cell_capture(self._h, _vp(c_ptr) if c_ptr else None, _vp(p_ptr) if p_ptr else None,
                                       int(ld), int(capacity)))

    def captured(self):
        """(columns written, columns dropped for lack of room)."""
        a, b = _i(), _i()
        _check(load().mbx_cell_captured(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_state(self, c, p, n):
        c, p, n = (np.ascontiguousarray(a, dtype=np.float64) for a in (c, p, n))
        _check(load().mbx_cell_set_state(self._h, _ptr(c), _ptr(p), _ptr(n), 0))

    def voltage(self) -> float:
        v = ctypes.c_double()
        _check(load().mbx_cell_voltage(self._h, ctypes.byref(v)))
        return v.value

    def inventory(self):
        out = (ctypes.c_double * 4)()
        _check(load().mbx_cell_inventory(self._h, out))
        return {"electrolyte": out[0], "anode": out[1], "cathode": out[2], "plated": out[3]}

    def mean_solid(self):
        """s_ac: mean solid concentration of the anode and the cathode, mol/m^3."""
        out = (ctypes.c_double * 2)()
        _check(load().mbx_cell_mean_solid(self._h, out))
        return out[0], out[1]

    def launch_shape(self):
        """(level-0 smoother, J*v) workgroup sizes the library's tuner picked for this cell."""
        a, b = _i(), _i()
        _check(load().mbx_cell_launch_shape(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def run(self, dt: float, max_steps: int):
        """Step loop with the voltage cutoff params.V_cut: returns
        (V after each step taken, cutoff fired, steps retried as half steps)."""
        V = np.empty(max(int(max_steps), 1))
        n, cut, ret = _i(), _i(), _i()
        _check(load().mbx_cell_run(self._h, float(dt), int(max_steps), V.ctypes.data_as(_dp), ctypes.byref(n),
                                   ctypes.byref(cut), ctypes.byref(ret)))
        return V[:n.value].copy(), bool(cut.value), ret.value

    def run_adaptive(self, t_end: float, dt0: float, dt_min: float, dt_max: float, tol: float,
                     max_steps: int = 10000):
        """Adaptive implicit Euler to t_end with factor-of-2 step control:
        returns (times, voltages after each accepted step, rejected steps,
        cutoff fired)."""
        k = max(int(max_steps), 1)
        t, V = np.empty(k), np.empty(k)
        n, rej, cut = _i(), _i(), _i()
        _check(load().mbx_cell_run_adaptive(self._h, float(t_end), float(dt0), float(dt_min), float(dt_max),
                                            float(tol), int(max_steps), t.ctypes.data_as(_dp),
                                            V.ctypes.data_as(_dp), ctypes.byref(n), ctypes.byref(rej),
                                            ctypes.byref(cut)))
        return t[:n.value].copy(), V[:n.value].copy(), rej.value, bool(cut.value)

    def residual(self, c, p, n, c_old, n_old, dt):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (c, p, n, c_old, n_old)]
        Rc = np.empty(self.counts.n_vox)
        Rp = np.empty(self.counts.n_vox)
        Rn = np.empty(self.counts.n_an_faces)
        _check(load().mbx_cell_residual(self._h, *[_ptr(a) for a in arrs], float(dt), _ptr(Rc), _ptr(Rp), _ptr(Rn)))
        return Rc, Rp, Rn

    def jvp(self, c, p, n, c_old, n_old, dt, v):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (c, p, n, c_old, n_old)]
        v = np.ascontiguousarray(v, dtype=np.float64)
        y = np.empty(2 * self.counts.n_vox)
        _check(load().mbx_cell_jvp(self._h, *[_ptr(a) for a in arrs], float(dt), _ptr(v), _ptr(y)))
        return y


def _probe(fn, cell, c, p, n, c_old, n_old, dt, v):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (c, p, n, c_old, n_old)]
    v = np.ascontiguousarray(v, dtype=np.float64)
    y = np.empty(2 * cell.counts.n_vox)
    _check(fn(cell.handle, *[_ptr(a) for a in arrs], float(dt), _ptr(v), _ptr(y)))
    return y


def precond(cell, c, p, n, c_old, n_old, dt, v):
    """z = M^-1 v with the solver's preconditioner at the given state."""
    return _probe(load().mbx_cell_precond, cell, c, p, n, c_old, n_old, dt, v)


def solve(cell, c, p, n, c_old, n_old, dt, rhs, rtol):
    """x with J_hat x = rhs by the solver's GMRES; returns (x, iterations)."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (c, p, n, c_old, n_old)]
    rhs = np.ascontiguousarray(rhs, dtype=np.float64)
    x = np.empty(2 * cell.counts.n_vox)
    its = _i()
    _check(load().mbx_cell_solve(cell.handle, *[_ptr(a) for a in arrs], float(dt), _ptr(rhs), float(rtol),
                                 _ptr(x), ctypes.byref(its)))
    return x, its.value


def batch_step(cells, dt: float):
    """Step several cells in shared launches; returns (status list, info dicts)."""
    lib = load()
    n = len(cells)
    hs = (_vp * n)(*[c.handle.value for c in cells])
    st = (_i * n)()
    infos = (StepInfo * n)()
    _check(lib.mbx_batch_step(hs, n, float(dt), st, infos))
    return list(st), [infos[k].as_dict() for k in range(n)]


def pod(S_ptr: int, n: int, m: int, lds: int, modes_ptr: int, ldm: int, k_max: int, rtol: float = 1e-7,
        w_ptr: int = 0, stream=None, noalloc: bool = False):
    """POD of the n x m device snapshots at S_ptr into the device modes at
    modes_ptr (column-major); returns (sigma: all m singular values, k).
    noalloc=True calls mbx_pod_noalloc (static device workspace)."""
    sigma = np.empty(m)
    k = _i()
    fn = load().mbx_pod_noalloc if noalloc else load().mbx_pod
    _check(fn(_vp(S_ptr), int(n), int(m), int(lds), _vp(w_ptr) if w_ptr else None, float(rtol),
                          int(k_max), _vp(modes_ptr), int(ldm), sigma.ctypes.data_as(_dp), ctypes.byref(k),
                          _vp(stream) if stream else None))
    return sigma, k.value


def sym_eig(A: np.ndarray):
    """Eigenvalues (descending) and eigenvectors of a symmetric matrix (host)."""
    A = np.asfortranarray(A, dtype=np.float64)
    m = A.shape[0]
    lam = np.empty(m)
    V = np.empty((m, m), order="F")
    _check(load().mbx_sym_eig(m, A.ctypes.data_as(_dp), lam.ctypes.data_as(_dp), V.ctypes.data_as(_dp)))
    return lam, V


PROFILE_KERNELS = {"residual": 1, "matvec": 2, "smooth0": 3, "precond": 4, "gram": 5}


def profile(kernel):
    """Start timing launches of one kernel class (name or id; None stops)."""
    k = 0 if kernel is None else PROFILE_KERNELS.get(kernel, kernel)
    _check(load().mbx_profile(int(k)))


def profile_read():
    """(launches, total ms, total algorithmic bytes) of the timed launches."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(load().mbx_profile_read(ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    return n.value, ms.value, by.value


def footprint(nx, ny, nz, precision="fp64", n_an_faces=0, n_ca_faces=0) -> int:
    return int(load().mbx_cell_footprint(nx, ny, nz, MBX_MIXED if precision == "mixed" else MBX_FP64,
                                         n_an_faces, n_ca_faces))


class Server:
    """Continuous-batching step server (worker thread in the library)."""

    def __init__(self, budget_bytes: int, precision: str, dt: float, keep_state: bool = False, stream=None):
        lib = load()
        h = _vp()
        prec = MBX_MIXED if precision == "mixed" else MBX_FP64
        _check(lib.mbx_server_create(int(budget_bytes), prec, float(dt), int(keep_state),
                                     _vp(stream) if stream else None, ctypes.byref(h)))
        self._h = h
        self.precision = precision

    def submit(self, labels: np.ndarray, params, n_steps: int, **knobs) -> int:
        lab = np.ascontiguousarray(labels, dtype=np.uint8)
        nz, ny, nx = lab.shape
        p = params if isinstance(params, Params) else make_params(params, self.precision, **knobs)
        rid = ctypes.c_int64()
        _check(load().mbx_server_submit(self._h, _ptr(lab), nx, ny, nz, ctypes.byref(p), int(n_steps),
                                        ctypes.byref(rid)))
        return rid.value

    def poll(self, rid: int) -> dict:
        info = RequestInfo()
        _check(load().mbx_server_poll(self._h, int(rid), ctypes.byref(info)))
        return info.as_dict()

    def error(self, rid: int) -> str:
        """Error message of a request that failed ('' otherwise)."""
        buf = ctypes.create_string_buffer(512)
        _check(load().mbx_server_error(self._h, int(rid), buf, len(buf)))
        return buf.value.decode(errors="replace")

    def result(self, rid: int):
        """Final (c, phi, n) of a finished request (keep_state servers)."""
        info = self.poll(rid)
        N, n_an = int(info["n_vox"]), int(info["n_an_faces"])
        c, phi, n = np.empty(N), np.empty(N), np.empty(n_an)
        _check(load().mbx_server_result(self._h, int(rid), _ptr(c), _ptr(phi), _ptr(n) if n_an else None))
        return c, phi, n

    def drain(self, timeout_s: float = 600.0):
        _check(load().mbx_server_drain(self._h, float(timeout_s)))

    def clock(self) -> float:
        return load().mbx_server_clock(self._h)

    def stats(self) -> dict:
        info = ServerInfo()
        _check(load().mbx_server_stats(self._h, ctypes.byref(info)))
        return info.as_dict()

    def close(self):
        if self._h:
            load().mbx_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
