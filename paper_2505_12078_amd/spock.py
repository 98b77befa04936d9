"""Thin ctypes binding of the C ABI in include/spock.h (argument marshalling only).

Every step of the CP iteration runs in the gfx950 library; this module only
converts NumPy arrays to pointers.  It fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libspock_mi355x.so")

SPOCK_OK = 0
SPOCK_E_INVALID = -1
SPOCK_E_INFEASIBLE_X0 = -2
SPOCK_E_NOT_CONVERGED = -3
SPOCK_E_DIVERGED = -4
SPOCK_E_HIP = -5
SPOCK_E_CAPACITY = -6
SPOCK_E_NOMEM = -7
FP64, MIXED, FP32 = 0, 1, 2
CP, SUPERMANN = 0, 1

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class ProblemDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("parent", _ip), ("cond_prob", _dp), ("nx", C.c_int32),
                ("nu", C.c_int32), ("A", _dp), ("B", _dp), ("c", _dp), ("Q_diag", _dp), ("R_diag", _dp),
                ("QN_diag", _dp), ("x_lo", _dp), ("x_hi", _dp), ("u_lo", _dp), ("u_hi", _dp),
                ("xN_lo", _dp), ("xN_hi", _dp), ("x_ball", C.c_double), ("xN_ball", C.c_double),
                ("gamma", _dp), ("q", _dp), ("r", _dp), ("qN", _dp), ("Q_edge", _dp), ("R_edge", _dp),
                ("QN_leaf", _dp), ("Q_dense", _dp), ("R_dense", _dp), ("QN_dense", _dp),
                ("n_con", C.c_int32), ("Gamma", _dp), ("con_lo", _dp), ("con_hi", _dp),
                ("n_conN", C.c_int32), ("GammaN", _dp), ("conN_lo", _dp), ("conN_hi", _dp),
                ("risk_ny", _ip), ("risk_nnu", _ip), ("risk_E", _dp), ("risk_F", _dp), ("risk_b", _dp),
                ("risk_cone", _ip)]


class Settings(C.Structure):
    _fields_ = [("alpha", C.c_double), ("eps", C.c_double), ("max_iters", C.c_int64),
                ("precision", C.c_int32), ("precondition", C.c_int32), ("check_every", C.c_int32),
                ("use_graph", C.c_int32), ("method", C.c_int32), ("aa_memory", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int64), ("iters_fp32", C.c_int64), ("rel_res", C.c_double),
                ("xi1_inf", C.c_double), ("xi2_inf", C.c_double), ("s0", C.c_double),
                ("t_setup_s", C.c_double), ("t_solve_s", C.c_double), ("status", C.c_int32), ("precision_used", C.c_int32),
                ("refined", C.c_int32), ("n_T", C.c_int64), ("n_K0", C.c_int64), ("n_K1", C.c_int64),
                ("n_K2", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Sizes(C.Structure):
    _fields_ = [("nz", C.c_int64), ("neta", C.c_int64), ("n", C.c_int32), ("n_nl", C.c_int32),
                ("n_leaf", C.c_int32), ("N", C.c_int32), ("nx", C.c_int32), ("nu", C.c_int32),
                ("nc", C.c_int32), ("ncN", C.c_int32), ("max_children", C.c_int32),
                ("alpha", C.c_double), ("L_norm", C.c_double), ("device_bytes", C.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Result(C.Structure):
    _fields_ = [("req_id", C.c_uint64), ("tree_id", C.c_int64), ("status", C.c_int32), ("warm", C.c_int32),
                ("info", Info), ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "info"}
        d["info"] = self.info.as_dict()
        return d


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("created", C.c_uint64),
                ("evicted", C.c_uint64), ("ticks", C.c_uint64), ("resident_bytes", C.c_size_t),
                ("budget_bytes", C.c_size_t), ("pending", C.c_size_t), ("in_flight", C.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes); the exported surface of include/spock.h
SIGNATURES = {
    "spock_last_error": (C.c_char_p, []),
    "spock_default_settings": (C.c_int32, [C.POINTER(Settings)]),
    "spock_problem_footprint": (C.c_int32, [C.POINTER(ProblemDesc), C.POINTER(Settings), C.POINTER(C.c_size_t)]),
    "spock_problem_create": (C.c_int32, [C.POINTER(ProblemDesc), C.POINTER(Settings), C.c_void_p, C.c_size_t,
                                         C.c_void_p, C.POINTER(C.c_void_p)]),
    "spock_problem_destroy": (C.c_int32, [C.c_void_p]),
    "spock_problem_sizes": (C.c_int32, [C.c_void_p, C.POINTER(Sizes)]),
    "spock_set_settings": (C.c_int32, [C.c_void_p, C.POINTER(Settings)]),
    "spock_solve": (C.c_int32, [C.c_void_p, _dp, C.c_int32, C.POINTER(Info)]),
    "spock_get_solution": (C.c_int32, [C.c_void_p, _dp, _dp, _dp]),
    "spock_get_iterate": (C.c_int32, [C.c_void_p, _dp, _dp]),
    "spock_set_iterate": (C.c_int32, [C.c_void_p, _dp, _dp]),
    "spock_set_x0": (C.c_int32, [C.c_void_p, _dp]),
    "spock_apply_T": (C.c_int32, [C.c_void_p, _dp, _dp, _dp, _dp, C.c_int32, _dp]),
    "spock_apply_L": (C.c_int32, [C.c_void_p, _dp, _dp, C.c_int32]),
    "spock_apply_T_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_int32, _dp]),
    "spock_project_S1": (C.c_int32, [C.c_void_p, _dp, _dp, _dp, _dp, C.c_int32]),
    "spock_project_S2": (C.c_int32, [C.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, C.c_int32]),
    "spock_apply_Lt": (C.c_int32, [C.c_void_p, _dp, _dp, C.c_int32]),
    "spock_prox_gconj": (C.c_int32, [C.c_void_p, _dp, _dp, C.c_int32]),
    "spock_time_steps": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, _dp, _dp, _dp]),
    "spock_step_bytes": (C.c_int32, [C.c_void_p, C.c_int32, _dp, _dp]),
    "spock_time_kernels": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, _dp, _dp]),
    "spock_kernel_bytes": (C.c_int32, [C.c_void_p, C.c_int32, _dp]),
    "spock_run_steps": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]),
    "spock_set_launch": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32]),
    "spock_get_launch": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "spock_batch_set_launch": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32]),
    "spock_batch_create": (C.c_int32, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(Settings),
                                       C.POINTER(C.c_void_p)]),
    "spock_batch_destroy": (C.c_int32, [C.c_void_p]),
    "spock_batch_size": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_size_t)]),
    "spock_batch_solve": (C.c_int32, [C.c_void_p, C.POINTER(_dp), _ip, C.POINTER(Info)]),
    "spock_batch_run_steps": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]),
    "spock_batch_time_steps": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, _dp, _dp, _dp]),
    "spock_batch_step_bytes": (C.c_int32, [C.c_void_p, C.c_int32, _dp, _dp]),
    "spock_batch_time_kernels": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, _dp, _dp]),
    "spock_batch_kernel_bytes": (C.c_int32, [C.c_void_p, C.c_int32, _dp]),
    "spock_server_create": (C.c_int32, [C.c_size_t, C.POINTER(Settings), C.POINTER(C.c_void_p)]),
    "spock_server_add_tree": (C.c_int32, [C.c_void_p, C.POINTER(ProblemDesc), C.POINTER(C.c_int64)]),
    "spock_server_submit": (C.c_int32, [C.c_void_p, C.c_int64, _dp, C.c_uint64]),
    "spock_server_poll": (C.c_int32, [C.c_void_p, C.POINTER(Result), C.c_int32, C.POINTER(C.c_int32)]),
    "spock_server_wait_idle": (C.c_int32, [C.c_void_p, C.c_double]),
    "spock_server_get_stats": (C.c_int32, [C.c_void_p, C.POINTER(ServerStats)]),
    "spock_server_solution": (C.c_int32, [C.c_void_p, C.c_int64, _dp, _dp, _dp]),
    "spock_server_destroy": (C.c_int32, [C.c_void_p]),
    "spock_now": (C.c_double, []),
}

_lib = None


def load(path=None):
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    path = path or LIB_PATH
    # PyTorch bundles its own HIP runtime under the same soname; loading it
    # first makes this library bind to that one runtime instead of a second
    # copy (two runtimes in one process cannot share the device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError("HIP library not built: %s is missing (run __graft_entry__.build())" % path)
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class SpockError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("spock error %d: %s" % (code, msg))
        self.code = code


def _check(code, allow=()):
    if code != SPOCK_OK and code not in allow:
        raise SpockError(code, load().spock_last_error().decode())
    return code


def _ptr(a, dtype=np.float64):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double if dtype == np.float64 else C.c_int32))


def default_settings(**kw):
    s = Settings()
    _check(load().spock_default_settings(C.byref(s)))
    for k, v in kw.items():
        setattr(s, k, v)
    return s


class _Desc:
    """Keeps the NumPy buffers of a ProblemDesc alive."""

    def __init__(self, prob):
        f = lambda k: np.ascontiguousarray(prob[k], dtype=np.float64)
        self.keep = {
            "parent": np.ascontiguousarray(prob["parent"], dtype=np.int32),
            "prob": f("prob"), "A": f("A"), "B": f("B"),
            "c": None if prob.get("c") is None else f("c"),
            "Q": f("Q"), "R": f("R"), "QN": f("QN"), "x_lo": f("x_lo"), "x_hi": f("x_hi"),
            "u_lo": f("u_lo"), "u_hi": f("u_hi"), "xN_lo": f("xN_lo"), "xN_hi": f("xN_hi"),
            "gamma": f("gamma"),
            "q": None if prob.get("q") is None else f("q"),
            "r": None if prob.get("r") is None else f("r"),
            "qN": None if prob.get("qN") is None else f("qN"),
        }
        k = self.keep
        self.desc = ProblemDesc(
            n_nodes=len(k["parent"]), parent=_ptr(k["parent"], np.int32), cond_prob=_ptr(k["prob"]),
            nx=int(prob["nx"]), nu=int(prob["nu"]), A=_ptr(k["A"]), B=_ptr(k["B"]), c=_ptr(k["c"]),
            Q_diag=_ptr(k["Q"]), R_diag=_ptr(k["R"]), QN_diag=_ptr(k["QN"]), x_lo=_ptr(k["x_lo"]),
            x_hi=_ptr(k["x_hi"]), u_lo=_ptr(k["u_lo"]), u_hi=_ptr(k["u_hi"]), xN_lo=_ptr(k["xN_lo"]),
            xN_hi=_ptr(k["xN_hi"]), x_ball=float(prob["x_ball"]), xN_ball=float(prob["xN_ball"]),
            gamma=_ptr(k["gamma"]), q=_ptr(k["q"]), r=_ptr(k["r"]), qN=_ptr(k["qN"]))
        # cost diagonals given per edge / per leaf (one row per node), or
        # dense matrices per edge / per leaf (one matrix per node)
        for key, shared, per, dense in (("Q", "Q_diag", "Q_edge", "Q_dense"), ("R", "R_diag", "R_edge", "R_dense"),
                                        ("QN", "QN_diag", "QN_leaf", "QN_dense")):
            if k[key].ndim == 2:
                setattr(self.desc, shared, None)
                setattr(self.desc, per, _ptr(k[key]))
            elif k[key].ndim == 3:
                setattr(self.desc, shared, None)
                setattr(self.desc, dense, _ptr(k[key]))
        # general constraint rows (Gamma = [Gamma_x | Gamma_u]) and leaf rows
        if prob.get("Gamma_x") is not None:
            k["Gamma"] = np.ascontiguousarray(np.hstack([prob["Gamma_x"], prob["Gamma_u"]]), dtype=np.float64)
            k["con_lo"], k["con_hi"] = f("c_lo"), f("c_hi")
            self.desc.n_con = k["Gamma"].shape[0]
            self.desc.Gamma, self.desc.con_lo, self.desc.con_hi = _ptr(k["Gamma"]), _ptr(k["con_lo"]), _ptr(k["con_hi"])
        if prob.get("Gamma_N") is not None:
            k["GammaN"] = f("Gamma_N")
            k["conN_lo"], k["conN_hi"] = f("cN_lo"), f("cN_hi")
            self.desc.n_conN = k["GammaN"].shape[0]
            self.desc.GammaN = _ptr(k["GammaN"])
            self.desc.conN_lo, self.desc.conN_hi = _ptr(k["conN_lo"]), _ptr(k["conN_hi"])
        # general coherent risks: per non-leaf node (E, F, b, cone codes),
        # concatenated in node order
        if prob.get("risk") is not None:
            risk = prob["risk"]
            cat = lambda parts, dt: np.ascontiguousarray(np.concatenate([np.ravel(a) for a in parts]) if parts
                                                         else np.zeros(0), dtype=dt)
            k["risk_ny"] = np.ascontiguousarray([len(r[2]) for r in risk], dtype=np.int32)
            k["risk_nnu"] = np.ascontiguousarray([0 if r[1] is None else np.shape(r[1])[1] for r in risk],
                                                 dtype=np.int32)
            k["risk_E"] = cat([r[0] for r in risk], np.float64)
            k["risk_F"] = cat([r[1] for r in risk if r[1] is not None], np.float64)
            k["risk_b"] = cat([r[2] for r in risk], np.float64)
            k["risk_cone"] = cat([r[3] for r in risk], np.int32)
            self.desc.risk_ny, self.desc.risk_nnu = _ptr(k["risk_ny"], np.int32), _ptr(k["risk_nnu"], np.int32)
            self.desc.risk_E, self.desc.risk_b = _ptr(k["risk_E"]), _ptr(k["risk_b"])
            self.desc.risk_F = _ptr(k["risk_F"]) if k["risk_F"].size else None
            self.desc.risk_cone = _ptr(k["risk_cone"], np.int32)


def footprint(prob, settings=None):
    d = _Desc(prob)
    s = settings or default_settings()
    out = C.c_size_t(0)
    _check(load().spock_problem_footprint(C.byref(d.desc), C.byref(s), C.byref(out)))
    return int(out.value)


class Problem:
    """One scenario-tree problem resident on the current HIP device."""

    def __init__(self, prob, settings=None, workspace=None, stream=None, **kw):
        lib = load()
        self.settings = settings or default_settings(**kw)
        d = _Desc(prob)
        h = C.c_void_p()
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:  # e.g. a torch uint8 device tensor
            ws_ptr, ws_bytes = C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
            self._ws = workspace
        st = None if stream is None else C.c_void_p(stream)
        _check(lib.spock_problem_create(C.byref(d.desc), C.byref(self.settings), ws_ptr, ws_bytes, st,
                                        C.byref(h)))
        self.h = h
        self._lib = lib
        sz = Sizes()
        _check(lib.spock_problem_sizes(h, C.byref(sz)))
        self.sizes = sz.as_dict()
        self.nz, self.neta = sz.nz, sz.neta
        self.n, self.n_nl, self.nx, self.nu = sz.n, sz.n_nl, sz.nx, sz.nu
        self.alpha = sz.alpha

    def close(self):
        if getattr(self, "h", None):
            self._lib.spock_problem_destroy(self.h)
            self.h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_settings(self, **kw):
        for k, v in kw.items():
            setattr(self.settings, k, v)
        _check(load().spock_set_settings(self.h, C.byref(self.settings)))

    def solve(self, x0, warm_start=False, raise_on_failure=False):
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        info = Info()
        code = load().spock_solve(self.h, _ptr(x0), int(bool(warm_start)), C.byref(info))
        allow = () if raise_on_failure else (SPOCK_E_NOT_CONVERGED, SPOCK_E_DIVERGED)
        _check(code, allow)
        out = info.as_dict()
        out["code"] = code
        return out

    def solution(self):
        x = np.zeros((self.n, self.nx))
        u = np.zeros((self.n_nl, self.nu))
        s0 = C.c_double(0)
        _check(load().spock_get_solution(self.h, _ptr(x), _ptr(u), C.byref(s0)))
        return x, u, s0.value

    def get_iterate(self):
        z, e = np.zeros(self.nz), np.zeros(self.neta)
        _check(load().spock_get_iterate(self.h, _ptr(z), _ptr(e)))
        return z, e

    def set_iterate(self, z, eta):
        z = np.ascontiguousarray(z, dtype=np.float64)
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        _check(load().spock_set_iterate(self.h, _ptr(z), _ptr(eta)))

    def set_x0(self, x0):
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        _check(load().spock_set_x0(self.h, _ptr(x0)))

    def apply_T(self, z, eta, precision=FP64):
        z = np.ascontiguousarray(z, dtype=np.float64)
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        zo, eo, xi = np.zeros(self.nz), np.zeros(self.neta), np.zeros(2)
        _check(load().spock_apply_T(self.h, _ptr(z), _ptr(eta), _ptr(zo), _ptr(eo), precision, _ptr(xi)))
        return zo, eo, xi

    def project_S1(self, xbar, ubar, precision=FP64):
        xbar = np.ascontiguousarray(xbar, dtype=np.float64).reshape(self.n, self.nx)
        ubar = np.ascontiguousarray(ubar, dtype=np.float64).reshape(self.n_nl, self.nu)
        x, u = np.zeros((self.n, self.nx)), np.zeros((self.n_nl, self.nu))
        _check(load().spock_project_S1(self.h, _ptr(xbar), _ptr(ubar), _ptr(x), _ptr(u), precision))
        return x, u

    def project_S2(self, y, tau, s, precision=FP64):
        y, tau, s = (np.ascontiguousarray(a, dtype=np.float64) for a in (y, tau, s))
        if tau.size != self.n - 1 or s.size != self.n - 1:
            raise ValueError("tau and s have one entry per node 1..n-1")
        if y.size != self.nz - 1 - self.n * self.nx - self.n_nl * self.nu - 2 * (self.n - 1):
            raise ValueError("y must hold one entry per row of every non-leaf node's risk (2 n_ch(i) + 1 for AV@R)")
        yo, to, so = np.zeros_like(y), np.zeros_like(tau), np.zeros_like(s)
        _check(load().spock_project_S2(self.h, _ptr(y), _ptr(tau), _ptr(s), _ptr(yo), _ptr(to), _ptr(so),
                                       precision))
        return yo, to, so

    def apply_T_noalloc(self, z_dev, eta_dev, z_out_dev, eta_out_dev, precision=FP64):
        """One CP step on device buffers given as integer addresses (e.g. a
        torch tensor's data_ptr()); scratch in the library's static array."""
        xi = np.zeros(2)
        _check(load().spock_apply_T_noalloc(self.h, C.c_void_p(z_dev), C.c_void_p(eta_dev), C.c_void_p(z_out_dev),
                                            C.c_void_p(eta_out_dev), precision, _ptr(xi)))
        return xi

    def apply_L(self, z, precision=FP64):
        z = np.ascontiguousarray(z, dtype=np.float64)
        out = np.zeros(self.neta)
        _check(load().spock_apply_L(self.h, _ptr(z), _ptr(out), precision))
        return out

    def apply_Lt(self, eta, precision=FP64):
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        out = np.zeros(self.nz)
        _check(load().spock_apply_Lt(self.h, _ptr(eta), _ptr(out), precision))
        return out

    def prox_gconj(self, w, precision=FP64):
        w = np.ascontiguousarray(w, dtype=np.float64)
        out = np.zeros(self.neta)
        _check(load().spock_prox_gconj(self.h, _ptr(w), _ptr(out), precision))
        return out

    def time_steps(self, steps, precision=FP64):
        t, b, f = C.c_double(), C.c_double(), C.c_double()
        _check(load().spock_time_steps(self.h, precision, int(steps), C.byref(t), C.byref(b), C.byref(f)))
        return t.value, b.value, f.value

    def run_steps(self, steps, precision=FP64, sync=True):
        _check(load().spock_run_steps(self.h, precision, int(steps), int(bool(sync))))

    def set_launch(self, workgroup, precision=FP64):
        _check(load().spock_set_launch(self.h, precision, int(workgroup)))

    def get_launch(self, precision=FP64):
        v = C.c_int32()
        _check(load().spock_get_launch(self.h, precision, C.byref(v)))
        return v.value

    def time_kernels(self, steps, precision=FP64):
        """Mean ms per launch (prep, bsweep, fsweep, dual) and per step."""
        t, k = C.c_double(), (C.c_double * 4)()
        _check(load().spock_time_kernels(self.h, precision, int(steps), C.byref(t), k))
        return t.value, list(k)

    def kernel_bytes(self, precision=FP64):
        """Algorithmic bytes of each launch of one step."""
        k = (C.c_double * 4)()
        _check(load().spock_kernel_bytes(self.h, precision, k))
        return list(k)

    def step_bytes(self, precision=FP64):
        b, f = C.c_double(), C.c_double()
        _check(load().spock_step_bytes(self.h, precision, C.byref(b), C.byref(f)))
        return b.value, f.value


class Batch:
    """Many problems advanced by one backward and one forward launch per step."""

    def __init__(self, problems, settings=None, **kw):
        lib = load()
        self._lib = lib
        self.problems = list(problems)
        self.settings = settings or default_settings(**kw)
        arr = (C.c_void_p * len(self.problems))(*[p.h.value for p in self.problems])
        h = C.c_void_p()
        _check(lib.spock_batch_create(arr, len(self.problems), C.byref(self.settings), C.byref(h)))
        self.h = h
        npb, nt, nb = C.c_int32(), C.c_int32(), C.c_size_t()
        _check(lib.spock_batch_size(h, C.byref(npb), C.byref(nt), C.byref(nb)))
        self.n_tasks, self.device_bytes = nt.value, nb.value

    def close(self):
        if getattr(self, "h", None):
            self._lib.spock_batch_destroy(self.h)
            self.h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def solve(self, x0s, warm=None):
        n = len(self.problems)
        keep = [np.ascontiguousarray(x, dtype=np.float64) for x in x0s]
        ptrs = (_dp * n)(*[_ptr(x) for x in keep])
        w = None if warm is None else np.ascontiguousarray(warm, dtype=np.int32)
        infos = (Info * n)()
        _check(load().spock_batch_solve(self.h, ptrs, None if w is None else _ptr(w, np.int32), infos))
        return [i.as_dict() for i in infos]

    def run_steps(self, steps, precision=FP64, sync=True):
        _check(load().spock_batch_run_steps(self.h, precision, int(steps), int(bool(sync))))

    def set_launch(self, workgroup, precision=FP64):
        _check(load().spock_batch_set_launch(self.h, precision, int(workgroup)))

    def time_steps(self, steps, precision=FP64):
        t, b, f = C.c_double(), C.c_double(), C.c_double()
        _check(load().spock_batch_time_steps(self.h, precision, int(steps), C.byref(t), C.byref(b), C.byref(f)))
        return t.value, b.value, f.value

    def time_kernels(self, steps, precision=FP64):
        t, k = C.c_double(), (C.c_double * 4)()
        _check(load().spock_batch_time_kernels(self.h, precision, int(steps), C.byref(t), k))
        return t.value, list(k)

    def kernel_bytes(self, precision=FP64):
        k = (C.c_double * 4)()
        _check(load().spock_batch_kernel_bytes(self.h, precision, k))
        return list(k)

    def step_bytes(self, precision=FP64):
        b, f = C.c_double(), C.c_double()
        _check(load().spock_batch_step_bytes(self.h, precision, C.byref(b), C.byref(f)))
        return b.value, f.value


class Server:
    """Continuous-batching MPC server (worker thread inside the library)."""

    def __init__(self, hbm_budget, settings=None, **kw):
        lib = load()
        self._lib = lib
        self.settings = settings or default_settings(**kw)
        h = C.c_void_p()
        _check(lib.spock_server_create(int(hbm_budget), C.byref(self.settings), C.byref(h)))
        self.h = h
        self.shapes = {}

    def close(self):
        if getattr(self, "h", None):
            self._lib.spock_server_destroy(self.h)
            self.h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def add_tree(self, prob):
        d = _Desc(prob)
        tid = C.c_int64()
        _check(load().spock_server_add_tree(self.h, C.byref(d.desc), C.byref(tid)))
        self.shapes[tid.value] = (len(prob["parent"]), int(prob["nx"]), int(prob["nu"]),
                                  int(np.asarray(prob["gamma"]).size))
        return tid.value

    def submit(self, tree_id, x0, req_id):
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        _check(load().spock_server_submit(self.h, int(tree_id), _ptr(x0), int(req_id)))

    def poll(self, max_results=1024):
        out = (Result * max_results)()
        n = C.c_int32()
        _check(load().spock_server_poll(self.h, out, max_results, C.byref(n)))
        return [out[i].as_dict() for i in range(n.value)]

    def wait_idle(self, timeout_s=600.0):
        _check(load().spock_server_wait_idle(self.h, float(timeout_s)))

    def stats(self):
        st = ServerStats()
        _check(load().spock_server_get_stats(self.h, C.byref(st)))
        return st.as_dict()

    def solution(self, tree_id):
        n, nx, nu, nl = self.shapes[tree_id]
        x, u, s0 = np.zeros((n, nx)), np.zeros((nl, nu)), C.c_double()
        _check(load().spock_server_solution(self.h, int(tree_id), _ptr(x), _ptr(u), C.byref(s0)))
        return x, u, s0.value


def now():
    return load().spock_now()
