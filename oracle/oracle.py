"""ctypes wrapper of the C oracle (test infrastructure only).

Every function forwards numpy arrays to ``liboracle.so``; the arithmetic is in
``phia_oracle.c``.  Nothing here is used by the device library.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

TAG_X, TAG_V, TAG_MH = 0, 1, 2


class _MhC(C.Structure):
    _fields_ = [("enable", C.c_int32), ("up", C.c_float), ("down", C.c_float),
                ("x0", C.c_void_p), ("Estart", C.c_void_p), ("Qstart", C.c_void_p),
                ("Elast", C.c_void_p), ("lam", C.c_void_p), ("acc", C.c_void_p),
                ("dec", C.c_void_p), ("trace", C.c_void_p)]


def use_library(path):
    """Load the oracle from `path` (a copy built for the host CPU) from now on."""
    global _lib, _LIB_PATH
    _lib = None
    _LIB_PATH = path


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    P = C.c_void_p
    lib.oracle_philox4x64_10.argtypes = [P, P, P]
    lib.oracle_exp_nonpos.argtypes = [C.c_float]
    lib.oracle_exp_nonpos.restype = C.c_float
    lib.oracle_ln_unit.argtypes = [C.c_float]
    lib.oracle_ln_unit.restype = C.c_float
    lib.oracle_sincos_2pi.argtypes = [C.c_float, P, P]
    lib.oracle_sech2.argtypes = [C.c_float]
    lib.oracle_sech2.restype = C.c_float
    lib.oracle_poly2.argtypes = [C.c_float]
    lib.oracle_poly2.restype = C.c_float
    lib.oracle_uniform.argtypes = [C.c_uint32]
    lib.oracle_uniform.restype = C.c_float
    lib.oracle_gauss.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint64]
    lib.oracle_gauss.restype = C.c_float
    lib.oracle_energy.argtypes = [C.c_int, P, P, P]
    lib.oracle_energy.restype = C.c_int64
    lib.oracle_local_field.argtypes = [C.c_int, P, P, P, P]
    lib.oracle_energy_f64.argtypes = [C.c_int, P, P, P]
    lib.oracle_energy_f64.restype = C.c_double
    lib.oracle_bruteforce.argtypes = [C.c_int, P, P, P]
    lib.oracle_bruteforce.restype = C.c_int64
    lib.oracle_pack.argtypes = [C.c_int, P, P, C.c_int, C.c_int, P, P, P]
    lib.oracle_pack.restype = C.c_int
    lib.oracle_beta_linear.argtypes = [C.c_float, C.c_float, C.c_int64, P]
    lib.oracle_anneal.argtypes = [C.c_int, P, P, C.c_int, C.c_int, C.c_int64, C.c_int64,
                                  C.c_int64, P, C.c_float, C.c_float, C.c_int64, C.c_uint64,
                                  C.c_int, C.c_int, P, P, P, P, P, P, C.c_int]
    lib.oracle_anneal.restype = C.c_int
    lib.oracle_anneal_mh.argtypes = lib.oracle_anneal.argtypes + [C.POINTER(_MhC)]
    lib.oracle_anneal_mh.restype = C.c_int
    a = list(lib.oracle_anneal.argtypes)
    lib.oracle_anneal_ex.argtypes = a[:15] + [C.c_int] + a[15:] + [C.POINTER(_MhC)]
    lib.oracle_anneal_ex.restype = C.c_int
    lib.oracle_argmin.argtypes = [C.c_int, P]
    lib.oracle_argmin.restype = C.c_int
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def philox(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint64)
    key = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _load().oracle_philox4x64_10(_p(ctr), _p(key), _p(out))
    return out


def exp_nonpos(y):
    return np.float32(_load().oracle_exp_nonpos(float(y)))


def ln_unit(u):
    return np.float32(_load().oracle_ln_unit(float(u)))


def sincos_2pi(u):
    c = np.zeros(1, np.float32)
    s = np.zeros(1, np.float32)
    _load().oracle_sincos_2pi(float(u), _p(c), _p(s))
    return c[0], s[0]


def sech2(u):
    return np.float32(_load().oracle_sech2(float(u)))


def poly2(u):
    return np.float32(_load().oracle_poly2(float(u)))


def uniform(w):
    return np.float32(_load().oracle_uniform(int(w)))


def gauss(seed, tag, r, rnd, i):
    return np.float32(_load().oracle_gauss(seed, tag, r, rnd, i))


def _ij(J, h):
    J = np.ascontiguousarray(J, dtype=np.int32)
    N = J.shape[0]
    h = np.zeros(N, np.int32) if h is None else np.ascontiguousarray(h, dtype=np.int32)
    return N, J, h


def energy(J, h, s):
    N, J, h = _ij(J, h)
    s = np.ascontiguousarray(s, dtype=np.int8)
    return int(_load().oracle_energy(N, _p(J), _p(h), _p(s)))


def local_field(J, h, s):
    N, J, h = _ij(J, h)
    s = np.ascontiguousarray(s, dtype=np.int8)
    out = np.zeros(N, np.int32)
    _load().oracle_local_field(N, _p(J), _p(h), _p(s), _p(out))
    return out


def energy_f64(J, h, s):
    J = np.ascontiguousarray(J, dtype=np.float64)
    N = J.shape[0]
    h = np.zeros(N) if h is None else np.ascontiguousarray(h, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.int8)
    return float(_load().oracle_energy_f64(N, _p(J), _p(h), _p(s)))


def bruteforce(J, h):
    N, J, h = _ij(J, h)
    s = np.zeros(N, np.int8)
    e = int(_load().oracle_bruteforce(N, _p(J), _p(h), _p(s)))
    return e, s


def pack(J, h=None, frac_bits=-1, quantize=0):
    J = np.ascontiguousarray(J, dtype=np.float64)
    N = J.shape[0]
    hh = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
    Ji = np.zeros((N, N), np.int32)
    hi = np.zeros(N, np.int32)
    f = np.zeros(1, np.int32)
    rc = _load().oracle_pack(N, _p(J), _p(hh), frac_bits, quantize, _p(Ji), _p(hi), _p(f))
    return rc, Ji, hi, int(f[0])


def beta_linear(b0, b1, T):
    out = np.zeros(T, np.float32)
    _load().oracle_beta_linear(b0, b1, T, _p(out))
    return out


class Run:
    """State of an oracle anneal of R replicas (arrays are [R][N])."""

    def __init__(self, N, R):
        self.x = np.zeros((R, N), np.float32)
        self.v = np.zeros((R, N), np.float32)
        self.bestE = np.zeros(R, np.int64)
        self.bestS = np.zeros((R, N), np.int8)
        self.bestStep = np.zeros(R, np.int64)
        self.Etrace = None
        # accept/reject state (used when the anneal runs with mh=...)
        self.x0 = np.zeros((R, N), np.float32)
        self.Estart = np.zeros(R, np.int64)
        self.Qstart = np.zeros(R, np.int64)
        self.Elast = np.zeros(R, np.int64)
        self.lam = np.ones(R, np.float32)
        self.acc = np.zeros(R, np.int32)
        self.dec = np.zeros(R, np.int32)
        self.mhtrace = None


def anneal(J, h, frac_bits, R, betas, eps, gamma, L, seed, k0=0, k1=None, r0=0,
           run=None, trace=False, threads=1, deriv="tanh", mh=None, ikick=False):
    """Run steps k0 <= k < k1 (default: all of betas) of the sweep.

    With run=None a fresh anneal starts (k0 must be 0); otherwise the given
    Run is continued in place.  deriv: "tanh" (Eq. 8) or "poly2" (the
    quadratic of the POLY2 mode).  mh: None, or (up, down) to accept or reject
    every trajectory of L steps and scale beta by up / down after each
    outcome (trace=True also records the outcomes in run.mhtrace).  ikick:
    the initial-kick variant (Table 3, state 2; not with mh).  Returns the
    Run.
    """
    N, J, h = _ij(J, h)
    betas = np.ascontiguousarray(betas, dtype=np.float32)
    if k1 is None:
        k1 = betas.shape[0]
    init = run is None
    if init:
        run = Run(N, R)
    run.Etrace = np.zeros((R, k1 - k0), np.int64) if trace else None
    args = (N, _p(J), _p(h), frac_bits, R, r0, k0, k1, _p(betas),
            float(eps), float(gamma), int(L), int(seed), int(init),
            {"tanh": 0, "poly2": 1}[deriv],
            _p(run.x), _p(run.v), _p(run.bestE), _p(run.bestS),
            _p(run.bestStep), _p(run.Etrace), int(threads))
    if ikick:
        if mh is not None:
            raise ValueError("the initial kick is not combined with the accept/reject step")
        rc = _load().oracle_anneal_ex(*args[:15], 1, *args[15:], None)
    elif mh is None:
        rc = _load().oracle_anneal(*args)
    else:
        L = int(L)
        kd0 = L if k0 < L else k0 + (L - k0 % L) % L
        nd = (k1 - 1 - kd0) // L + 1 if k1 > kd0 else 0
        run.mhtrace = np.zeros((R, nd), np.int8) if trace else None
        st = _MhC(1, float(mh[0]), float(mh[1]), _p(run.x0), _p(run.Estart), _p(run.Qstart),
                  _p(run.Elast), _p(run.lam), _p(run.acc), _p(run.dec), _p(run.mhtrace))
        rc = _load().oracle_anneal_mh(*args, C.byref(st))
    if rc != 0:
        raise ValueError("oracle_anneal rejected its arguments")
    return run


def argmin(bestE):
    bestE = np.ascontiguousarray(bestE, dtype=np.int64)
    return int(_load().oracle_argmin(bestE.shape[0], _p(bestE)))
