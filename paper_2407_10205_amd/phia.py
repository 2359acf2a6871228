"""Python binding of libphia.so (include/phia.h): argument marshalling only.

Every step of the sweep runs in the HIP kernels of the shared library.  If
the library is missing this module raises at import; there is no CPU
fallback.  torch is imported first so that the process holds a single HIP
runtime (torch's), which the library then shares; torch supplies streams and
events for timing.
"""
import ctypes as C
import os

import numpy as np

try:  # one HIP runtime per process: load torch's before the library's
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libphia.so")

PATHS = {"auto": 0, "fp32": 1, "i8": 2, "bf16hilo": 3, "ell": 4}
PATH_NAMES = {v: k for k, v in PATHS.items()}
STATUS = {0: "PHIA_OK", -1: "PHIA_EINVAL", -2: "PHIA_ENOTSYM", -3: "PHIA_EDIAG", -4: "PHIA_ERANGE",
          -5: "PHIA_ENOMEM", -6: "PHIA_EDEVICE", -7: "PHIA_ESTATE"}

# Every symbol declared in include/phia.h.
EXPORTS = ("phia_create", "phia_anneal", "phia_anneal_noalloc", "phia_anneal_start", "phia_anneal_run",
           "phia_sync",
           "phia_best", "phia_best_exact", "phia_best_f64", "phia_replica_best", "phia_replica_mh", "phia_get_state",
           "phia_set_state", "phia_get_info", "phia_set_incremental", "phia_incremental_stats",
           "phia_set_exchange_seq", "phia_raise_error_word", "phia_autotune", "phia_set_trace", "phia_get_trace", "phia_eval_fmath",
           "phia_batch_run", "phia_batch_create", "phia_batch_launch", "phia_batch_sync", "phia_batch_destroy",
           "phia_server_create", "phia_server_submit", "phia_server_footprint", "phia_server_poll",
           "phia_server_wait", "phia_server_spins", "phia_server_cancel", "phia_server_destroy",
           "phia_valu_crossover", "phia_destroy", "phia_last_error", "phia_version")

REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_CANCELLED, REQ_FAILED = 0, 1, 2, 3, -1


class PhiaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Options(C.Structure):
    _fields_ = [("frac_bits", C.c_int32), ("quantize", C.c_int32), ("path", C.c_int32),
                ("device", C.c_int32), ("stream", C.c_void_p), ("defer_upload", C.c_int32)]


class Schedule(C.Structure):
    _fields_ = [("beta0", C.c_float), ("beta1", C.c_float), ("betas", C.c_void_p),
                ("eps", C.c_float), ("gamma", C.c_float), ("refresh_L", C.c_int64), ("deriv_mode", C.c_int32),
                ("metropolis", C.c_int32), ("mh_up", C.c_float), ("mh_down", C.c_float),
                ("initial_kick", C.c_int32)]


DERIV = {"tanh": 0, "poly2": 1}


class Result(C.Structure):
    _fields_ = [("state", C.c_int32), ("success", C.c_int32), ("frac_bits", C.c_int32), ("replica", C.c_int32),
                ("energy_units", C.c_int64), ("steps_used", C.c_int64), ("t_arrive", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [("N", C.c_int32), ("Np", C.c_int32), ("path", C.c_int32), ("frac_bits", C.c_int32),
                ("exact", C.c_int32), ("group", C.c_int32), ("replicas", C.c_int32),
                ("rows_per_block", C.c_int32), ("j_in_lds", C.c_int32), ("sweep_kernel", C.c_int32),
                ("steps", C.c_int64), ("step", C.c_int64),
                ("max_abs_J", C.c_int64), ("device_bytes", C.c_size_t), ("group_on_one_xcd", C.c_int32),
                ("incremental", C.c_int32)]


def _declare(lib):
    P, I32, I64, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    sig = {
        "phia_create": [P, P, I32, P, P],
        "phia_anneal": [P, I32, I64, P, U64],
        "phia_anneal_noalloc": [P, I32, I64, P, U64, P, P, P, P, P, P, P],
        "phia_anneal_start": [P, I32, I64, P, U64],
        "phia_anneal_run": [P, I64],
        "phia_sync": [P],
        "phia_best": [P, P, P],
        "phia_best_exact": [P, P, P, P],
        "phia_best_f64": [P, P],
        "phia_replica_best": [P, P, P, P],
        "phia_replica_mh": [P, P, P, P],
        "phia_get_state": [P, P, P, P],
        "phia_set_state": [P, P, P, I64],
        "phia_get_info": [P, P],
        "phia_autotune": [P, I32, I64, P],
        "phia_set_trace": [P, I32],
        "phia_set_incremental": [P, I32],
        "phia_incremental_stats": [P, P],
        "phia_set_exchange_seq": [P, C.c_uint32],
        "phia_raise_error_word": [P, I32],
        "phia_get_trace": [P, P],
        "phia_eval_fmath": [I32, P, P, P, I64, I32],
        "phia_batch_run": [P, I32, P, P, P, P],
        "phia_batch_create": [P, I32, P, P, P, P],
        "phia_batch_launch": [P, P],
        "phia_batch_sync": [P],
        "phia_server_create": [C.c_size_t, I32, I32, I32, P],
        "phia_server_submit": [P, P, I32, I64, I64, P, U64, P],
        "phia_server_poll": [P, U64, P],
        "phia_server_footprint": [P, I32, I64, P],
        "phia_server_wait": [P, U64, C.c_double, P],
        "phia_server_spins": [P, U64, P],
        "phia_server_cancel": [P, U64],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.phia_destroy.argtypes = [P]
    lib.phia_destroy.restype = None
    lib.phia_server_destroy.argtypes = [P]
    lib.phia_server_destroy.restype = None
    lib.phia_batch_destroy.argtypes = [P]
    lib.phia_batch_destroy.restype = None
    lib.phia_last_error.restype = C.c_char_p
    lib.phia_version.restype = C.c_char_p
    lib.phia_valu_crossover.argtypes = [I32]
    lib.phia_valu_crossover.restype = C.c_int32


_lib = None


def lib():
    """Load libphia.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2407_10205_amd.build.build()")
        handle = C.CDLL(LIB_PATH)
        _declare(handle)
        _lib = handle
    return _lib


def _check(rc):
    if rc != 0:
        raise PhiaError(rc, lib().phia_last_error().decode(errors="replace"))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_schedule(steps, eps, gamma, beta0=None, beta1=None, betas=None, refresh_L=50, deriv="tanh", mh=None,
                  ikick=False):
    """Build a Schedule; keeps a reference to the betas array on the object.
    deriv: "tanh" (Eq. 8) or "poly2" (the FPGA's quadratic).  mh: None, or
    (up, down) to accept or reject every trajectory of refresh_L steps and
    multiply beta by up / down after each outcome ((1, 1): fixed schedule).
    ikick: the initial-kick variant (half a kick after every momentum draw)."""
    s = Schedule()
    s.initial_kick = 1 if ikick else 0
    s.eps = eps
    s.gamma = gamma
    s.refresh_L = int(refresh_L)
    s.deriv_mode = DERIV[deriv] if isinstance(deriv, str) else int(deriv)
    s.metropolis = 0 if mh is None else 1
    s.mh_up, s.mh_down = (1.0, 1.0) if mh is None else (float(mh[0]), float(mh[1]))
    if betas is not None:
        b = np.ascontiguousarray(betas, dtype=np.float32)
        if b.shape[0] < steps:
            raise ValueError("betas shorter than steps")
        s.betas = b.ctypes.data
        s._keep = b
        s.beta0 = float(b[0])
        s.beta1 = float(b[-1])
    else:
        s.beta0 = beta0
        s.beta1 = beta1
        s.betas = None
    return s


class Problem:
    """One Ising instance on the device (phia_problem)."""

    def __init__(self, J, h=None, frac_bits=-1, quantize=False, path="auto", device=0, stream=None,
                 defer_upload=False):
        J = np.ascontiguousarray(J, dtype=np.float64)
        if J.ndim != 2 or J.shape[0] != J.shape[1]:
            raise ValueError("J must be square")
        self.N = J.shape[0]
        hh = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
        o = Options(frac_bits, 1 if quantize else 0, PATHS[path] if isinstance(path, str) else int(path),
                    device, C.c_void_p(stream) if stream else None, 1 if defer_upload else 0)
        p = C.c_void_p()
        _check(lib().phia_create(_ptr(J), _ptr(hh), self.N, C.byref(o), C.byref(p)))
        self._p = p
        self._sched = None
        self.R = 0

    # -- lifetime
    def close(self):
        if getattr(self, "_p", None):
            lib().phia_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- anneal
    def set_trace(self, enable=True):
        _check(lib().phia_set_trace(self._p, 1 if enable else 0))

    def set_incremental(self, on=True):
        """Flip-incremental J.s update where the sweep has it (identical
        results): True, False, or None for the default (on, except with the
        accept/reject step)."""
        _check(lib().phia_set_incremental(self._p, -1 if on is None else 1 if on else 0))

    def incremental_stats(self):
        """(incremental steps, full-product steps, k blocks of the incremental
        products) since the anneal started, summed over replica blocks."""
        out = (C.c_int64 * 3)()
        _check(lib().phia_incremental_stats(self._p, out))
        return tuple(int(v) for v in out)

    def set_exchange_seq(self, seq):
        """Test hook: sequence number of the next column-split launch."""
        _check(lib().phia_set_exchange_seq(self._p, int(seq)))

    def raise_error_word(self, on=True):
        """Test hook: raise the device error word before every following launch."""
        _check(lib().phia_raise_error_word(self._p, 1 if on else 0))

    def start(self, replicas, steps, eps, gamma, beta0=None, beta1=None, betas=None, refresh_L=50, seed=0,
              deriv="tanh", mh=None, ikick=False):
        self._sched = make_schedule(steps, eps, gamma, beta0, beta1, betas, refresh_L, deriv, mh, ikick)
        _check(lib().phia_anneal_start(self._p, int(replicas), int(steps), C.byref(self._sched), int(seed)))
        self.R = int(replicas)

    def run(self, k_end):
        _check(lib().phia_anneal_run(self._p, int(k_end)))

    def sync(self):
        _check(lib().phia_sync(self._p))

    def anneal(self, replicas, steps, eps, gamma, beta0=None, beta1=None, betas=None, refresh_L=50, seed=0,
               deriv="tanh", mh=None, ikick=False):
        self._sched = make_schedule(steps, eps, gamma, beta0, beta1, betas, refresh_L, deriv, mh, ikick)
        _check(lib().phia_anneal(self._p, int(replicas), int(steps), C.byref(self._sched), int(seed)))
        self.R = int(replicas)

    def anneal_noalloc(self, replicas, steps, eps, gamma, x, v, bestE, bestS, bestStep, beta0=None, beta1=None,
                       betas=None, refresh_L=50, seed=0, deriv="tanh", ikick=False):
        """phia_anneal_noalloc: x, v, bestE, bestS, bestStep are device
        addresses (ints) of caller-owned buffers ([replicas][Np] float, float,
        [replicas] int64, [replicas][Np] int8, [replicas] int64).  Returns the
        argmin (energy in units, replica)."""
        sch = make_schedule(steps, eps, gamma, beta0, beta1, betas, refresh_L, deriv, None, ikick)
        e, r = C.c_int64(), C.c_int32()
        _check(lib().phia_anneal_noalloc(self._p, int(replicas), int(steps), C.byref(sch), int(seed),
                                         C.c_void_p(x), C.c_void_p(v), C.c_void_p(bestE), C.c_void_p(bestS),
                                         C.c_void_p(bestStep), C.byref(e), C.byref(r)))
        return e.value, r.value

    # -- results
    def best(self):
        e = C.c_double()
        s = np.zeros(self.N, np.int8)
        _check(lib().phia_best(self._p, C.byref(e), _ptr(s)))
        return e.value, s

    def best_exact(self):
        e, f, r = C.c_int64(), C.c_int32(), C.c_int32()
        _check(lib().phia_best_exact(self._p, C.byref(e), C.byref(f), C.byref(r)))
        return e.value, f.value, r.value

    def best_f64(self):
        e = C.c_double()
        _check(lib().phia_best_f64(self._p, C.byref(e)))
        return e.value

    def replica_best(self):
        E = np.zeros(self.R, np.int64)
        S = np.zeros((self.R, self.N), np.int8)
        K = np.zeros(self.R, np.int64)
        _check(lib().phia_replica_best(self._p, _ptr(E), _ptr(S), _ptr(K)))
        return E, S, K

    def replica_mh(self):
        """Per replica: trajectories accepted, trajectories decided, beta multiplier."""
        acc = np.zeros(self.R, np.int32)
        dec = np.zeros(self.R, np.int32)
        lam = np.zeros(self.R, np.float32)
        _check(lib().phia_replica_mh(self._p, _ptr(acc), _ptr(dec), _ptr(lam)))
        return acc, dec, lam

    def trace(self, steps):
        E = np.zeros((self.R, steps), np.int64)
        _check(lib().phia_get_trace(self._p, _ptr(E)))
        return E

    def get_state(self):
        x = np.zeros((self.R, self.N), np.float32)
        v = np.zeros((self.R, self.N), np.float32)
        k = C.c_int64()
        _check(lib().phia_get_state(self._p, _ptr(x), _ptr(v), C.byref(k)))
        return x, v, k.value

    def set_state(self, x, v, k):
        x = np.ascontiguousarray(x, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        _check(lib().phia_set_state(self._p, _ptr(x), _ptr(v), int(k)))

    def autotune(self, replicas, probe_steps=200):
        """Time every feasible sweep geometry and keep the fastest (us/step)."""
        us = C.c_double()
        _check(lib().phia_autotune(self._p, int(replicas), int(probe_steps), C.byref(us)))
        return us.value

    def info(self):
        i = Info()
        _check(lib().phia_get_info(self._p, C.byref(i)))
        d = {f: getattr(i, f) for f, _ in Info._fields_}
        d["path_name"] = PATH_NAMES.get(d["path"], "?")
        return d


def _schedules(steps, schedules):
    n = len(schedules)
    scheds = (Schedule * n)()
    keep = []
    for i, sc in enumerate(schedules):
        one = make_schedule(int(steps[i]), sc["eps"], sc["gamma"], sc.get("beta0"), sc.get("beta1"),
                            sc.get("betas"), sc.get("refresh_L", 50), sc.get("deriv", "tanh"), sc.get("mh"),
                            sc.get("ikick", False))
        keep.append(one)
        C.memmove(C.byref(scheds, i * C.sizeof(Schedule)), C.byref(one), C.sizeof(Schedule))
    return scheds, keep


class Batch:
    """A reusable batch plan (phia_batch_create): set up once, then launch
    the anneal of every problem many times with new seeds."""

    def __init__(self, problems, replicas, steps, schedules):
        n = len(problems)
        self.problems = list(problems)
        arr = (C.c_void_p * n)(*[p._p for p in problems])
        self._reps = np.ascontiguousarray(replicas, dtype=np.int32)
        stp = np.ascontiguousarray(steps, dtype=np.int64)
        scheds, keep = _schedules(stp, schedules)
        b = C.c_void_p()
        _check(lib().phia_batch_create(arr, n, _ptr(self._reps), _ptr(stp), C.cast(scheds, C.c_void_p),
                                       C.byref(b)))
        del keep
        self._b = b
        for p, r in zip(problems, self._reps):
            p.R = int(r)

    def launch(self, seeds):
        """Enqueue one anneal of every problem (returns without waiting)."""
        sd = np.ascontiguousarray(seeds, dtype=np.uint64)
        _check(lib().phia_batch_launch(self._b, _ptr(sd)))

    def sync(self):
        _check(lib().phia_batch_sync(self._b))

    def close(self):
        if getattr(self, "_b", None):
            lib().phia_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def batch_run(problems, replicas, steps, schedules, seeds):
    """Anneal several problems in one graph launch (phia_batch_run).

    schedules: list of dicts with eps, gamma, beta0, beta1 (or betas), refresh_L,
    optionally deriv and mh (see make_schedule).
    """
    n = len(problems)
    arr = (C.c_void_p * n)(*[p._p for p in problems])
    reps = np.ascontiguousarray(replicas, dtype=np.int32)
    stp = np.ascontiguousarray(steps, dtype=np.int64)
    sd = np.ascontiguousarray(seeds, dtype=np.uint64)
    scheds = (Schedule * n)()
    keep = []
    for i, sc in enumerate(schedules):
        one = make_schedule(int(stp[i]), sc["eps"], sc["gamma"], sc.get("beta0"), sc.get("beta1"),
                            sc.get("betas"), sc.get("refresh_L", 50), sc.get("deriv", "tanh"), sc.get("mh"),
                            sc.get("ikick", False))
        keep.append(one)
        C.memmove(C.byref(scheds, i * C.sizeof(Schedule)), C.byref(one), C.sizeof(Schedule))
    _check(lib().phia_batch_run(arr, n, _ptr(reps), _ptr(stp), C.cast(scheds, C.c_void_p), _ptr(sd)))
    for p, r in zip(problems, reps):
        p.R = int(r)
    del keep


def valu_crossover(Np):
    """Largest replica count for which an I8 anneal takes the VALU sweep (phia_valu_crossover)."""
    return int(lib().phia_valu_crossover(int(Np)))


def server_footprint(problem, replicas, max_steps):
    b = C.c_size_t()
    _check(lib().phia_server_footprint(problem._p, int(replicas), int(max_steps), C.byref(b)))
    return b.value


class Server:
    """Continuous-batching annealing server (phia_server)."""

    def __init__(self, hbm_budget, max_slots=64, chunk_steps=1000, device=0):
        s = C.c_void_p()
        _check(lib().phia_server_create(int(hbm_budget), int(max_slots), int(chunk_steps), int(device),
                                        C.byref(s)))
        self._s = s
        self._keep = {}

    def submit(self, problem, replicas, max_steps, target, eps, gamma, beta0=None, beta1=None, betas=None,
               refresh_L=50, seed=0, deriv="tanh", mh=None):
        sch = make_schedule(max_steps, eps, gamma, beta0, beta1, betas, refresh_L, deriv, mh)
        t = C.c_uint64()
        _check(lib().phia_server_submit(self._s, problem._p, int(replicas), int(max_steps), int(target),
                                        C.byref(sch), int(seed), C.byref(t)))
        self._keep[t.value] = (problem, sch)
        return t.value

    def poll(self, ticket):
        r = Result()
        _check(lib().phia_server_poll(self._s, int(ticket), C.byref(r)))
        return r.as_dict()

    def wait(self, ticket, timeout=-1.0):
        r = Result()
        _check(lib().phia_server_wait(self._s, int(ticket), float(timeout), C.byref(r)))
        return r.as_dict()

    def spins(self, ticket):
        p = self._keep[ticket][0]
        out = np.zeros(p.N, np.int8)
        _check(lib().phia_server_spins(self._s, int(ticket), _ptr(out)))
        return out

    def cancel(self, ticket):
        _check(lib().phia_server_cancel(self._s, int(ticket)))

    def close(self):
        if getattr(self, "_s", None):
            lib().phia_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def eval_fmath(kind, values=None, quads=None, seed=0, device=0):
    """Evaluate the device's elementary functions (self-check hook)."""
    if kind == 4:
        q = np.ascontiguousarray(quads, dtype=np.uint64).reshape(-1, 4)
        n = q.shape[0]
        in64 = np.concatenate([np.array([seed], np.uint64), q.reshape(-1)])
        out = np.zeros(n, np.float32)
        _check(lib().phia_eval_fmath(4, None, _ptr(in64), _ptr(out), n, device))
        return out
    vals = np.ascontiguousarray(values, dtype=np.float32)
    n = vals.shape[0]
    out = np.zeros(2 * n if kind == 2 else n, np.float32)
    _check(lib().phia_eval_fmath(kind, _ptr(vals), None, _ptr(out), n, device))
    return out.reshape(n, 2) if kind == 2 else out
