"""Device residency of the couplings: deferred uploads bound the serving
budget, and the FP64 copy of J exists only for rounded input."""
import sys

import numpy as np
import pytest

from paper_2407_10205_amd import instances as inst

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    from paper_2407_10205_amd import phia
    phia.lib()
    return phia


SCHED = dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25)


def test_fp64_copy_only_for_rounded_input(P):
    """An exact integer instance holds J (int8, plus its FP4 operand copy)
    and h on the device but no FP64 copy; its FP64 energy is the integer one
    times 2^-f.  A rounded instance also holds the N^2 FP64 couplings."""
    J, h = inst.sk_pm1(300, 1)
    p = P.Problem(J, h, path="i8")
    small = p.info()["device_bytes"]
    Np = p.info()["Np"]
    assert small < 2 * Np * Np < 300 * 300 * 8
    p.anneal(8, 50, seed=3, **SCHED)
    E, f, _ = p.best_exact()
    assert p.best_f64() == E * 2.0 ** -f
    p.close()
    Jr = J * (1.0 + 1e-3)
    q = P.Problem(Jr, h, path="i8", frac_bits=0, quantize=True)
    assert q.info()["device_bytes"] >= 300 * 300 * 8
    q.close()


def test_deferred_upload_and_release(P):
    """defer_upload: nothing of J on the device until the first anneal; the
    results equal those of an eagerly uploaded problem."""
    J, h = inst.er_maxcut(500, 0.05, 2, signed=True)
    eager = P.Problem(J, h, path="i8")
    lazy = P.Problem(J, h, path="i8", defer_upload=True)
    assert lazy.info()["device_bytes"] < 4096 < eager.info()["device_bytes"]
    for p in (eager, lazy):
        p.anneal(20, 300, seed=5, **SCHED)
    assert lazy.info()["device_bytes"] >= eager.info()["device_bytes"] - 4096
    a, b = eager.replica_best(), lazy.replica_best()
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    eager.close()
    lazy.close()


def test_server_budget_bounds_deferred_requests(P):
    """Requests of deferred problems hold no device memory while queued: with
    a budget that admits one at a time, the queued problems' couplings are
    not resident, and every problem is back to its small buffers when all
    requests are done.  Results equal those of eagerly uploaded problems."""
    specs = []
    for i in range(4):
        J, h, E, _ = inst.planted_loops(400, 300 + i, alpha=0.4)
        specs.append((J, h))
    T = 4000
    lazy = [P.Problem(J, h, path="i8", defer_upload=True) for J, h in specs]
    fps = [P.server_footprint(p, 16, T) for p in lazy]
    srv = P.Server(int(max(fps) * 1.3), max_slots=8, chunk_steps=500)
    tickets = [srv.submit(p, 16, T, -10**9, seed=7 + i, **SCHED) for i, p in enumerate(lazy)]
    queued_bytes = lazy[3].info()["device_bytes"]
    res = [srv.wait(t, 120.0) for t in tickets]
    srv.close()
    say("queued request held", queued_bytes, "bytes; footprints", fps)
    assert queued_bytes < 4096
    for a, b in zip(res, res[1:]):
        assert b["t_admit"] >= a["t_done"]
    assert all(r["state"] == P.REQ_DONE for r in res)
    assert all(p.info()["device_bytes"] < 4096 for p in lazy)
    eager = [P.Problem(J, h, path="i8") for J, h in specs]
    srv = P.Server(1 << 34, max_slots=8, chunk_steps=500)
    ref = [srv.wait(srv.submit(p, 16, T, -10**9, seed=7 + i, **SCHED), 120.0) for i, p in enumerate(eager)]
    srv.close()
    for r1, r2 in zip(res, ref):
        assert (r1["energy_units"], r1["replica"], r1["steps_used"]) == (r2["energy_units"], r2["replica"],
                                                                         r2["steps_used"])
    for p in lazy + eager:
        p.close()
