"""GPU tests of the column-split exchange's host-side logic, through the C ABI.

Workgroups that split one replica block's columns swap their spins every
step through words tagged with a sequence number.  The host restarts the
sequence (and clears the words) before the tag would wrap, and a kernel whose
bounded wait gives up raises the device error word, after which the handle
is poisoned.  Both paths are reached here with the test hooks of the ABI; no
kernel faults or hangs: a wait that gives up leaves the sweep normally.
"""
import os
import sys

import numpy as np
import pytest

from paper_2407_10205_amd import instances as inst

pytestmark = pytest.mark.gpu

EDEVICE = -6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    from paper_2407_10205_amd import phia
    phia.lib()
    return phia


class _Geometry:
    def __init__(self, spec):
        self.spec = spec

    def __enter__(self):
        os.environ["PHIA_GEOMETRY"] = self.spec

    def __exit__(self, *exc):
        del os.environ["PHIA_GEOMETRY"]


SCHED = dict(beta0=0.05, beta1=1.5, refresh_L=23)


def _run(P, J, h, spec, R, T, chunks=None, seq=None):
    with _Geometry(spec):
        p = P.Problem(J, h, path="i8")
        p.start(R, T, 0.2, 1.0, seed=71, **SCHED)
    if seq is not None:
        p.set_exchange_seq(seq)
    for k in (chunks or [T]):
        p.run(k)
    p.sync()
    info = p.info()
    got = p.replica_best() + p.get_state()[:2]
    p.close()
    return info, got


@pytest.mark.parametrize("spec,room", [("pp,3", (1 << 24) - 2), ("1,3,1", (1 << 32) - 2)])
def test_tag_restart_near_the_wrap(P, O, spec, room):
    """Interleaved sweep (24-bit tags) and one-block-per-workgroup sweep
    (32-bit tags): a run whose first launch ends just below the top of the
    tag range and whose second launch makes the host restart the sequence is
    bit-identical to a plain run, which matches the oracle."""
    J, h = inst.sk_gauss_fixed(150, 5, frac_bits=5, bits=8)
    R, T = 45, 137
    info, ref = _run(P, J, h, spec, R, T)
    say("geometry", spec, info)
    assert info["group"] == 3
    # every replica block of these geometries runs at once (one pass per
    # launch), so a launch of n steps uses n + 1 sequence numbers
    first = 50
    use1 = first + 1
    for seq in (room - use1, room - use1 - 5):
        _, got = _run(P, J, h, spec, R, T, chunks=[first, T], seq=seq)
        for u, w in zip(ref, got):
            assert np.array_equal(u, w), (spec, seq)
    Ji, hi = np.rint(J * 32).astype(np.int32), np.rint(h * 32).astype(np.int32)
    for r in (0, 44):
        o = O.anneal(Ji, hi, 5, 1, O.beta_linear(SCHED["beta0"], SCHED["beta1"], T), 0.2, 1.0, SCHED["refresh_L"],
                     71, r0=r)
        assert ref[0][r] == o.bestE[0] and np.array_equal(ref[3][r].view(np.uint32), o.x[0].view(np.uint32))


def test_exchange_seq_hook_rejects_bad_use(P):
    J, h = inst.sk_gauss_fixed(150, 5, frac_bits=5, bits=8)
    with _Geometry("pp,3"):
        p = P.Problem(J, h, path="i8")
        with pytest.raises(P.PhiaError) as e:
            p.set_exchange_seq(5)
        assert e.value.code == -7  # before phia_anneal_start
        p.start(45, 10, 0.2, 1.0, seed=1, **SCHED)
        with pytest.raises(P.PhiaError) as e:
            p.set_exchange_seq(1 << 24)
        assert e.value.code == -1
        p.close()
    q = P.Problem(J, h, path="i8")
    q.start(16, 10, 0.2, 1.0, seed=1, **SCHED)
    if q.info()["group"] == 1:
        with pytest.raises(P.PhiaError) as e:
            q.set_exchange_seq(5)
        assert e.value.code == -7
    q.close()


@pytest.mark.parametrize("spec", ["pp,4", "1,8,0"])
def test_wait_that_gives_up_poisons_the_handle(P, O, spec):
    """The device error word raised from the host before a launch, as if a
    workgroup's bounded wait had given up: the kernels leave the sweep at
    their next check (or finish), phia_sync reports PHIA_EDEVICE and every
    later call on the handle does too.  A fresh problem then runs normally."""
    J, h = inst.er_maxcut(400, 0.05, 2)
    R, T = 1024, 300
    say("error word raised", spec)
    with _Geometry(spec):
        p = P.Problem(J, h, path="i8")
        p.start(R, T, 0.2, 1.0, seed=3, **SCHED)
    assert p.info()["group"] > 1
    p.raise_error_word()
    p.run(T)
    with pytest.raises(P.PhiaError) as e:
        p.sync()
    assert e.value.code == EDEVICE
    with pytest.raises(P.PhiaError) as e:
        p.best()
    assert e.value.code == EDEVICE
    with pytest.raises(P.PhiaError) as e:
        p.anneal(R, T, 0.2, 1.0, seed=3, **SCHED)
    assert e.value.code == EDEVICE
    p.close()
    # the device is healthy: the same anneal on a fresh handle matches the oracle
    with _Geometry(spec):
        q = P.Problem(J, h, path="i8")
        q.anneal(64, 40, 0.2, 1.0, seed=3, **SCHED)
    E, S, K = q.replica_best()
    q.close()
    o = O.anneal(J.astype(np.int32), h.astype(np.int32), 0, 1, O.beta_linear(SCHED["beta0"], SCHED["beta1"], 40),
                 0.2, 1.0, SCHED["refresh_L"], 3, r0=63)
    assert E[63] == o.bestE[0] and np.array_equal(S[63], o.bestS[0])


def test_served_request_whose_wait_gives_up_fails_alone(P, O):
    """A served column-split request whose device error word is raised from
    the host (as if one of its workgroups' bounded waits had given up) runs in
    the same cooperative table launch as another column-split request: the
    round's batched read-out reports its error word, the request ends
    FAILED, and the other requests (one column-split, one batched) give the
    same results as when served without it."""
    sched = dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25)
    specs = []
    for i, (N, dense, R, T) in enumerate([(700, False, 32, 400), (650, False, 32, 400), (60, True, 32, 400)]):
        J, h, E, _ = inst.planted_loops(N, 400 + i, alpha=0.4, dense=dense)
        specs.append((J, h, E, R, T, 30 + i))

    def serve(raise_first):
        srv = P.Server(1 << 36, max_slots=8, chunk_steps=100)
        probs, tickets = [], []
        for k, (J, h, E, R, T, seed) in enumerate(specs):
            if k == 0 and not raise_first:
                continue
            p = P.Problem(J, h, path="i8")
            if k == 0:
                p.raise_error_word()
            probs.append(p)
            tickets.append(srv.submit(p, R, T, E, seed=seed, **sched))
        res = [srv.wait(t, 120.0) for t in tickets]
        spins = [srv.spins(t) if r["state"] == P.REQ_DONE else None for t, r in zip(tickets, res)]
        kinds = []
        for p in probs:  # the failed request's problem is poisoned
            try:
                i = p.info()
                kinds.append((i["sweep_kernel"], i["group"]))
            except P.PhiaError as e:
                kinds.append(e.code)
        srv.close()
        for p in probs:
            p.close()
        return res, spins, kinds

    res, spins, kinds = serve(True)
    say("raised", res[0], "geometries", kinds)
    # only column-split requests carry an error word into the read-out
    assert res[0]["state"] == P.REQ_FAILED and kinds[1][0] == 0 and kinds[1][1] > 1
    ref, ref_spins, _ = serve(False)
    for r1, s1, r2, s2 in zip(res[1:], spins[1:], ref, ref_spins):
        assert r1["state"] == P.REQ_DONE and r2["state"] == P.REQ_DONE
        for key in ("success", "energy_units", "replica", "steps_used"):
            assert r1[key] == r2[key], key
        assert np.array_equal(s1, s2)
