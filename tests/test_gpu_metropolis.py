"""GPU parity of the accept/reject step (App. A; Table 3, state 4) against the
CPU oracle, through the C ABI.

Every quantity is compared exactly, as for the plain sweep: x, v, records,
energy traces, and per replica the accepted and decided trajectory counts and
the beta multiplier.
"""
import os
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


def int_units(J, h, f):
    return (np.rint(J * 2**f).astype(np.int32), np.rint(h * 2**f).astype(np.int32))


class _Geometry:
    def __init__(self, spec):
        self.spec = spec

    def __enter__(self):
        if self.spec:
            os.environ["PHIA_GEOMETRY"] = self.spec

    def __exit__(self, *exc):
        os.environ.pop("PHIA_GEOMETRY", None)


def device_run(P, J, h, f, path, R, T, sched, seed, mh, trace=True, chunks=None, geometry=None):
    with _Geometry(geometry):
        p = P.Problem(J, h, frac_bits=f, path=path)
        if trace:
            p.set_trace(True)
        p.start(R, T, seed=seed, mh=mh, **sched)
    for k in (chunks or []) + [T]:
        p.run(k)
    p.sync()
    E, S, K = p.replica_best()
    x, v, _ = p.get_state()
    acc, dec, lam = p.replica_mh()
    out = dict(E=E, S=S, K=K, x=x, v=v, acc=acc, dec=dec, lam=lam, info=p.info(),
               trace=p.trace(T) if trace else None)
    p.close()
    return out


def oracle_rows(O, J, h, f, T, sched, seed, mh, rows, trace=True):
    Ji, hi = int_units(J, h, f)
    betas = O.beta_linear(sched["beta0"], sched["beta1"], T)
    return {r: O.anneal(Ji, hi, f, 1, betas, sched["eps"], sched["gamma"], sched["refresh_L"], seed, r0=r,
                        trace=trace, mh=mh) for r in rows}


def assert_parity(dev, runs):
    for r, o in runs.items():
        assert np.array_equal(dev["x"][r].view(np.uint32), o.x[0].view(np.uint32)), f"x replica {r}"
        assert np.array_equal(dev["v"][r].view(np.uint32), o.v[0].view(np.uint32)), f"v replica {r}"
        assert dev["E"][r] == o.bestE[0], f"bestE replica {r}"
        assert dev["K"][r] == o.bestStep[0], f"bestStep replica {r}"
        assert np.array_equal(dev["S"][r], o.bestS[0]), f"bestS replica {r}"
        assert dev["acc"][r] == o.acc[0] and dev["dec"][r] == o.dec[0], f"accept counts replica {r}"
        assert dev["lam"][r].view(np.uint32) == o.lam[0].view(np.uint32), f"beta multiplier replica {r}"
        if dev["trace"] is not None and o.Etrace is not None:
            assert np.array_equal(dev["trace"][r], o.Etrace[0]), f"energy trace replica {r}"


RAGGED = dict(eps=0.3, gamma=1.0, beta0=0.2, beta1=3.0, refresh_L=23)


@pytest.mark.parametrize("path", ["fp32", "i8", "bf16hilo", "ell"])
def test_mh_parity_paths(P, O, path):
    """Ragged N, R and refresh period, fixed-point couplings on the 2^-5 grid,
    lam driven by the outcomes (1.25 up, 0.8 down): every replica matches."""
    J, h = inst.sk_gauss_fixed(77, 3, frac_bits=5, bits=8)
    R, T, seed, mh = 37, 301, 99, (1.25, 0.8)
    say(f"mh parity path={path} N=77 R={R} T={T}")
    dev = device_run(P, J, h, 5, path, R, T, RAGGED, seed, mh)
    assert dev["info"]["path_name"] == path
    runs = oracle_rows(O, J, h, 5, T, RAGGED, seed, mh, range(R))
    assert_parity(dev, runs)
    assert np.all(dev["dec"] == 12)
    assert 0 < dev["acc"].sum() < dev["dec"].sum()


@pytest.mark.parametrize("path", ["fp32", "ell"])
def test_mh_wide_workgroups(P, O, path):
    """The accept/reject step in the 1024-thread FP32 and ELL workgroups
    (Np = 640): the kinetic sums over 16 waves, a ragged replica count,
    every replica against the oracle."""
    if path == "fp32":
        J, h = inst.sk_gauss_fixed(600, 4, frac_bits=5, bits=8)
        f = 5
    else:
        J, h = inst.regular3_pm1(600, 4)
        f = 0
    R, T, seed, mh = 9, 151, 17, (1.25, 0.8)
    say(f"mh wide path={path} N=600 R={R} T={T}")
    dev = device_run(P, J, h, f, path, R, T, RAGGED, seed, mh)
    assert dev["info"]["path_name"] == path and dev["info"]["sweep_kernel"] == 4
    runs = oracle_rows(O, J, h, f, T, RAGGED, seed, mh, range(R))
    assert_parity(dev, runs)
    assert np.all(dev["dec"] == 5)  # k = 23, ..., 138; the first trajectory is taken undecided


def test_mh_off_by_default_and_counts_rejected(P, O):
    J, h = inst.sk_pm1(16, 0)
    p = P.Problem(J, h, path="i8")
    p.anneal(8, 100, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=25, seed=1)
    with pytest.raises(P.PhiaError) as e:
        p.replica_mh()
    assert e.value.code == -7
    with pytest.raises(P.PhiaError) as e:
        p.anneal(8, 100, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=25, seed=1, mh=(0.0, 1.0))
    assert e.value.code == -1
    p.close()


@pytest.mark.parametrize("G,jl", [(2, 1), (2, 0), (3, 0), (7, 1), (19, 0)])
def test_mh_column_split_geometries(P, O, G, jl):
    """Column-split groups exchange the decision's energy and kinetic
    partials: every group size gives the oracle's run (sampled replicas,
    ragged replica count, trajectory ends inside and at launch boundaries)."""
    J, h = inst.sk_gauss_fixed(300, 21, frac_bits=5, bits=8)
    R, T, seed, mh = 70, 180, 8, (1.1, 0.9)
    sched = dict(eps=0.25, gamma=1.0, beta0=0.05, beta1=1.5, refresh_L=20)
    say(f"mh geometry G={G} jl={jl}")
    dev = device_run(P, J, h, 5, "i8", R, T, sched, seed, mh, chunks=[40, 97], geometry=f"1,{G},{jl},2")
    assert dev["info"]["group"] == G
    runs = oracle_rows(O, J, h, 5, T, sched, seed, mh, [0, 15, 16, 47, 69])
    assert_parity(dev, runs)
    assert 0 < dev["acc"].sum() < dev["dec"].sum()


@pytest.mark.parametrize("path", ["fp32", "i8"])
def test_mh_chunked_run_is_bit_identical(P, O, path):
    J, h = inst.sk_gauss_fixed(40, 2, frac_bits=4)
    sched = dict(eps=0.3, gamma=1.0, beta0=0.5, beta1=3.0, refresh_L=30)
    ref = device_run(P, J, h, 4, path, 20, 400, sched, 17, (1.5, 0.75), trace=False)
    got = device_run(P, J, h, 4, path, 20, 400, sched, 17, (1.5, 0.75), trace=False,
                     chunks=[1, 7, 30, 60, 61, 100, 101, 390])
    for key in ("E", "S", "K", "x", "v", "acc", "dec", "lam"):
        assert np.array_equal(ref[key], got[key]), key
    runs = oracle_rows(O, J, h, 4, 400, sched, 17, (1.5, 0.75), [0, 19], trace=False)
    assert_parity(got, runs)


def test_mh_benchmark_shape_sampled(P, O):
    """Max-cut G(800, 0.06), 1024 replicas: column-split sweep with the
    accept/reject step, sampled replicas against the oracle."""
    J, h = inst.er_maxcut(800, 0.06, 0)
    sched = dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25)
    T, mh = 150, (1.02, 0.98)
    dev = device_run(P, J, h, 0, "i8", 1024, T, sched, 11, mh)
    say("geometry", dev["info"])
    assert dev["info"]["sweep_kernel"] == 0 and dev["info"]["group"] > 1
    runs = oracle_rows(O, J, h, 0, T, sched, 11, mh, [0, 1, 31, 32, 500, 1023])
    assert_parity(dev, runs)


def test_mh_batch_matches_single_runs(P, O):
    """A batch mixing accept/reject and plain instances: each equals its
    standalone anneal, and the oracle on a sampled replica."""
    specs = [("sk", 17, "i8", 16, 120, 1, (1.2, 0.9)), ("reg3", 64, "i8", 37, 90, 2, None),
             ("fixed", 250, "i8", 20, 60, 4, (1.0, 1.0)), ("sk", 100, "bf16hilo", 32, 75, 3, (1.3, 0.7)),
             ("fixed", 400, "i8", 18, 70, 5, (1.1, 0.8))]
    probs, insts, reps, steps, scheds, seeds = [], [], [], [], [], []
    for kind, N, path, R, T, seed, mh in specs:
        if kind == "sk":
            J, h = inst.sk_pm1(N, seed)
        elif kind == "reg3":
            J, h = inst.regular3_pm1(N, seed)
        else:
            J, h = inst.sk_gauss_fixed(N, seed, frac_bits=5, bits=8)
        insts.append((J, h))
        probs.append(P.Problem(J, h, path=path))
        reps.append(R)
        steps.append(T)
        scheds.append(dict(eps=0.25, gamma=1.0, beta0=0.1 * seed, beta1=2.0 + seed, refresh_L=7 + seed, mh=mh))
        seeds.append(500 + seed)
    say("mh batch of", len(probs))
    P.batch_run(probs, reps, steps, scheds, seeds)
    for i, p in enumerate(probs):
        got = p.replica_best() + p.get_state()[:2]
        J, h = insts[i]
        sc = dict(scheds[i])
        mh = sc.pop("mh")
        if mh is not None:
            got = got + p.replica_mh()
        q = P.Problem(J, h, path=specs[i][2])
        q.anneal(reps[i], steps[i], seed=seeds[i], mh=mh, **sc)
        ref = q.replica_best() + q.get_state()[:2] + (q.replica_mh() if mh is not None else ())
        for u, w in zip(ref, got):
            assert np.array_equal(u, w), specs[i]
        f = 5 if specs[i][0] == "fixed" else 0
        o = oracle_rows(O, J, h, f, steps[i], sc, seeds[i], mh, [reps[i] - 1], trace=False)[reps[i] - 1]
        assert got[0][-1] == o.bestE[0] and np.array_equal(got[3][-1], o.x[0]), specs[i]
        q.close()
        p.close()


def test_mh_server_same_alone_and_in_mix(P, O):
    """Served requests with the accept/reject step (small batched ones and a
    column-split one) give the same result alone and in a mix."""
    specs = []
    for i, (N, dense, R, T) in enumerate([(40, False, 32, 600), (300, True, 20, 500), (700, False, 32, 400)]):
        J, h, E, t = inst.planted_loops(N, 60 + i, alpha=0.4, dense=dense)
        specs.append((J, h, E, R, T, 40 + i))
    sched = dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25, mh=(1.05, 0.95))

    def serve(sub, slots):
        srv = P.Server(1 << 36, max_slots=slots, chunk_steps=70)
        probs, tickets = [], []
        for J, h, E, R, T, seed in sub:
            p = P.Problem(J, h, path="i8")
            probs.append(p)
            tickets.append(srv.submit(p, R, T, E, seed=seed, **sched))
        res = [srv.wait(t, 120.0) for t in tickets]
        spins = [srv.spins(t) for t in tickets]
        srv.close()
        for p in probs:
            p.close()
        return res, spins

    alone = [serve([sp], 1) for sp in specs]
    mix, mix_spins = serve(specs, 8)
    for i in range(len(specs)):
        r1, r2 = alone[i][0][0], mix[i]
        say("request", i, r1, r2)
        assert r1["state"] == P.REQ_DONE and r2["state"] == P.REQ_DONE
        for key in ("success", "energy_units", "replica", "steps_used"):
            assert r1[key] == r2[key], (i, key)
        assert np.array_equal(alone[i][1][0], mix_spins[i])
        J, h = specs[i][0], specs[i][1]
        assert O.energy(J.astype(np.int32), h.astype(np.int32), mix_spins[i]) == r2["energy_units"]


def test_mh_largest_int8_instance(P, O):
    """The accept/reject variant at its largest int8 instance (N = 4992),
    column-split, every replica against the oracle."""
    J, h = inst.sk_pm1(4992, 5)
    sched = dict(eps=0.2, gamma=1.0, beta0=0.5, beta1=2.0, refresh_L=3)
    say("mh largest N=4992")
    dev = device_run(P, J, h, 0, "i8", 16, 8, sched, 23, (1.1, 0.9), trace=False)
    say("geometry", dev["info"])
    runs = oracle_rows(O, J, h, 0, 8, sched, 23, (1.1, 0.9), range(16), trace=False)
    assert_parity(dev, runs)
