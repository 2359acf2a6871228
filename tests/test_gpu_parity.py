"""GPU parity of the HIP sweep against the CPU oracle, through the C ABI.

Every quantity is compared exactly: the sweep is a fixed sequence of IEEE
binary32 operations and exact integer arithmetic, so x, v, spins, energies,
records and record steps must be bit-identical (which is tighter than the
1e-5 relative bound required of FP32 trajectories).
"""
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


def run_both(P, O, J, h, f, path, R, T, eps, gamma, b0, b1, L, seed, trace=True, sample=None, deriv="tanh"):
    """Run device and oracle on the same instance; returns (dev dict, oracle Run)."""
    say(f"case N={J.shape[0]} R={R} T={T} path={path} f={f} seed={seed} deriv={deriv}")
    prob = P.Problem(J, h, frac_bits=f, path=path)
    if trace:
        prob.set_trace(True)
    prob.anneal(R, T, eps, gamma, beta0=b0, beta1=b1, refresh_L=L, seed=seed, deriv=deriv)
    E, S, K = prob.replica_best()
    x, v, k = prob.get_state()
    dev = dict(E=E, S=S, K=K, x=x, v=v, k=k, info=prob.info(),
               trace=prob.trace(T) if trace else None, best=prob.best(), best_exact=prob.best_exact())
    prob.close()
    Ji, hi = int_units(J, h, f)
    betas = O.beta_linear(b0, b1, T)
    rows = range(R) if sample is None else sample
    runs = {}
    for r in rows:
        runs[r] = O.anneal(Ji, hi, f, 1, betas, eps, gamma, L, seed, r0=r, trace=trace, threads=1, deriv=deriv)
    return dev, runs


def assert_parity(dev, runs):
    for r, o in runs.items():
        assert np.array_equal(dev["x"][r].view(np.uint32), o.x[0].view(np.uint32)), f"x replica {r}"
        assert np.array_equal(dev["v"][r].view(np.uint32), o.v[0].view(np.uint32)), f"v replica {r}"
        assert dev["E"][r] == o.bestE[0], f"bestE replica {r}"
        assert dev["K"][r] == o.bestStep[0], f"bestStep replica {r}"
        assert np.array_equal(dev["S"][r], o.bestS[0]), f"bestS replica {r}"
        if dev["trace"] is not None:
            assert np.array_equal(dev["trace"][r], o.Etrace[0]), f"energy trace replica {r}"


# ------------------------------------------------------------ fmath ----
def test_fmath_bit_exact(P, O):
    rs = np.random.default_rng(0)
    ys = np.concatenate([np.linspace(-80, 0, 20001), -rs.exponential(3.0, 20000), [0.0, -81.0, -80.0]])
    ys = ys.astype(np.float32)
    got = P.eval_fmath(0, ys)
    ref = np.array([O.exp_nonpos(y) for y in ys], np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    us = ((2 * rs.integers(0, 2**23, 30000) + 1) / 2**24).astype(np.float32)
    got = P.eval_fmath(1, us)
    ref = np.array([O.ln_unit(u) for u in us], np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    got = P.eval_fmath(2, us)
    ref = np.array([O.sincos_2pi(u) for u in us], np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    xs = np.concatenate([rs.normal(0, 3, 30000), [0.0, -0.0, 40.0, 41.0], np.linspace(-90, 90, 721),
                         rs.normal(0, 0.01, 2000)]).astype(np.float32)
    got = P.eval_fmath(3, xs)
    ref = np.array([O.sech2(x) for x in xs], np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    xs = np.concatenate([rs.normal(0, 1, 30000), [0.0, -0.0, 1.5, -1.5, 40.0]]).astype(np.float32)
    got = P.eval_fmath(5, xs)
    ref = np.array([O.poly2(x) for x in xs], np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    quads = np.stack([rs.integers(0, 2, 20000), rs.integers(0, 2**40, 20000),
                      rs.integers(0, 2**20, 20000), rs.integers(0, 2**16, 20000)], axis=1).astype(np.uint64)
    got = P.eval_fmath(4, quads=quads, seed=0xABCDEF)
    ref = np.array([O.gauss(0xABCDEF, int(t), int(r), int(k), int(i)) for t, r, k, i in quads], np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


# ------------------------------------------------------- small cases ----
@pytest.mark.parametrize("path", ["fp32", "i8", "bf16hilo"])
def test_c1_sk16_parity(P, O, path):
    """SK N=16, J uniform +-1, h=0, 64 replicas x 1000 steps, linear beta."""
    J, h = inst.sk_pm1(16, 0)
    dev, runs = run_both(P, O, J, h, 0, path, 64, 1000, 0.2, 1.0, 0.1, 3.0, 50, 1234)
    assert dev["info"]["path_name"] == path
    assert_parity(dev, runs)
    Eg, _ = O.bruteforce(J.astype(np.int32), h.astype(np.int32))
    e, s = dev["best"]
    assert e == Eg
    assert O.energy(J.astype(np.int32), h.astype(np.int32), s) == Eg


@pytest.mark.parametrize("path", ["fp32", "i8", "bf16hilo"])
def test_final_argmin_matches_oracle(P, O, path):
    """Final choice (App. B, Table 3, state 5; ties over replicas take the
    lowest index): SK N = 16 with most of its 64 replicas at the exhaustive
    ground energy, and the ragged fixed-point case.  phia_best_exact's
    (energy, replica) and phia_best's spins equal the oracle's argmin over
    its per-replica records and that replica's best state."""
    J, h = inst.sk_pm1(16, 0)
    cases = [(J, h, 0, 64, 1000, 0.2, 1.0, 0.1, 3.0, 50, 1234)]
    J2, h2 = inst.sk_gauss_fixed(77, 3, frac_bits=5, bits=8)
    cases.append((J2, h2, 5, 37, 301, 0.15, 1.5, 0.05, 2.0, 37, 99))
    for J, h, f, R, T, eps, gamma, b0, b1, L, seed in cases:
        dev, runs = run_both(P, O, J, h, f, path, R, T, eps, gamma, b0, b1, L, seed, trace=False)
        oE = np.array([runs[r].bestE[0] for r in range(R)], np.int64)
        r_star = O.argmin(oE)
        E_units, f_dev, r_dev = dev["best_exact"]
        say("argmin", path, J.shape[0], "oracle", r_star, oE[r_star], "device", r_dev, E_units,
            "ties", int(np.sum(oE == oE[r_star])))
        assert (E_units, r_dev, f_dev) == (int(oE[r_star]), r_star, f)
        e, s = dev["best"]
        assert e == oE[r_star] * 2.0**-f
        assert np.array_equal(s, runs[r_star].bestS[0])


def test_final_argmin_many_ties_across_threads(P, O):
    """4096 replicas of SK N = 16: ties at the ground energy spread over every
    thread slot of the device reduction; the device picks the oracle's
    lowest-index replica, whose state it returns."""
    J, h = inst.sk_pm1(16, 0)
    R, T = 4096, 300
    p = P.Problem(J, h, path="i8")
    p.anneal(R, T, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=50, seed=31)
    E_units, _, r_dev = p.best_exact()
    e, s = p.best()
    Ed, Sd, _ = p.replica_best()
    p.close()
    Ji, hi = int_units(J, h, 0)
    o = O.anneal(Ji, hi, 0, R, O.beta_linear(0.1, 3.0, T), 0.2, 1.0, 50, 31, threads=8)
    assert np.array_equal(Ed, o.bestE) and np.array_equal(Sd, o.bestS)
    r_star = O.argmin(o.bestE)
    say("ties", int(np.sum(o.bestE == o.bestE[r_star])), "r*", r_star)
    assert np.sum(o.bestE == o.bestE[r_star]) > 100
    assert (E_units, r_dev) == (int(o.bestE[r_star]), r_star)
    assert np.array_equal(s, o.bestS[r_star])


def _betas_table(T):
    """A non-linear inverse-temperature table: geometric rise, a plateau and
    a drop (App. B, Table 3, state 4 leaves the temperature rule open)."""
    k = np.arange(T, dtype=np.float64)
    b = 0.05 * np.power(1.02, k)
    b = np.minimum(b, 2.5)
    b[T // 2: T // 2 + 7] = 0.3
    return b.astype(np.float32)


@pytest.mark.parametrize("path,geometry", [("fp32", None), ("i8", None), ("bf16hilo", None), ("i8", "1,3,1"),
                                           ("i8", "pp,3")])
def test_explicit_beta_table(P, O, path, geometry):
    """An explicit, non-linear beta table (phia_schedule.betas) is used step
    by step exactly as the oracle uses it: every replica bit-identical, on
    every sweep kernel (plain FP32, one block per workgroup, column split,
    interleaved column split)."""
    import os
    J, h = inst.sk_gauss_fixed(150, 5, frac_bits=5, bits=8)
    R, T, L, seed = 45, 211, 23, 71
    betas = _betas_table(T)
    say(f"betas path={path} geometry={geometry}")
    if geometry:
        os.environ["PHIA_GEOMETRY"] = geometry
    try:
        p = P.Problem(J, h, frac_bits=5, path=path)
        p.set_trace(geometry is None or not geometry.startswith("pp"))
        p.anneal(R, T, 0.2, 1.0, betas=betas, refresh_L=L, seed=seed)
    finally:
        os.environ.pop("PHIA_GEOMETRY", None)
    info = p.info()
    say("geometry", info)
    if geometry == "pp,3":
        assert info["sweep_kernel"] == 1
    elif geometry:
        assert info["group"] == 3 and info["sweep_kernel"] == 0
    E, S, K = p.replica_best()
    x, v, _ = p.get_state()
    tr = p.trace(T) if (geometry is None or not geometry.startswith("pp")) else None
    p.close()
    Ji, hi = int_units(J, h, 5)
    o = O.anneal(Ji, hi, 5, R, betas, 0.2, 1.0, L, seed, trace=True, threads=8)
    assert np.array_equal(x.view(np.uint32), o.x.view(np.uint32))
    assert np.array_equal(v.view(np.uint32), o.v.view(np.uint32))
    assert np.array_equal(E, o.bestE) and np.array_equal(K, o.bestStep) and np.array_equal(S, o.bestS)
    if tr is not None:
        assert np.array_equal(tr, o.Etrace)
    # the linear table it replaces gives a different run
    lin = O.anneal(Ji, hi, 5, 2, O.beta_linear(float(betas[0]), float(betas[-1]), T), 0.2, 1.0, L, seed)
    assert not np.array_equal(lin.x, o.x[:2])


@pytest.mark.parametrize("path", ["fp32", "i8", "bf16hilo"])
def test_ragged_fixed_point_parity(P, O, path):
    """Ragged N (not a multiple of 16 or 64), ragged R, fractional couplings
    and fields on the 2^-5 grid, momentum refresh period not dividing T."""
    J, h = inst.sk_gauss_fixed(77, 3, frac_bits=5, bits=8)
    dev, runs = run_both(P, O, J, h, 5, path, 37, 301, 0.15, 1.5, 0.05, 2.0, 37, 99)
    assert_parity(dev, runs)


@pytest.mark.parametrize("path", ["fp32", "i8", "bf16hilo"])
def test_poly2_mode_parity(P, O, path):
    """POLY2 derivative mode (quadratic in place of sech^2) on the ragged
    fixed-point case: every replica bit-identical to the oracle."""
    J, h = inst.sk_gauss_fixed(77, 3, frac_bits=5, bits=8)
    dev, runs = run_both(P, O, J, h, 5, path, 37, 301, 0.15, 1.5, 0.05, 2.0, 37, 99, deriv="poly2")
    assert_parity(dev, runs)


def test_bf16_hilo_sixteen_bit_couplings(P, O):
    """16-bit couplings (sigma = 2^-12): the hi plane is not zero."""
    J, h = inst.sk_gauss_fixed(50, 8, frac_bits=12, bits=16)
    assert np.abs(J * 4096).max() > 255
    dev, runs = run_both(P, O, J, h, 12, "bf16hilo", 20, 200, 0.2, 1.0, 0.001, 0.02, 25, 5)
    assert dev["info"]["path_name"] == "bf16hilo"
    assert_parity(dev, runs)


def test_single_spin_and_tiny(P, O):
    J = np.zeros((1, 1))
    h = np.array([0.75])
    dev, runs = run_both(P, O, J, h, 2, "i8", 5, 50, 0.2, 1.0, 0.1, 3.0, 7, 3)
    assert_parity(dev, runs)
    J, h = inst.sk_pm1(3, 1)
    dev, runs = run_both(P, O, J, h, 0, "fp32", 3, 20, 0.2, 1.0, 0.1, 3.0, 1, 3)
    assert_parity(dev, runs)


# ------------------------------------------------ resume and state ----
@pytest.mark.parametrize("path", ["fp32", "i8"])
def test_chunked_run_is_bit_identical(P, O, path):
    J, h = inst.sk_gauss_fixed(40, 2, frac_bits=4)
    a = P.Problem(J, h, path=path)
    a.anneal(20, 400, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=30, seed=17)
    ref = a.replica_best(), a.get_state()
    b = P.Problem(J, h, path=path)
    b.start(20, 400, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=30, seed=17)
    for k in (1, 7, 100, 101, 399, 400):
        b.run(k)
    b.sync()
    got = b.replica_best(), b.get_state()
    for u, w in zip(ref[0], got[0]):
        assert np.array_equal(u, w)
    assert np.array_equal(ref[1][0], got[1][0]) and np.array_equal(ref[1][1], got[1][1])
    a.close()
    b.close()


def test_set_state_continues_like_oracle(P, O):
    """Explicit (x, v) at step k: the device continues exactly as the oracle."""
    J, h = inst.sk_gauss_fixed(33, 4, frac_bits=3)
    Ji, hi = int_units(J, h, 3)
    T, R = 200, 6
    p = P.Problem(J, h, path="i8")
    p.start(R, T, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=1000, seed=1)
    rs = np.random.default_rng(7)
    x0 = rs.standard_normal((R, 33)).astype(np.float32)
    v0 = rs.standard_normal((R, 33)).astype(np.float32)
    p.set_state(x0, v0, 5)
    p.run(T)
    x, v, _ = p.get_state()
    run = O.Run(33, R)
    run.x[:] = x0
    run.v[:] = v0
    run.bestE[:] = np.iinfo(np.int64).max
    run.bestStep[:] = -1
    O.anneal(Ji, hi, 3, R, O.beta_linear(0.1, 3.0, T), 0.2, 1.0, 1000, 1, k0=5, k1=T, run=run)
    assert np.array_equal(x, run.x) and np.array_equal(v, run.v)
    E, S, K = p.replica_best()
    assert np.array_equal(E, run.bestE) and np.array_equal(K, run.bestStep)
    p.close()


def test_best_energy_f64_against_original_couplings(P, O):
    """Rounded input: phia_best reports the FP64 energy of the best state
    against the original real couplings."""
    rs = np.random.default_rng(2)
    N = 30
    U = rs.uniform(-1, 1, (N, N))
    J = np.triu(U, 1) + np.triu(U, 1).T
    h = rs.uniform(-1, 1, N)
    p = P.Problem(J, h, frac_bits=6, quantize=True, path="i8")
    assert p.info()["exact"] == 0
    p.anneal(16, 300, 0.2, 1.0, beta0=0.5, beta1=20.0, refresh_L=50, seed=3)
    e, s = p.best()
    assert abs(e - O.energy_f64(J, h, s)) <= 1e-12 * max(1.0, abs(e))
    p.close()


# ------------------------------------------- workgroup-group path ----
def test_group_split_parity_sampled(P, O):
    """Max-cut on G(800, 0.06), int8 J too large for one CU's LDS: the
    columns are split over a group of workgroups.  Full replica count of the
    benchmark workload shape (1024); sampled replicas against the oracle."""
    J, h = inst.er_maxcut(800, 0.06, 0)
    sample = [0, 1, 31, 32, 500, 1023]
    dev, runs = run_both(P, O, J, h, 0, "i8", 1024, 120, 0.2, 1.0, 0.02, 0.6, 40, 11, sample=sample)
    say("geometry", dev["info"])
    assert dev["info"]["group"] > 1
    assert_parity(dev, runs)


def test_every_geometry_gives_identical_results(P, O):
    """Race check across tilings: every feasible launch geometry (replicas
    per block, workgroups per block, J in LDS or streamed) reproduces the
    same bit-exact run, which also matches the oracle on sampled replicas."""
    import os
    J, h = inst.sk_gauss_fixed(300, 21, frac_bits=5, bits=8)
    R, T = 70, 90
    ref = None
    ran = 0
    Ji, hi = int_units(J, h, 5)
    betas = O.beta_linear(0.05, 1.0, T)
    for mt in (1, 2):
        for G in (1, 2, 3, 5, 7, 10, 20):
            for jl in (1, 0):
                os.environ["PHIA_GEOMETRY"] = f"{mt},{G},{jl}"
                try:
                    p = P.Problem(J, h, path="i8")
                    try:
                        p.anneal(R, T, 0.2, 1.0, beta0=0.05, beta1=1.0, refresh_L=20, seed=8)
                    except P.PhiaError as e:
                        assert e.code == -4, str(e)  # geometry does not fit: skipped
                        continue
                    say("geometry", mt, G, jl, p.info())
                    got = p.replica_best() + p.get_state()[:2]
                    p.close()
                finally:
                    del os.environ["PHIA_GEOMETRY"]
                ran += 1
                if ref is None:
                    ref = got
                    for r in (0, 69):
                        o = O.anneal(Ji, hi, 5, 1, betas, 0.2, 1.0, 20, 8, r0=r)
                        assert got[0][r] == o.bestE[0] and np.array_equal(got[3][r], o.x[0])
                else:
                    for u, w in zip(ref, got):
                        assert np.array_equal(u, w), (mt, G, jl)
    assert ran >= 6


class _Geometry:
    """Force one launch geometry for the problems created inside the block."""

    def __init__(self, spec):
        self.spec = spec

    def __enter__(self):
        import os
        os.environ["PHIA_GEOMETRY"] = self.spec

    def __exit__(self, *exc):
        import os
        del os.environ["PHIA_GEOMETRY"]


def test_interleaved_group_sweep_full_parity(P, O):
    """Interleaved sub-block sweep (two 16-replica sub-blocks per workgroup,
    column split over G workgroups): every replica of a ragged case (N not a
    multiple of 16, R not a multiple of 32, refresh period not dividing T)
    bit-identical to the oracle, energy traces included through the records."""
    J, h = inst.sk_gauss_fixed(150, 5, frac_bits=5, bits=8)
    with _Geometry("pp,3"):
        dev, runs = run_both(P, O, J, h, 5, "i8", 45, 137, 0.2, 1.0, 0.05, 1.5, 23, 71, trace=False)
    say("geometry", dev["info"])
    assert dev["info"]["sweep_kernel"] == 1 and dev["info"]["group"] == 3
    assert_parity(dev, runs)


@pytest.mark.parametrize("path,geometry", [("i8", None), ("i8", "pp,3"), ("i8", "pp4,3"), ("i8", "ppg,3"),
                                           ("i8", "1,3,1"), ("fp32", None), ("ell", None), ("bf16hilo", None)])
def test_refresh_period_extremes(P, O, path, geometry):
    """The momentum refresh at its extremes: a fresh draw at every step
    (L = 1) and a single draw at step 0 (L > T), and the shortest anneals
    (one step, whose linear schedule is beta0 alone, and two), on every sweep
    kernel; ragged N and R, every replica bit-identical to the oracle."""
    J, h = inst.sk_pm1(150, 9)
    T = 40
    import contextlib
    for TT, L in ((T, 1), (T, T + 5), (1, 25), (2, 1)):
        with _Geometry(geometry) if geometry else contextlib.nullcontext():
            dev, runs = run_both(P, O, J, h, 0, path, 19, TT, 0.2, 1.0, 0.1, 2.0, L, 60 + L + TT,
                                 trace=not (geometry or "").startswith("pp"))  # no traces in the interleaved sweep
        say("geometry", path, geometry, TT, L, dev["info"]["sweep_kernel"], dev["info"]["group"])
        if geometry:
            assert dev["info"]["group"] == int(geometry.split(",")[1])
        assert_parity(dev, runs)
    # the persistent batch kernel, against single runs
    if path == "i8" and geometry is None:
        probs = [P.Problem(J, h, path="i8") for _ in range(2)]
        scheds = [dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=2.0, refresh_L=L) for L in (1, T + 5)]
        plan = P.Batch(probs, [19, 19], [T, T], scheds)
        assert [p.info()["sweep_kernel"] for p in probs] == [3, 3]
        plan.launch([71, 72])
        plan.sync()
        for p, sc, seed in zip(probs, scheds, (71, 72)):
            got = p.replica_best() + p.get_state()[:2]
            q = P.Problem(J, h, path="i8")
            q.anneal(19, T, 0.2, 1.0, beta0=0.1, beta1=2.0, refresh_L=sc["refresh_L"], seed=seed)
            ref = q.replica_best() + q.get_state()[:2]
            q.close()
            for u, w in zip(ref, got):
                assert np.array_equal(u, w), sc
        plan.close()
        for p in probs:
            p.close()


def test_interleaved_streamed_j_full_parity(P, O):
    """Interleaved sweep with the int8 J read from global memory at every
    product (no slice per member): the ragged case bit-identical to the
    oracle, and a run split into uneven chunks, in the other XCD placement,
    bit-identical to the one-launch run."""
    J, h = inst.sk_gauss_fixed(150, 5, frac_bits=5, bits=8)
    with _Geometry("ppg,3"):
        dev, runs = run_both(P, O, J, h, 5, "i8", 45, 137, 0.2, 1.0, 0.05, 1.5, 23, 71, trace=False)
    say("geometry", dev["info"])
    assert dev["info"]["sweep_kernel"] == 1 and dev["info"]["group"] == 3 and dev["info"]["j_in_lds"] == 0
    assert_parity(dev, runs)
    with _Geometry("ppg,4,0"):
        p = P.Problem(J, h, frac_bits=5, path="i8")
        p.start(45, 137, 0.2, 1.0, beta0=0.05, beta1=1.5, refresh_L=23, seed=71)
        for k in (1, 40, 96, 137):  # end steps of uneven chunks
            p.run(k)
        p.sync()
        info = p.info()
        E, S, K = p.replica_best()
        x, v, _ = p.get_state()
        p.close()
    assert info["j_in_lds"] == 0 and info["group"] == 4
    assert np.array_equal(E, dev["E"]) and np.array_equal(K, dev["K"]) and np.array_equal(S, dev["S"])
    assert np.array_equal(x.view(np.uint32), dev["x"].view(np.uint32))
    assert np.array_equal(v.view(np.uint32), dev["v"].view(np.uint32))


def test_interleaved_streamed_j_split_parity(P, O):
    """Streamed J at the size it is built for (N = 1990, G = 16: 32 k blocks
    per column block, 16 streamed by each team through the fragment ring and
    its tail): ragged columns and a partly filled second sub-block,
    bit-identical to the oracle."""
    J, h = inst.sk_gauss_fixed(1990, 7, frac_bits=5, bits=8)
    with _Geometry("ppg,16"):
        dev, runs = run_both(P, O, J, h, 5, "i8", 20, 40, 0.2, 1.0, 0.05, 1.5, 13, 73, trace=False)
    say("geometry", dev["info"])
    assert dev["info"]["sweep_kernel"] == 1 and dev["info"]["group"] == 16 and dev["info"]["j_in_lds"] == 0
    assert_parity(dev, runs)


def test_interleaved_geometries_and_chunks_identical(P, O):
    """Group sizes, several passes over the replica blocks per launch
    (R = 4096 on a 320-spin instance) and runs split into uneven chunks all
    give the run of the one-workgroup-per-block kernel, bit for bit."""
    J, h = inst.sk_gauss_fixed(300, 21, frac_bits=5, bits=8)
    R, T = 4096, 61
    sched = dict(beta0=0.05, beta1=1.0, refresh_L=20, seed=8)

    def once(spec, chunks=None):
        with _Geometry(spec):
            p = P.Problem(J, h, path="i8")
            if chunks is None:
                p.anneal(R, T, 0.2, 1.0, **sched)
            else:
                p.start(R, T, 0.2, 1.0, **sched)
                for k in chunks:
                    p.run(k)
                p.sync()
            info = p.info()
            got = p.replica_best() + p.get_state()[:2]
            p.close()
        say("geometry", spec, info)
        return info, got

    _, ref = once("1,2,1")
    for spec, chunks in (("pp,3", None), ("pp,10", None), ("pp,20", None), ("pp,5", [1, 2, 30, 61])):
        info, got = once(spec, chunks)
        assert info["sweep_kernel"] == 1
        for u, w in zip(ref, got):
            assert np.array_equal(u, w), spec
    Ji, hi = int_units(J, h, 5)
    betas = O.beta_linear(0.05, 1.0, T)
    for r in (0, 31, 32, 4095):
        o = O.anneal(Ji, hi, 5, 1, betas, 0.2, 1.0, 20, 8, r0=r)
        assert ref[0][r] == o.bestE[0] and np.array_equal(ref[3][r], o.x[0])


def test_interleaved_lds_resident_j_sampled(P, O):
    """Np > 1024: the interleaved kernel keeps each member's J slice in LDS
    instead of VGPRs.  Sampled replicas against the oracle, and the whole
    run against the one-block-per-workgroup kernel."""
    J, h = inst.sk_gauss_fixed(1100, 4, frac_bits=5, bits=8)
    R, T = 70, 45
    sample = [0, 16, 33, 69]
    with _Geometry("pp,12"):
        dev, runs = run_both(P, O, J, h, 5, "i8", R, T, 0.2, 1.0, 0.05, 1.0, 20, 5, trace=False, sample=sample)
    say("geometry", dev["info"])
    assert dev["info"]["sweep_kernel"] == 1 and dev["info"]["Np"] > 1024
    assert_parity(dev, runs)
    with _Geometry("1,12,0"):
        p = P.Problem(J, h, frac_bits=5, path="i8")
        p.anneal(R, T, 0.2, 1.0, beta0=0.05, beta1=1.0, refresh_L=20, seed=5)
        E, S, K = p.replica_best()
        x, v, _ = p.get_state()
        p.close()
    assert np.array_equal(E, dev["E"]) and np.array_equal(K, dev["K"]) and np.array_equal(S, dev["S"])
    assert np.array_equal(x.view(np.uint32), dev["x"].view(np.uint32))


def test_interleaved_fp4_operands(P, O):
    """Couplings whose integer codes are all FP4 values (0, +-1, +-2, +-3,
    +-4, +-6) run the interleaved kernel with FP4 MFMA operands: full parity
    with the oracle on a ragged case that uses every code, and bit-identical
    to the int8-operand kernel; a code outside the set leaves the FP4 variant
    unavailable."""
    rs = np.random.default_rng(12)
    N = 230
    codes = np.array([0, 1, -1, 2, -2, 3, -3, 4, -4, 6, -6])
    U = rs.choice(codes, size=(N, N)).astype(np.float64)
    J = np.triu(U, 1) + np.triu(U, 1).T
    h = rs.integers(-3, 4, N).astype(np.float64)
    R, T = 45, 97
    with _Geometry("pp4,3"):
        dev, runs = run_both(P, O, J, h, 0, "i8", R, T, 0.2, 1.0, 0.02, 0.5, 19, 23, trace=False)
    say("geometry", dev["info"])
    assert dev["info"]["sweep_kernel"] == 2
    assert_parity(dev, runs)
    with _Geometry("pp,3"):
        p = P.Problem(J, h, path="i8")
        p.anneal(R, T, 0.2, 1.0, beta0=0.02, beta1=0.5, refresh_L=19, seed=23)
        assert p.info()["sweep_kernel"] == 1
        E, S, K = p.replica_best()
        x, v, _ = p.get_state()
        p.close()
    assert np.array_equal(E, dev["E"]) and np.array_equal(K, dev["K"]) and np.array_equal(S, dev["S"])
    assert np.array_equal(x.view(np.uint32), dev["x"].view(np.uint32))
    assert np.array_equal(v.view(np.uint32), dev["v"].view(np.uint32))
    J5 = J.copy()
    J5[0, 1] = J5[1, 0] = 5.0
    with _Geometry("pp4,3"):
        p = P.Problem(J5, h, path="i8")
        with pytest.raises(P.PhiaError) as e:
            p.anneal(R, T, 0.2, 1.0, beta0=0.02, beta1=0.5, refresh_L=19, seed=23)
        assert e.value.code == -4
        p.close()


def test_interleaved_benchmark_shape_sampled(P, O):
    """Max-cut G(800, 0.06), 1024 replicas on the interleaved kernel with
    eight workgroups per block: sampled replicas against the oracle."""
    J, h = inst.er_maxcut(800, 0.06, 0)
    sample = [0, 15, 16, 31, 32, 511, 1023]
    for spec, kind, deriv in (("pp,8", 1, "tanh"), ("pp4,7", 2, "tanh"), ("pp4,7", 2, "poly2")):
        with _Geometry(spec):
            dev, runs = run_both(P, O, J, h, 0, "i8", 1024, 120, 0.2, 1.0, 0.02, 0.6, 40, 11, trace=False,
                                 sample=sample, deriv=deriv)
        say("geometry", dev["info"])
        assert dev["info"]["sweep_kernel"] == kind
        assert_parity(dev, runs)


def test_autotune_keeps_results(P, O):
    J, h = inst.er_maxcut(400, 0.05, 2)
    p = P.Problem(J, h, path="i8")
    us = p.autotune(96, 40)
    assert us > 0
    p.anneal(96, 150, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=25, seed=4)
    E, S, K = p.replica_best()
    say("tuned", p.info(), us)
    Ji, hi = int_units(J, h, 0)
    o = O.anneal(Ji, hi, 0, 1, O.beta_linear(0.1, 3.0, 150), 0.2, 1.0, 25, 4, r0=95)
    assert E[95] == o.bestE[0] and np.array_equal(S[95], o.bestS[0])
    p.close()


def test_batch_matches_single_runs_and_oracle(P, O):
    """Uneven-N batch (int8 and BF16 hi/lo, J in LDS and streamed, ragged
    replica counts, per-instance schedules and seeds) is bit-identical to
    annealing every instance alone, and to the oracle on sampled replicas."""
    specs = [
        ("sk", 17, "i8", 16, 120, 1), ("reg3", 64, "i8", 37, 90, 2), ("sk", 100, "bf16hilo", 32, 75, 3),
        ("fixed", 250, "i8", 20, 60, 4), ("reg3", 302, "i8", 33, 50, 5), ("sk", 400, "i8", 16, 40, 6),
        ("fixed", 512, "i8", 18, 30, 7), ("sk", 33, "bf16hilo", 5, 100, 8), ("fixed16", 130, "bf16hilo", 17, 40, 9),
    ]
    inst_list, probs, reps, steps, scheds, seeds = [], [], [], [], [], []
    for kind, N, path, R, T, seed in specs:
        if kind == "sk":
            J, h = inst.sk_pm1(N, seed)
        elif kind == "reg3":
            J, h = inst.regular3_pm1(N, seed)
        elif kind == "fixed":
            J, h = inst.sk_gauss_fixed(N, seed, frac_bits=5, bits=8)
        else:
            J, h = inst.sk_gauss_fixed(N, seed, frac_bits=12, bits=16)
        sc = dict(eps=0.2, gamma=1.0, beta0=0.05 * seed, beta1=1.0 + seed, refresh_L=10 + seed,
                  deriv="poly2" if seed % 2 else "tanh")
        inst_list.append((J, h))
        probs.append(P.Problem(J, h, path=path))
        reps.append(R)
        steps.append(T)
        scheds.append(sc)
        seeds.append(100 + seed)
    say("batch of", len(probs))
    P.batch_run(probs, reps, steps, scheds, seeds)
    for i, p in enumerate(probs):
        got = p.replica_best() + p.get_state()[:2]
        J, h = inst_list[i]
        q = P.Problem(J, h, path=specs[i][2])
        sc = scheds[i]
        q.anneal(reps[i], steps[i], sc["eps"], sc["gamma"], beta0=sc["beta0"], beta1=sc["beta1"],
                 refresh_L=sc["refresh_L"], seed=seeds[i], deriv=sc["deriv"])
        ref = q.replica_best() + q.get_state()[:2]
        for u, w in zip(ref, got):
            assert np.array_equal(u, w), specs[i]
        if i in (1, 4, 6):
            f = 5 if specs[i][0] == "fixed" else 0
            Ji, hi = int_units(J, h, f)
            o = O.anneal(Ji, hi, f, 1, O.beta_linear(sc["beta0"], sc["beta1"], steps[i]), sc["eps"], sc["gamma"],
                         sc["refresh_L"], seeds[i], r0=reps[i] - 1, deriv=sc["deriv"])
            assert got[0][-1] == o.bestE[0] and np.array_equal(got[3][-1], o.x[0]), specs[i]
        q.close()
        p.close()


def test_batch_fp4_edge_sizes(P, O):
    """The persistent FP4 batch kernel at its edges: a single spin with a
    field, N = 2, one column block (only wave 0 owns columns), 32 / 33 spins
    around a column-block boundary, 511 and the largest N = 512; one replica,
    a full 32-replica item, and 33 replicas (a second item with one real
    row).  Bit-identical to single runs, and to the oracle on the last
    replica of each instance."""
    specs = [(1, 1, 60), (2, 32, 45), (16, 33, 50), (32, 7, 40), (33, 32, 41), (511, 33, 23), (512, 1, 30)]
    insts, probs, reps, steps, scheds, seeds = [], [], [], [], [], []
    for i, (N, R, T) in enumerate(specs):
        J, h = inst.sk_pm1(N, 40 + i)
        h = np.asarray(h, np.float64).copy()
        h[: min(N, 3)] = [1.0, -1.0, 1.0][: min(N, 3)]  # non-zero fields, incl. the single spin's
        insts.append((J, h))
        probs.append(P.Problem(J, h, path="i8"))
        reps.append(R)
        steps.append(T)
        scheds.append(dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=2.5, refresh_L=7 + i,
                           deriv="poly2" if i % 3 == 2 else "tanh"))
        seeds.append(500 + i)
    plan = P.Batch(probs, reps, steps, scheds)
    kinds = [p.info()["sweep_kernel"] for p in probs]
    say("batch edge sizes, sweep kernels", kinds)
    assert kinds == [3] * len(specs)
    plan.launch(seeds)
    plan.sync()
    for i, p in enumerate(probs):
        got = p.replica_best() + p.get_state()[:2]
        J, h = insts[i]
        sc = scheds[i]
        q = P.Problem(J, h, path="i8")
        q.anneal(reps[i], steps[i], sc["eps"], sc["gamma"], beta0=sc["beta0"], beta1=sc["beta1"],
                 refresh_L=sc["refresh_L"], seed=seeds[i], deriv=sc["deriv"])
        ref = q.replica_best() + q.get_state()[:2]
        q.close()
        for u, w in zip(ref, got):
            assert np.array_equal(u, w), specs[i]
        Ji, hi = int_units(J, h, 0)
        o = O.anneal(Ji, hi, 0, 1, O.beta_linear(sc["beta0"], sc["beta1"], steps[i]), sc["eps"], sc["gamma"],
                     sc["refresh_L"], seeds[i], r0=reps[i] - 1, deriv=sc["deriv"])
        assert got[0][-1] == o.bestE[0] and got[2][-1] == o.bestStep[0], specs[i]
        assert np.array_equal(got[1][-1], o.bestS[0]), specs[i]
        assert np.array_equal(got[3][-1].view(np.uint32), o.x[0].view(np.uint32)), specs[i]
        assert np.array_equal(got[4][-1].view(np.uint32), o.v[0].view(np.uint32)), specs[i]
    plan.close()
    for p in probs:
        p.close()


def test_batch_plan_relaunch_and_ownership(P, O):
    """A batch plan built once and launched twice with different seeds: every
    instance bit-identical to annealing it alone with that seed, on the
    persistent FP4 sweep (every k-block count 1-4, workgroups with idle
    waves, single-buffered spins at Np = 512, partial 32-replica blocks)
    and on the one-item-per-workgroup sweep (8-bit couplings) in the same
    graph.  While the plan exists its problems refuse to anneal alone."""
    specs = [("sk", 40, 32), ("reg3", 100, 45), ("sk", 200, 16), ("reg3", 330, 64), ("sk", 450, 33),
             ("reg3", 470, 32), ("fixed", 150, 20), ("sk", 17, 5)]
    insts, probs = [], []
    for i, (kind, N, R) in enumerate(specs):
        if kind == "sk":
            J, h = inst.sk_pm1(N, 60 + i)
        elif kind == "reg3":
            J, h = inst.regular3_pm1(N, 60 + i)
        else:
            J, h = inst.sk_gauss_fixed(N, 60 + i, frac_bits=5, bits=8)
        insts.append((J, h))
        probs.append(P.Problem(J, h, path="i8"))
    reps = [R for _, _, R in specs]
    T = 150
    sched = [dict(eps=0.2, gamma=1.0, beta0=0.05, beta1=2.0 + i, refresh_L=23, deriv="poly2" if i == 3 else "tanh")
             for i in range(len(specs))]
    plan = P.Batch(probs, reps, [T] * len(specs), sched)
    kinds = [p.info()["sweep_kernel"] for p in probs]
    say("sweep kernels", kinds)
    assert kinds[:6] == [3] * 6 and kinds[6] == 0
    with pytest.raises(P.PhiaError) as e:
        probs[0].anneal(8, 10, 0.2, 1.0, beta0=0.1, beta1=1.0)
    assert e.value.code == -7
    for launch in range(2):
        seeds = [1000 * launch + 7 * i + 3 for i in range(len(specs))]
        plan.launch(seeds)
        plan.sync()
        for i, p in enumerate(probs):
            got = p.replica_best() + p.get_state()[:2]
            J, h = insts[i]
            q = P.Problem(J, h, path="i8")
            sc = sched[i]
            q.anneal(reps[i], T, sc["eps"], sc["gamma"], beta0=sc["beta0"], beta1=sc["beta1"],
                     refresh_L=sc["refresh_L"], seed=seeds[i], deriv=sc["deriv"])
            ref = q.replica_best() + q.get_state()[:2]
            q.close()
            for u, w in zip(ref, got):
                assert np.array_equal(u, w), (launch, specs[i])
        # one replica of the largest instance against the oracle
        J, h = insts[5]
        o = O.anneal(J.astype(np.int32), h.astype(np.int32), 0, 1, O.beta_linear(0.05, 7.0, T), 0.2, 1.0, 23,
                     seeds[5], r0=31)
        E, S, K = probs[5].replica_best()
        assert E[31] == o.bestE[0] and K[31] == o.bestStep[0] and np.array_equal(S[31], o.bestS[0])
    plan.close()
    probs[0].anneal(8, 10, 0.2, 1.0, beta0=0.1, beta1=1.0)  # released by the plan
    for p in probs:
        p.close()


def _serve_specs():
    out = []
    for i, (N, dense, R, T) in enumerate([(40, False, 32, 900), (120, True, 16, 1200), (300, False, 20, 700),
                                          (600, False, 32, 500), (90, True, 64, 400)]):
        J, h, E, t = inst.planted_loops(N, 50 + i, alpha=0.4, dense=dense)
        out.append((J, h, E, R, T, 77 + i))
    return out


def _serve(P, specs, max_slots, budget=1 << 36, chunk=100):
    sched = dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25)
    srv = P.Server(budget, max_slots=max_slots, chunk_steps=chunk)
    probs, tickets = [], []
    for J, h, E, R, T, seed in specs:
        p = P.Problem(J, h, path="i8")
        probs.append(p)
        tickets.append(srv.submit(p, R, T, E, seed=seed, **sched))
    res = [srv.wait(t, 120.0) for t in tickets]
    spins = [srv.spins(t) for t in tickets]
    srv.close()
    for p in probs:
        p.close()
    return res, spins


def test_server_result_same_alone_and_in_mix(P, O):
    """Continuous batching: every request gives the same result (energy,
    replica, steps used, success, best state) alone and in a mix of batched
    small instances and a column-split large one."""
    specs = _serve_specs()
    alone = [_serve(P, [sp], 1) for sp in specs]
    mix, mix_spins = _serve(P, specs, 8)
    for i, ((res1, sp1), r2, s2) in enumerate(zip(alone, mix, mix_spins)):
        r1 = res1[0]
        say("request", i, r1, r2)
        assert r1["state"] == P.REQ_DONE and r2["state"] == P.REQ_DONE
        for key in ("success", "energy_units", "replica", "steps_used"):
            assert r1[key] == r2[key], (i, key)
        assert np.array_equal(sp1[0], s2)
        J, h, E = specs[i][0], specs[i][1], specs[i][2]
        assert O.energy(J.astype(np.int32), h.astype(np.int32), s2) == r2["energy_units"]
        assert r2["energy_units"] >= E
        assert r2["success"] == (r2["energy_units"] <= E)
    # a request that ran its whole budget equals a plain anneal of that many steps
    J, h, E, R, T, seed = specs[3]
    if mix[3]["steps_used"] == T:
        p = P.Problem(J, h, path="i8")
        p.anneal(R, T, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=25, seed=seed)
        assert p.best_exact()[0] == mix[3]["energy_units"]
        p.close()


def test_server_valu_requests_overlap_same_alone_and_in_mix(P, O):
    """Requests on the VALU sweeps (ELL, FP32) run their own launches on the
    server's auxiliary streams, overlapped with each other and with the
    batched small instances, after the round's cooperative column-split
    launch: five of them (more than the three streams) in a mix with a
    batched and a column-split request give the same results as each request
    served alone."""
    specs = [  # (N, dense, path, R, T, seed)
        (700, False, "ell", 32, 600, 1), (300, True, "fp32", 16, 500, 2), (200, False, "ell", 24, 700, 3),
        (500, False, "ell", 16, 450, 4), (90, True, "fp32", 8, 800, 5), (40, False, "i8", 32, 600, 6),
        (700, False, "i8", 32, 500, 7),
    ]
    sched = dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25)
    inst_list = []
    for N, dense, path, R, T, seed in specs:
        J, h, E, _ = inst.planted_loops(N, 300 + seed, alpha=0.4, dense=dense)
        inst_list.append((J, h, E))

    def serve(idx, slots):
        srv = P.Server(1 << 36, max_slots=slots, chunk_steps=90)
        probs, tickets = [], []
        for i in idx:
            J, h, E = inst_list[i]
            N, dense, path, R, T, seed = specs[i]
            p = P.Problem(J, h, path=path)
            probs.append(p)
            tickets.append(srv.submit(p, R, T, E, seed=seed, **sched))
        res = [srv.wait(t, 120.0) for t in tickets]
        spins = [srv.spins(t) for t in tickets]
        kinds = [p.info()["sweep_kernel"] for p in probs]
        srv.close()
        for p in probs:
            p.close()
        return res, spins, kinds

    alone = [serve([i], 1) for i in range(len(specs))]
    mix, mix_spins, kinds = serve(list(range(len(specs))), 8)
    say("sweep kernels", kinds)
    assert sum(k == 4 for k in kinds) == 5
    for i in range(len(specs)):
        r1, s1 = alone[i][0][0], alone[i][1][0]
        r2, s2 = mix[i], mix_spins[i]
        say("request", i, specs[i][2], r1, r2)
        assert r1["state"] == P.REQ_DONE and r2["state"] == P.REQ_DONE
        for key in ("success", "energy_units", "replica", "steps_used"):
            assert r1[key] == r2[key], (i, key)
        assert np.array_equal(s1, s2), i
        J, h, E = inst_list[i]
        assert O.energy(J.astype(np.int32), h.astype(np.int32), s2) == r2["energy_units"]
        assert r2["energy_units"] >= E and r2["success"] == (r2["energy_units"] <= E)


def test_server_read_out_of_more_than_64_requests(P, O):
    """80 requests running at once (100 slots): the round's batched argmin
    takes them in launches of 64 and 16; every result's energy is the Eq. 2
    energy of the state it returns, and sampled requests equal the same
    request served alone."""
    sched = dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25)
    specs = []
    for i in range(80):
        J, h = inst.sk_pm1(20 + (i % 7), 500 + i)
        specs.append((J, h, 8 + (i % 3), 600, 900 + i))

    def serve(idx, slots):
        srv = P.Server(1 << 36, max_slots=slots, chunk_steps=60)
        probs = [P.Problem(specs[i][0], specs[i][1], path="i8") for i in idx]
        tickets = []  # submitted together, so that the requests' ten rounds overlap
        for i, p in zip(idx, probs):
            J, h, R, T, seed = specs[i]
            tickets.append(srv.submit(p, R, T, -10**9, seed=seed, **sched))  # unreachable target: full budget
        res = [srv.wait(t, 120.0) for t in tickets]
        spins = [srv.spins(t) for t in tickets]
        srv.close()
        for p in probs:
            p.close()
        return res, spins

    res, spins = serve(range(80), 100)
    for (J, h, R, T, seed), r, sp in zip(specs, res, spins):
        assert r["state"] == P.REQ_DONE and r["steps_used"] == T and not r["success"]
        assert O.energy(J.astype(np.int32), h.astype(np.int32), sp) == r["energy_units"]
    for i in (0, 63, 64, 79):
        (r1,), (s1,) = serve([i], 1)
        for key in ("energy_units", "replica", "steps_used"):
            assert r1[key] == res[i][key], (i, key)
        assert np.array_equal(s1, spins[i]), i


def test_server_column_split_requests_share_launches(P, O):
    """Large requests (column-split geometries) of several sizes and replica
    counts run together, several per cooperative launch; with an unreachable
    target each runs its whole budget and must equal a plain anneal of that
    many steps (best energy, replica, best state), and the oracle on a
    sampled replica."""
    specs = []
    for i, (N, R, T) in enumerate([(600, 32, 300), (777, 48, 250), (1000, 16, 200), (700, 64, 260)]):
        J, h, E, t = inst.planted_loops(N, 90 + i, alpha=0.4, dense=(i % 2 == 1))
        specs.append((J, h, -(1 << 60), R, T, 300 + i))
    res, spins = _serve(P, specs, 8, chunk=90)
    for i, (J, h, _, R, T, seed) in enumerate(specs):
        r = res[i]
        say("request", i, r)
        assert r["state"] == P.REQ_DONE and r["steps_used"] == T and not r["success"]
        p = P.Problem(J, h, path="i8")
        p.anneal(R, T, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=25, seed=seed)
        E, S, K = p.replica_best()
        info = p.info()
        p.close()
        say("plain", info)
        assert r["energy_units"] == E.min() and r["replica"] == int(np.argmin(E))
        assert np.array_equal(spins[i], S[r["replica"]])
        Ji, hi = int_units(J, h, 0)
        o = O.anneal(Ji, hi, 0, 1, O.beta_linear(0.1, 3.0, T), 0.2, 1.0, 25, seed, r0=R - 1)
        assert E[R - 1] == o.bestE[0]


def test_server_budget_forces_queueing_and_cancel(P, O):
    specs = []
    for i in range(3):
        J, h, E, t = inst.planted_loops(100, 200 + i, alpha=0.4)
        specs.append((J, h, E, 16, 300, 5 + i))
    sched = dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25)
    probs = [P.Problem(J, h, path="i8") for J, h, E, R, T, s in specs]
    # budget below any two footprints: requests run one after another
    fps = [P.server_footprint(p, R, T) for p, (J, h, E, R, T, s) in zip(probs, specs)]
    assert max(fps) < min(fps) * 2
    srv = P.Server(int(max(fps) * 1.2), max_slots=8, chunk_steps=100)
    tickets = [srv.submit(p, R, T, -10**9, seed=s, **sched) for p, (J, h, E, R, T, s) in zip(probs, specs)]
    res = [srv.wait(t, 120.0) for t in tickets]
    for a, b in zip(res, res[1:]):
        assert b["t_admit"] >= a["t_done"]
    assert all(r["state"] == P.REQ_DONE and r["success"] == 0 for r in res)
    srv.close()
    # cancel a long running request; the other one is unaffected
    srv = P.Server(1 << 36, max_slots=8, chunk_steps=50)
    t_long = srv.submit(probs[0], 32, 200000, -10**9, seed=1, **sched)
    t_short = srv.submit(probs[1], 16, 300, -10**9, seed=2, **sched)
    r_short = srv.wait(t_short, 60.0)
    srv.cancel(t_long)
    r_long = srv.wait(t_long, 60.0)
    assert r_long["state"] == P.REQ_CANCELLED and r_long["steps_used"] < 200000
    srv.close()
    ref = _serve(P, [(specs[1][0], specs[1][1], -10**9, 16, 300, 2)], 1, chunk=50)[0][0]
    assert r_short["state"] == P.REQ_DONE
    assert ref["energy_units"] == r_short["energy_units"] and ref["steps_used"] == r_short["steps_used"]
    for p in probs:
        p.close()


# ------------------------------------------------------ maximum sizes ----
@pytest.mark.parametrize("path,N,R,T", [("i8", 5056, 17, 6), ("bf16hilo", 2496, 16, 6), ("fp32", 4096, 5, 4)])
def test_largest_instance_per_path(P, O, path, N, R, T):
    """The largest N each path holds (int8 5056, BF16 hi/lo 2496, FP32
    4096), ragged replica count: every replica bit-identical to the oracle."""
    if path == "bf16hilo":
        J, h = inst.sk_gauss_fixed(N, 3, frac_bits=12, bits=16)
        f = 12
    else:
        J, h = inst.sk_pm1(N, 3)
        f = 0
    say(f"largest {path} N={N}")
    prob = P.Problem(J, h, frac_bits=f, path=path)
    prob.anneal(R, T, 0.2, 1.0, beta0=0.5, beta1=2.0, refresh_L=3, seed=21)
    E, S, K = prob.replica_best()
    x, v, _ = prob.get_state()
    info = prob.info()
    prob.close()
    say("geometry", info)
    Ji, hi = int_units(J, h, f)
    betas = O.beta_linear(0.5, 2.0, T)
    o = O.anneal(Ji, hi, f, R, betas, 0.2, 1.0, 3, 21, threads=8)
    assert np.array_equal(x.view(np.uint32), o.x.view(np.uint32))
    assert np.array_equal(v.view(np.uint32), o.v.view(np.uint32))
    assert np.array_equal(E, o.bestE) and np.array_equal(K, o.bestStep) and np.array_equal(S, o.bestS)


# -------------------------------------- the other workloads at full size ----
@pytest.mark.parametrize("path,geometry", [("i8", None), ("i8", "1,8,0,2"), ("i8", "ppg,16,0"), ("i8", "ppg,16,1"),
                                           ("bf16hilo", None)])
def test_sk2000_full_shape_sampled(P, O, path, geometry):
    """Dense SK N = 2000 on the 2^-5 grid (8-bit couplings), 512 replicas:
    the full instance and replica count (short run), in the default launch
    geometry and in the one the profile measured; sampled replicas against
    the oracle."""
    import os
    J, h = inst.sk_gauss_fixed(2000, 0, frac_bits=5, bits=8)
    R, T = 512, 120
    say(f"sk2000 path={path} geometry={geometry}")
    if geometry:
        os.environ["PHIA_GEOMETRY"] = geometry
    try:
        p = P.Problem(J, h, path=path)
        p.anneal(R, T, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=25, seed=77)
    finally:
        os.environ.pop("PHIA_GEOMETRY", None)
    E, S, K = p.replica_best()
    x, v, _ = p.get_state()
    info = p.info()
    say("geometry", info)
    p.close()
    if geometry and geometry.startswith("ppg"):
        assert info["sweep_kernel"] == 1 and info["j_in_lds"] == 0 and info["group"] == 16
    Ji, hi = int_units(J, h, 5)
    betas = O.beta_linear(0.1, 3.0, T)
    for r in (0, 255, 511):
        o = O.anneal(Ji, hi, 5, 1, betas, 0.2, 1.0, 25, 77, r0=r)
        assert np.array_equal(x[r].view(np.uint32), o.x[0].view(np.uint32)), r
        assert E[r] == o.bestE[0] and K[r] == o.bestStep[0] and np.array_equal(S[r], o.bestS[0]), r


def _batch4096():
    """The 4096-instance batch workload: N uniform in [32, 512], even ids SK
    +-1, odd ids 3-regular +-1 with h in {-1, 0, 1}."""
    g = inst.rng(0)
    sizes = g.integers(32, 513, size=4096)
    out = []
    for i, n in enumerate(sizes):
        n = int(n)
        out.append(inst.sk_pm1(n, 10_000 + i) if i % 2 == 0 else inst.regular3_pm1(n + (n % 2), 10_000 + i))
    return out


def test_batch_full_size_sampled(P, O):
    """All 4096 instances in one graph (32 replicas each, short run); sampled
    instances and replicas against the oracle, and every instance's best
    state has the energy it reports."""
    insts = _batch4096()
    T = 40
    sched = dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25)
    probs = [P.Problem(J, h, path="i8") for J, h in insts]
    say("batch of", len(probs))
    P.batch_run(probs, [32] * len(probs), [T] * len(probs), [sched] * len(probs), list(range(5000, 5000 + len(probs))))
    betas = O.beta_linear(0.1, 3.0, T)
    for i in (0, 1, 777, 2048, 4094, 4095):
        J, h = insts[i]
        Ji, hi = J.astype(np.int32), h.astype(np.int32)
        E, S, K = probs[i].replica_best()
        x, v, _ = probs[i].get_state()
        for r in (0, 13, 16, 31):
            o = O.anneal(Ji, hi, 0, 1, betas, 0.2, 1.0, 25, 5000 + i, r0=r)
            assert E[r] == o.bestE[0] and K[r] == o.bestStep[0], (i, r)
            assert np.array_equal(S[r], o.bestS[0]), (i, r)
            assert np.array_equal(x[r].view(np.uint32), o.x[0].view(np.uint32)), (i, r)
            assert np.array_equal(v[r].view(np.uint32), o.v[0].view(np.uint32)), (i, r)
    for i in range(0, len(probs), 97):
        e, s = probs[i].best()
        J, h = insts[i]
        assert O.energy(J.astype(np.int32), h.astype(np.int32), s) == round(e), i
    for p in probs:
        p.close()


def test_serving_full_stream_energies(P, O):
    """The serving workload's 60 requests (N log-uniform in [100, 4000], dense
    and sparse, integer and fixed point): every result's energy is the Eq. 2
    energy of the state it returns, success means reaching the planted
    energy, and no result lies below the planted ground state.  The three
    smallest requests are also replayed on the oracle for the steps they
    used: the served record (lowest energy over the replicas, lowest replica
    on ties, and its spins) is the oracle's (App. B, Table 3, state 5)."""
    import time
    g = inst.rng(0)
    n = 60
    sizes = np.rint(np.exp(g.uniform(np.log(100), np.log(4000), size=n))).astype(int)
    srv = P.Server(1 << 36, max_slots=64, chunk_steps=500)
    sched = dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25)
    reqs = []
    for i in range(n):
        J, h, E, _ = inst.planted_loops(int(sizes[i]), 20_000 + i, alpha=0.4, dense=(i % 2 == 1))
        f = 0
        if (i // 2) % 2 == 1:
            J, f = J / 16.0, 4
        p = P.Problem(J, h, frac_bits=f, path="i8")
        # energies in grid units: the fixed-point copy J / 16 on the 2^-4 grid
        # has the integer instance's units, so E is the target either way
        t = srv.submit(p, 64, 20000, E, seed=900 + i, **sched)
        reqs.append((p, t, J, h, E, f))
    say("submitted", n)
    smallest = set(np.argsort(sizes, kind="stable")[:3].tolist())
    betas = O.beta_linear(sched["beta0"], sched["beta1"], 20000)
    for i, (p, t, J, h, E, f) in enumerate(reqs):
        r = srv.wait(t, 300.0)
        assert r["state"] == P.REQ_DONE, r
        s = srv.spins(t)
        Ji = np.rint(J * (1 << f)).astype(np.int32)
        hi = np.rint(h * (1 << f)).astype(np.int32)
        e = O.energy(Ji, hi, s)
        assert e == r["energy_units"]
        assert e >= E and r["success"] == (e <= E)
        if i in smallest:
            o = O.anneal(Ji, hi, f, 64, betas, sched["eps"], sched["gamma"], sched["refresh_L"], 900 + i,
                         k1=int(r["steps_used"]), threads=8)
            rs = int(np.argmin(o.bestE))  # first index of the minimum
            say("replayed request", i, "N", J.shape[0], "steps", r["steps_used"], "replica", rs)
            assert o.bestE[rs] == r["energy_units"] and rs == r["replica"], (i, rs, r)
            assert np.array_equal(o.bestS[rs], s), i
    srv.close()
    for p, *_ in reqs:
        p.close()


def test_xcd_placements_identical(P, O):
    """Column-split groups with all members on one XCD and with member m of
    every group on XCD m (J streamed or in LDS): bit-identical runs, which
    match the oracle on sampled replicas."""
    import os
    J, h = inst.sk_gauss_fixed(300, 9, frac_bits=5, bits=8)
    R, T = 256, 60
    ref = None
    for geo in ("1,8,0,2,0", "1,8,0,2,1", "1,8,1,2,0", "1,8,1,2,1", "2,16,0,1,0"):
        os.environ["PHIA_GEOMETRY"] = geo
        try:
            p = P.Problem(J, h, path="i8")
            p.anneal(R, T, 0.2, 1.0, beta0=0.05, beta1=1.0, refresh_L=20, seed=4)
        finally:
            del os.environ["PHIA_GEOMETRY"]
        info = p.info()
        say("geometry", geo, info)
        got = p.replica_best() + p.get_state()[:2]
        p.close()
        assert info["group"] in (8, 16)
        assert info["group_on_one_xcd"] == int(geo[-1])
        if ref is None:
            ref = got
        else:
            for u, w in zip(ref, got):
                assert np.array_equal(u, w), geo
    Ji, hi = int_units(J, h, 5)
    for r in (0, 255):
        o = O.anneal(Ji, hi, 5, 1, O.beta_linear(0.05, 1.0, T), 0.2, 1.0, 20, 4, r0=r)
        assert ref[0][r] == o.bestE[0] and np.array_equal(ref[3][r], o.x[0])
