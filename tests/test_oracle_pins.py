"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a third-party implementation
(numpy's Philox), FP64 libm within a stated error bound, a closed form, an
exact identity of Eq. 2 / Eq. 6, or an invariance of the sweep's arithmetic.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2407_10205_amd import instances as inst

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ulp32(x):
    return float(np.spacing(np.float32(abs(x))))


# --------------------------------------------------------------- RNG -----
@pytest.mark.parametrize("key,counter", [
    ((0, 0), (0, 0, 0, 0)),
    ((5, 0), (7, 3, 2, 1)),
    ((0xDEADBEEFCAFEF00D, 0), (41, 12345, 77, 1)),
    ((1, 0), (2**64 - 1, 9, 0, 0)),          # carry into word 1
    ((2**64 - 1, 0), (2**64 - 1, 2**64 - 1, 5, 0)),  # carry into word 2
])
def test_philox_matches_numpy(O, key, counter):
    """numpy.random.Philox is Philox4x64-10; it increments its counter before
    each block, so the block for counter c is numpy's first block at c - 1."""
    c = list(counter)
    words = c[0] + (c[1] << 64) + (c[2] << 128) + (c[3] << 192)
    prev = (words - 1) % (1 << 256)
    prev_c = [(prev >> (64 * m)) & (2**64 - 1) for m in range(4)]
    g = np.random.Philox(key=np.array(key, dtype=np.uint64),
                         counter=np.array(prev_c, dtype=np.uint64))
    ref = g.random_raw(4).astype(np.uint64)
    got = O.philox(np.array(c, dtype=np.uint64), np.array(key, dtype=np.uint64))
    assert np.array_equal(got, ref)


def test_uniform_open_interval_and_mirror(O):
    """u(w) lies in (0,1) on the 2^-24 grid and u(w) + u(~w) = 1 exactly."""
    rs = np.random.default_rng(1)
    ws = np.concatenate([[0, 1, 511, 512, 2**31, 2**32 - 1], rs.integers(0, 2**32, 2000)])
    for w in ws:
        u = float(O.uniform(int(w)))
        assert 0.0 < u < 1.0
        assert u * 2**24 == math.floor(u * 2**24)
        assert float(O.uniform(int(w))) + float(O.uniform(int(w) ^ 0xFFFFFFFF)) == 1.0
    assert float(O.uniform(0)) == 2.0**-24
    assert float(O.uniform(2**32 - 1)) == 1.0 - 2.0**-24


# ---------------------------------------------------------- fmath --------
def test_exp_within_2ulp_of_libm(O):
    ys = np.concatenate([np.linspace(-80, 0, 8001), -np.logspace(-8, 1.9, 2000)]).astype(np.float32)
    worst = max(abs(float(O.exp_nonpos(y)) - math.exp(float(y))) / ulp32(math.exp(float(y))) for y in ys)
    assert worst <= 2.0
    assert float(O.exp_nonpos(0.0)) == 1.0
    assert float(O.exp_nonpos(-81.0)) == 0.0


def test_ln_within_3ulp_of_libm(O):
    us = np.concatenate([np.linspace(2**-24, 1 - 2**-24, 8001),
                         np.logspace(-7.2, -1e-7, 2000)]).astype(np.float32)
    worst = max(abs(float(O.ln_unit(u)) - math.log(float(u))) / ulp32(math.log(float(u))) for u in us)
    assert worst <= 3.0


def test_sincos_2pi_abs_error_and_quarter_turns(O):
    us = np.linspace(2**-24, 1 - 2**-24, 8001).astype(np.float32)
    worst = 0.0
    for u in us:
        c, s = O.sincos_2pi(u)
        worst = max(worst, abs(float(c) - math.cos(2 * math.pi * float(u))),
                    abs(float(s) - math.sin(2 * math.pi * float(u))))
    assert worst <= 2.0**-23
    # quarter turns are exact: theta reduces to 0
    for u, (ce, se) in [(0.25, (0.0, 1.0)), (0.5, (-1.0, 0.0)), (0.75, (0.0, -1.0))]:
        c, s = O.sincos_2pi(u)
        assert (float(c), float(s)) == (ce, se)


def test_sech2_within_6ulp_and_even(O):
    us = np.concatenate([np.linspace(-40, 40, 16001), np.linspace(-1e-3, 1e-3, 1001)]).astype(np.float32)
    worst = 0.0
    for u in us:
        ref = 1.0 / math.cosh(float(u)) ** 2
        got = float(O.sech2(u))
        worst = max(worst, abs(got - ref) / ulp32(ref))
        assert got == float(O.sech2(-u))
    assert worst <= 6.0
    assert float(O.sech2(0.0)) == 1.0
    # -2|u| is clamped at -80: a constant tail of 4 e^-80 (1 + O(e^-80))
    tail = float(O.sech2(40.0))
    assert abs(tail - 4.0 * math.exp(-80.0)) <= 4 * ulp32(tail)
    assert float(O.sech2(41.0)) == tail and float(O.sech2(-1e4)) == tail


def test_gauss_is_standard_normal(O):
    """Mean, variance and a Kolmogorov-Smirnov test over 2e5 draws."""
    from scipy import stats
    z = np.array([O.gauss(42, 1, r, 3, i) for r in range(200) for i in range(1000)], np.float64)
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_gauss_box_muller_pairing(O):
    """Draws 2p and 2p+1 share one word pair: z0^2 + z1^2 = -2 ln u_a and
    atan2(z1, z0) = 2 pi u_b (checked in FP64 against numpy's Philox words)."""
    seed, tag, r, rnd = 9, 1, 4, 2
    for q in range(3):
        g = np.random.Philox(key=np.array([seed, 0], np.uint64),
                             counter=np.array([q - 1 if q else 2**64 - 1, rnd - (0 if q else 1), r, tag],
                                              np.uint64))
        out = g.random_raw(4)
        for p in range(4):
            wa, wb = int(out[p]) & 0xFFFFFFFF, int(out[p]) >> 32
            ua = (2 * (wa >> 9) + 1) / 2**24
            ub = (2 * (wb >> 9) + 1) / 2**24
            i0 = 8 * q + 2 * p
            z0 = float(O.gauss(seed, tag, r, rnd, i0))
            z1 = float(O.gauss(seed, tag, r, rnd, i0 + 1))
            assert abs(z0 * z0 + z1 * z1 + 2 * math.log(ua)) < 1e-5 * (1 - 2 * math.log(ua))
            ang = math.atan2(z1, z0) / (2 * math.pi) % 1.0
            d = abs(ang - ub)
            assert min(d, 1 - d) < 1e-5


# --------------------------------------------------- energy / field -----
def _golden_J(case):
    N = case["N"]
    J = np.zeros((N, N), np.int32)
    if case["edges"] == "complete":
        J[:] = case["J"]
        np.fill_diagonal(J, 0)
    elif case["edges"] == "cycle":
        for i in range(N):
            J[i, (i + 1) % N] = J[(i + 1) % N, i] = case["J"]
    h = case["h"]
    h = np.array(h if isinstance(h, list) else [h] * N, np.int32)
    return J, h


def test_bruteforce_closed_forms(O):
    with open(os.path.join(GOLDEN, "closed_form_ground_states.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        J, h = _golden_J(case)
        e, s = O.bruteforce(J, h)
        assert e == case["ground"], case["name"]
        assert O.energy(J, h, s) == e


def test_energy_hand_values(O):
    J = np.array([[0, 3], [3, 0]], np.int32)
    h = np.array([1, -2], np.int32)
    # E = -3 s0 s1 - s0 + 2 s1
    for s0 in (1, -1):
        for s1 in (1, -1):
            assert O.energy(J, h, np.array([s0, s1], np.int8)) == -3 * s0 * s1 - s0 + 2 * s1


def test_field_identities(O):
    """E = -1/2 sum s_i (I_i + h_i) and flipping spin i changes E by 2 s_i I_i."""
    rs = np.random.default_rng(3)
    for N in (1, 2, 7, 31):
        Jf, hf = inst.sk_gauss_fixed(N, 11 + N, frac_bits=3)
        J = np.rint(Jf * 8).astype(np.int32)
        h = np.rint(hf * 8).astype(np.int32)
        for _ in range(5):
            s = rs.choice(np.array([-1, 1], np.int8), size=N)
            I = O.local_field(J, h, s)
            E = O.energy(J, h, s)
            assert 2 * E == -int(np.sum(s.astype(np.int64) * (I.astype(np.int64) + h)))
            for i in range(N):
                t = s.copy()
                t[i] = -t[i]
                assert O.energy(J, h, t) - E == 2 * int(s[i]) * int(I[i])


def test_energy_f64_matches_integer_energy_on_grid(O):
    Jf, hf = inst.sk_gauss_fixed(40, 5, frac_bits=5)
    J = np.rint(Jf * 32).astype(np.int32)
    h = np.rint(hf * 32).astype(np.int32)
    s = np.random.default_rng(0).choice(np.array([-1, 1], np.int8), size=40)
    assert O.energy_f64(Jf, hf, s) == O.energy(J, h, s) / 32.0


# ----------------------------------------------------------- packing -----
def test_pack_validation_and_grid(O):
    J = np.array([[0, 0.5], [0.5, 0]])
    rc, Ji, hi, f = O.pack(J, np.array([0.25, -1.0]))
    assert rc == 0 and f == 2 and Ji[0, 1] == 2 and list(hi) == [1, -4]
    assert O.pack(np.array([[0, 1.0], [2.0, 0]]))[0] == -2
    assert O.pack(np.array([[1.0, 0], [0, 0]]))[0] == -3
    assert O.pack(np.array([[0, 0.3], [0.3, 0]]), frac_bits=2)[0] == -4
    # round half to even on the grid: 0.125 * 4 = 0.5 -> 0, 0.375 * 4 = 1.5 -> 2
    rc, Ji, _, f = O.pack(np.array([[0, 0.125], [0.125, 0]]), frac_bits=2, quantize=1)
    assert rc == 0 and Ji[0, 1] == 0
    rc, Ji, _, f = O.pack(np.array([[0, 0.375], [0.375, 0]]), frac_bits=2, quantize=1)
    assert rc == 0 and Ji[0, 1] == 2


def test_beta_linear(O):
    b = O.beta_linear(0.1, 3.0, 1000)
    assert b[0] == np.float32(0.1) and b[-1] == np.float32(3.0)
    assert np.all(np.diff(b) > 0)
    assert O.beta_linear(0.7, 9.0, 1)[0] == np.float32(0.7)


# -------------------------------------------------------- the sweep -----
def _c1():
    J, h = inst.sk_pm1(16, 0)
    return J.astype(np.int32), h.astype(np.int32)


def test_c1_reaches_bruteforce_ground_state(O):
    """SK N=16 (uniform +-1): 64 replicas x 1000 steps reach the exhaustive
    minimum over all 2^16 states, and no replica reports anything lower."""
    J, h = _c1()
    Eg, _ = O.bruteforce(J, h)
    betas = O.beta_linear(0.1, 3.0, 1000)
    run = O.anneal(J, h, 0, 64, betas, 0.2, 1.0, 50, 1234, threads=4)
    assert run.bestE.min() == Eg
    assert np.all(run.bestE >= Eg)
    assert np.mean(run.bestE == Eg) > 0.5


def test_best_tracking_matches_trace_and_eq2(O):
    J, h = _c1()
    betas = O.beta_linear(0.1, 3.0, 300)
    run = O.anneal(J, h, 0, 8, betas, 0.2, 1.0, 50, 7, trace=True)
    for r in range(8):
        tr = run.Etrace[r]
        assert run.bestE[r] == tr.min()
        assert run.bestStep[r] == int(np.argmin(tr))
        assert O.energy(J, h, run.bestS[r]) == run.bestE[r]


# -------------------------------------------------- final argmin -----
I64MAX = np.iinfo(np.int64).max


@pytest.mark.parametrize("bestE,want", [
    ([5], 0),                                   # one replica
    ([I64MAX], 0),                              # one replica without a record
    ([I64MAX, I64MAX, I64MAX], 0),              # no replica has a record: the first
    ([I64MAX, -3, I64MAX], 1),                  # records beat the empty rows
    ([-7, -9, -9, -8, -9], 1),                  # three-way tie: the lowest index
    ([4, 3, 2, 1, 0, -1], 5),                   # minimum in the last row
    ([-(2**62), 2**62, -(2**62) + 1], 0),       # full int64 range, no overflow
    ([0, -1, I64MAX, -1, -2, -2], 4),           # tie after the first minimum
])
def test_argmin_hand_cases(O, bestE, want):
    """Final choice of the reported configuration (App. B, Table 3, state 5:
    the best result so far; ties over replicas take the lowest index): hand
    cases covering ties, rows that never recorded an energy and R = 1."""
    assert O.argmin(np.array(bestE, np.int64)) == want


def test_argmin_matches_numpy_first_occurrence(O):
    """numpy.argmin returns the first occurrence of the minimum: on random
    arrays with many ties it must agree with the oracle everywhere."""
    rs = np.random.default_rng(11)
    for R in (1, 2, 3, 63, 64, 65, 255, 256, 257, 1000, 4096):
        for _ in range(20):
            E = rs.integers(-4, 3, size=R).astype(np.int64)
            E[rs.random(R) < 0.1] = I64MAX
            assert O.argmin(E) == int(np.argmin(E)), (R, E)


def test_argmin_of_an_anneal_reports_a_ground_state(O):
    """SK N = 16 after an anneal: many replicas tie at the exhaustive ground
    energy, and the chosen one is the first of them."""
    J, h = _c1()
    Eg, _ = O.bruteforce(J, h)
    betas = O.beta_linear(0.1, 3.0, 1000)
    run = O.anneal(J, h, 0, 64, betas, 0.2, 1.0, 50, 1234, threads=4)
    r = O.argmin(run.bestE)
    ties = np.nonzero(run.bestE == Eg)[0]
    assert ties.size > 1 and r == ties[0]
    assert O.energy(J, h, run.bestS[r]) == Eg


def test_harmonic_closed_form(O):
    """J = h = 0: each coordinate follows (x, v) <- (x + eps v, v - eps (x + eps v)),
    i.e. powers of [[1, eps], [-eps, 1 - eps^2]] (A7 with grad H = x)."""
    N, R, eps = 5, 3, 0.125
    J = np.zeros((N, N), np.int32)
    h = np.zeros(N, np.int32)
    T = 400
    betas = np.full(T, 1.0, np.float32)
    run = O.Run(N, R)
    rs = np.random.default_rng(5)
    run.x[:] = rs.standard_normal((R, N)).astype(np.float32)
    run.v[:] = rs.standard_normal((R, N)).astype(np.float32)
    run.bestE[:] = np.iinfo(np.int64).max
    x0, v0 = run.x.astype(np.float64).copy(), run.v.astype(np.float64).copy()
    O.anneal(J, h, 0, R, betas, eps, 1.0, 10**9, 0, k0=1, k1=T, run=run)
    M = np.array([[1.0, eps], [-eps, 1.0 - eps * eps]])
    Mk = np.linalg.matrix_power(M, T - 1)
    xr = Mk[0, 0] * x0 + Mk[0, 1] * v0
    vr = Mk[1, 0] * x0 + Mk[1, 1] * v0
    scale = np.abs(x0) + np.abs(v0)
    assert np.max(np.abs(run.x - xr) / scale) < 1e-4
    assert np.max(np.abs(run.v - vr) / scale) < 1e-4


def _leapfrog_closed_form(x0, v0, eps, n, center=0.0):
    """Stormer-Verlet leapfrog for x'' = center - x started with a half kick:
    x_n = c + (x0 - c) cos(n t) + (eps v0 / sin t) sin(n t), cos t = 1 - eps^2 / 2
    (x_1 = x0 + eps (v0 + eps (c - x0) / 2) fixes the sine coefficient)."""
    t = math.acos(1.0 - eps * eps / 2.0)
    return center + (x0 - center) * np.cos(n * t) + (eps * v0 / math.sin(t)) * np.sin(n * t)


def _ikick_draws(O, seed, R, N, rnd):
    return np.array([[O.gauss(seed, 1, r, rnd, i) for i in range(N)] for r in range(R)], np.float64)


def test_initial_kick_is_a_leapfrog_harmonic(O):
    """Initial-kick variant (Table 3, state 2), J = h = 0: one trajectory
    from the drawn x0 and momentum v0 follows the leapfrog closed form for
    every step count, and the returned momentum is the half-step one,
    (x_{n+1} - x_n) / eps.  Without the half kick (A7 alone) the same run
    misses the closed form."""
    N, R, eps, seed = 4, 3, 0.2, 17
    J = np.zeros((N, N), np.int32)
    h = np.zeros(N, np.int32)
    x0 = np.array([[O.gauss(seed, 0, r, 0, i) for i in range(N)] for r in range(R)], np.float64)
    v0 = _ikick_draws(O, seed, R, N, 0)
    for T in (1, 2, 7, 50):
        betas = np.full(T, 1.0, np.float32)
        run = O.anneal(J, h, 0, R, betas, eps, 1.0, 10**9, seed, ikick=True)
        xr = _leapfrog_closed_form(x0, v0, eps, T)
        vr = (_leapfrog_closed_form(x0, v0, eps, T + 1) - xr) / eps
        assert np.max(np.abs(run.x - xr)) < 2e-5 * T, T
        assert np.max(np.abs(run.v - vr)) < 2e-5 * T, T
    plain = O.anneal(J, h, 0, R, np.full(50, 1.0, np.float32), eps, 1.0, 10**9, seed)
    assert np.max(np.abs(plain.x - _leapfrog_closed_form(x0, v0, eps, 50))) > 1e-2


def test_initial_kick_every_trajectory_and_field_term(O):
    """The half kick opens every trajectory of L steps (fresh momentum of
    round m, chained closed forms), and it carries the field: with J = 0,
    h = 1 unit, c = beta gamma sigma = 1 (beta = 2^20, gamma = 2^-20, where
    sech^2 = 1 in FP32) the force is 1 - x, a leapfrog about x = 1."""
    N, R, eps, seed, L, T = 3, 2, 0.25, 5, 20, 60
    J = np.zeros((N, N), np.int32)
    for hv, center, beta, gamma in ((0, 0.0, 1.0, 1.0), (1, 1.0, 2.0**20, 2.0**-20)):
        h = np.full(N, hv, np.int32)
        betas = np.full(T, beta, np.float32)
        run = O.anneal(J, h, 0, R, betas, eps, gamma, L, seed, ikick=True)
        x = np.array([[O.gauss(seed, 0, r, 0, i) for i in range(N)] for r in range(R)], np.float64)
        for m in range(T // L):
            v = _ikick_draws(O, seed, R, N, m)
            x_end = _leapfrog_closed_form(x, v, eps, L, center)
            v_end = (_leapfrog_closed_form(x, v, eps, L + 1, center) - x_end) / eps
            x = x_end
        assert np.max(np.abs(run.x - x)) < 1e-5, hv
        assert np.max(np.abs(run.v - v_end)) < 1e-5, hv
        plain = O.anneal(J, h, 0, R, betas, eps, gamma, L, seed)
        assert np.max(np.abs(plain.x - x)) > 1e-2, hv
    with pytest.raises(ValueError):
        O.anneal(J, h, 0, 1, betas, eps, gamma, L, seed, ikick=True, mh=(1.0, 1.0))


def test_decoupled_spins_conserve_surrogate_energy(O):
    """J = 0, h != 0, constant beta: the kick is the gradient of
    U(x) = -beta sigma h tanh(gamma x) + x^2/2 (Eq. 5 with Eq. 7-8), so the
    symplectic Euler step of A7 keeps H = U + v^2/2 within O(eps)."""
    N, R = 4, 2
    f = 2
    h = np.array([4, -8, 2, 12], np.int32)          # sigma = 1/4: h = 1, -2, 0.5, 3
    J = np.zeros((N, N), np.int32)
    beta, gamma, eps = 1.5, 2.0, 0.01
    T = 3000
    betas = np.full(T, beta, np.float32)

    def Hs(x, v):
        return (-beta * (h / 4.0) * np.tanh(gamma * x) + 0.5 * x * x + 0.5 * v * v)

    run = O.Run(N, R)
    rs = np.random.default_rng(2)
    run.x[:] = rs.standard_normal((R, N)).astype(np.float32)
    run.v[:] = rs.standard_normal((R, N)).astype(np.float32)
    run.bestE[:] = np.iinfo(np.int64).max
    H0 = Hs(run.x.astype(np.float64), run.v.astype(np.float64))
    worst = 0.0
    for k in range(1, T, 100):
        O.anneal(J, h, f, R, betas, eps, gamma, 10**9, 0, k0=k, k1=min(k + 100, T), run=run)
        worst = max(worst, np.max(np.abs(Hs(run.x.astype(np.float64), run.v.astype(np.float64)) - H0)))
    assert worst < 40 * eps


def test_resume_equals_single_run(O):
    J, h = _c1()
    betas = O.beta_linear(0.1, 3.0, 500)
    full = O.anneal(J, h, 0, 6, betas, 0.2, 1.0, 50, 99)
    part = O.anneal(J, h, 0, 6, betas, 0.2, 1.0, 50, 99, k0=0, k1=173)
    O.anneal(J, h, 0, 6, betas, 0.2, 1.0, 50, 99, k0=173, k1=500, run=part)
    for a in ("x", "v", "bestE", "bestS", "bestStep"):
        assert np.array_equal(getattr(full, a), getattr(part, a)), a


def test_replica_offset_equals_rows(O):
    J, h = _c1()
    betas = O.beta_linear(0.1, 3.0, 200)
    full = O.anneal(J, h, 0, 10, betas, 0.2, 1.0, 50, 5)
    sub = O.anneal(J, h, 0, 3, betas, 0.2, 1.0, 50, 5, r0=4)
    assert np.array_equal(full.x[4:7], sub.x) and np.array_equal(full.bestE[4:7], sub.bestE)


def test_power_of_two_scaling_is_bit_exact(O):
    """(J, h) * 2^a on grid f + a is the same real instance: the trajectory is
    bit-identical and integer energies scale by 2^a (sigma enters the kick)."""
    Jf, hf = inst.sk_gauss_fixed(24, 3, frac_bits=4)
    J = np.rint(Jf * 16).astype(np.int32)
    h = np.rint(hf * 16).astype(np.int32)
    betas = O.beta_linear(0.2, 2.0, 300)
    a = O.anneal(J, h, 4, 4, betas, 0.2, 1.0, 40, 8, trace=True)
    b = O.anneal(J * 8, h * 8, 7, 4, betas, 0.2, 1.0, 40, 8, trace=True)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    assert np.array_equal(a.Etrace * 8, b.Etrace)


def test_negation_symmetry_without_field(O):
    """h = 0: starting from (-x, -v) gives exactly (-x_k, -v_k) and the same
    energies (negation is exact and fmaf is odd under round-to-nearest)."""
    J, h = _c1()
    T = 300
    betas = O.beta_linear(0.1, 3.0, T)
    rs = np.random.default_rng(4)
    runs = []
    for sgn in (1, -1):
        run = O.Run(16, 2)
        x = rs.standard_normal((2, 16)).astype(np.float32) if sgn == 1 else -runs[0][1]
        v = rs.standard_normal((2, 16)).astype(np.float32) if sgn == 1 else -runs[0][2]
        run.x[:] = x
        run.v[:] = v
        run.bestE[:] = np.iinfo(np.int64).max
        x0, v0 = run.x.copy(), run.v.copy()
        O.anneal(J, h, 0, 2, betas, 0.2, 1.0, 10**9, 0, k0=1, k1=T, run=run, trace=True)
        runs.append((run, x0, v0))
    a, b = runs[0][0], runs[1][0]
    assert np.array_equal(a.x, -b.x) and np.array_equal(a.v, -b.v)
    assert np.array_equal(a.Etrace, b.Etrace)


@pytest.mark.parametrize("dense", [False, True])
def test_planted_loops_energy_is_the_ground_state(O, dense):
    """Frustrated-loop planting: the gauge state t has the planted energy and
    exhaustive search finds nothing lower (N = 14)."""
    for seed in range(3):
        J, h, E, t = inst.planted_loops(14, seed, alpha=0.6, dense=dense)
        Ji = J.astype(np.int32)
        assert np.array_equal(J, J.T) and np.all(np.diag(J) == 0)
        assert O.energy(Ji, h.astype(np.int32), t) == E
        Eg, _ = O.bruteforce(Ji, h.astype(np.int32))
        assert Eg == E



# ------------------------------------------------------------ POLY2 ----
def test_poly2_closed_form(O):
    """POLY2 mode: d(u) = max(0, 1 - u^2 / 2.25), the truncated parabola with
    d(0) = sech^2(0) = 1 and the same integral over the line (2)."""
    us = np.concatenate([np.linspace(-2.0, 2.0, 4001), [0.0, -0.0, 1.5, -1.5, 40.0]]).astype(np.float32)
    got = np.array([O.poly2(u) for u in us], np.float64)
    ref = np.maximum(0.0, 1.0 - us.astype(np.float64) ** 2 / 2.25)
    assert np.max(np.abs(got - ref)) <= 3 * 2.0 ** -24
    assert O.poly2(0.0) == 1.0 and O.poly2(1.5) == 0.0 and O.poly2(-1.5) == 0.0 and O.poly2(2.0) == 0.0
    assert all(O.poly2(u) == O.poly2(-u) for u in us)
    du = 1e-4
    grid = np.arange(-1.6, 1.6 + du / 2, du, dtype=np.float64)
    vals = np.array([O.poly2(np.float32(u)) for u in grid], np.float64)
    integral = du * (vals.sum() - 0.5 * (vals[0] + vals[-1]))
    assert abs(integral - 2.0) < 1e-3


def test_poly2_decoupled_spins_conserve_energy(O):
    """J = 0, h != 0, constant beta, POLY2 mode: the kick is the gradient of
    U(x) = -beta sigma h Q(gamma x) + x^2/2 with Q(u) = u - u^3/6.75 on
    |u| <= 1.5 (and +-1 beyond; Q' is the quadratic), so A7 keeps
    H = U + v^2/2 within O(eps)."""
    N, R = 4, 2
    h = np.array([4, -8, 2, 12], np.int32)          # sigma = 1/4
    J = np.zeros((N, N), np.int32)
    beta, gamma, eps = 1.5, 2.0, 0.01
    T = 3000
    betas = np.full(T, beta, np.float32)

    def Q(u):
        c = np.clip(u, -1.5, 1.5)
        return c - c ** 3 / 6.75

    def Hs(x, v):
        return -beta * (h / 4.0) * Q(gamma * x) + 0.5 * x * x + 0.5 * v * v

    run = O.Run(N, R)
    rs = np.random.default_rng(2)
    run.x[:] = rs.standard_normal((R, N)).astype(np.float32)
    run.v[:] = rs.standard_normal((R, N)).astype(np.float32)
    run.bestE[:] = np.iinfo(np.int64).max
    H0 = Hs(run.x.astype(np.float64), run.v.astype(np.float64))
    worst = 0.0
    for k in range(1, T, 100):
        O.anneal(J, h, 2, R, betas, eps, gamma, 10**9, 0, k0=k, k1=min(k + 100, T), run=run, deriv="poly2")
        worst = max(worst, np.max(np.abs(Hs(run.x.astype(np.float64), run.v.astype(np.float64)) - H0)))
    assert worst < 40 * eps


def test_poly2_mode_only_changes_the_kick_factor(O):
    """With beta = 0 the derivative factor is multiplied by zero, so both
    modes run bit-identically; with beta > 0 they differ."""
    J, h = _c1()
    zero = np.zeros(300, np.float32)
    a = O.anneal(J, h, 0, 4, zero, 0.2, 1.0, 50, 7)
    b = O.anneal(J, h, 0, 4, zero, 0.2, 1.0, 50, 7, deriv="poly2")
    assert np.array_equal(a.x.view(np.uint32), b.x.view(np.uint32))
    betas = O.beta_linear(0.1, 3.0, 300)
    a = O.anneal(J, h, 0, 4, betas, 0.2, 1.0, 50, 7)
    b = O.anneal(J, h, 0, 4, betas, 0.2, 1.0, 50, 7, deriv="poly2")
    assert not np.array_equal(a.x, b.x)


def test_poly2_c1_reaches_bruteforce_ground_state(O):
    J, h = _c1()
    Eg, _ = O.bruteforce(J, h)
    betas = O.beta_linear(0.1, 3.0, 1000)
    run = O.anneal(J, h, 0, 64, betas, 0.2, 1.0, 50, 1234, deriv="poly2", threads=4)
    assert run.bestE.min() == Eg


# ------------------------------------------------ accept/reject (state 4) -----
def _mh_rate_closed_form(eps, L, N, n=400000, seed=11):
    """Acceptance probability of the first decided trajectory for J = h = 0,
    by FP64 Monte Carlo over the closed-form map [[1, eps], [-eps, 1 - eps^2]]^L:
    the first trajectory carries (x0, v0) to its end, the second starts there with
    a fresh v1, and H = (x.x + v.v) / 2 (no coupling term)."""
    rs = np.random.default_rng(seed)
    M = np.linalg.matrix_power(np.array([[1.0, eps], [-eps, 1.0 - eps * eps]]), L)
    x0, v0, v1 = (rs.standard_normal((n, N)) for _ in range(3))
    xs = M[0, 0] * x0 + M[0, 1] * v0
    xe = M[0, 0] * xs + M[0, 1] * v1
    ve = M[1, 0] * xs + M[1, 1] * v1
    dH = 0.5 * ((xe * xe + ve * ve).sum(1) - (xs * xs + v1 * v1).sum(1))
    return float(np.minimum(1.0, np.exp(-dH)).mean())


@pytest.mark.parametrize("eps,L,N", [(1.2, 2, 1), (1.2, 3, 2)])
def test_mh_acceptance_rate_harmonic(O, eps, L, N):
    """With no couplings H is the kinetic-plus-quadratic term alone; the
    fraction of replicas that accept their first decided trajectory matches the
    closed-form expectation (a sign error gives ~0.93, a dropped 1/2 ~0.84 or
    ~0.50, a doubled one ~0.64 or ~0.29)."""
    R = 20000
    J = np.zeros((N, N), np.int32)
    betas = np.full(2 * L + 1, 1.0, np.float32)
    run = O.anneal(J, None, 0, R, betas, eps, 1.0, L, 31, mh=(1.0, 1.0), trace=True, threads=4)
    assert run.mhtrace.shape == (R, 2)
    assert np.all(run.mhtrace[:, 0] == -1)
    rate = float(np.mean(run.mhtrace[:, 1] == 1))
    p = _mh_rate_closed_form(eps, L, N)
    sd = math.sqrt(p * (1 - p) / R)
    assert abs(rate - p) < 5 * sd + 0.003, (rate, p)
    assert np.array_equal(run.acc, (run.mhtrace[:, 1] == 1).astype(np.int32))
    assert np.all(run.dec == 1)


def test_mh_large_beta_accepts_exactly_the_energy_drops(O):
    """beta large in H while gamma is tiny (the kick scales with beta gamma):
    beta sigma dE dominates dH, so a trajectory whose end energy differs from
    its start is accepted iff the energy fell; rejected ends restore the start."""
    J, h = inst.sk_pm1(12, 3)
    J, h = J.astype(np.int32), h.astype(np.int32)
    L = 5
    betas = np.full(600, 1e4, np.float32)
    run = O.anneal(J, h, 0, 16, betas, 0.2, 1e-6, L, 3, mh=(1.0, 1.0), trace=True)
    E, tr = run.Etrace, run.mhtrace
    checked = rejected = 0
    for r in range(16):
        Es = None
        for m in range(tr.shape[1]):
            Ee = E[r, (m + 1) * L - 1]
            if tr[r, m] == -1:
                assert m == 0
                Es = Ee
                continue
            if Ee != Es:
                assert (tr[r, m] == 1) == (Ee < Es)
                checked += 1
            rejected += tr[r, m] == 0
            if tr[r, m] == 1:
                Es = Ee
    assert checked > 1000 and rejected > 1000


def test_mh_reject_restores_the_trajectory_start(O):
    J, h = _c1()
    L = 6
    betas = O.beta_linear(2.0, 3.0, 2 * L + 1)
    run = O.anneal(J, h, 0, 32, betas, 0.4, 1.0, L, 17, k1=L, mh=(1.0, 1.0))
    xA, EA = run.x.copy(), run.Elast.copy()
    O.anneal(J, h, 0, 32, betas, 0.4, 1.0, L, 17, k0=L, k1=2 * L, run=run, mh=(1.0, 1.0))
    xB, EB = run.x.copy(), run.Elast.copy()
    assert np.array_equal(run.x0, xA)   # snapshot at the start of trajectory 1
    O.anneal(J, h, 0, 32, betas, 0.4, 1.0, L, 17, k0=2 * L, k1=2 * L + 1, run=run,
             mh=(1.0, 1.0), trace=True)
    acc = run.mhtrace[:, 0] == 1
    assert 0 < acc.sum() < 32
    for r in range(32):
        assert np.array_equal(run.x0[r], xB[r] if acc[r] else xA[r])
        assert run.Estart[r] == (EB[r] if acc[r] else EA[r])


def test_mh_all_accepted_equals_plain_sweep(O):
    """Small steps and short trajectories: every trajectory is accepted, and the
    run is bit-identical to the sweep without the accept/reject step."""
    J, h = inst.sk_pm1(8, 3)
    J, h = J.astype(np.int32), h.astype(np.int32)
    betas = np.full(400, 0.001, np.float32)
    a = O.anneal(J, h, 0, 8, betas, 0.01, 1.0, 4, 3, mh=(1.0, 1.0), trace=True)
    b = O.anneal(J, h, 0, 8, betas, 0.01, 1.0, 4, 3, trace=True)
    assert np.all(a.acc == a.dec) and a.dec.sum() == 8 * 98
    for f in ("x", "v", "bestE", "bestS", "Etrace"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert np.count_nonzero(np.diff(b.Etrace, axis=1)) > 50


def test_mh_lambda_multiplies_beta(O):
    """up = down = 2 doubles lam after every decision, which must equal a run
    with lam fixed and beta doubled per trajectory (powers of two are exact):
    lam enters the kick and H exactly as a factor of beta."""
    J, h = inst.sk_pm1(12, 4)
    J, h = J.astype(np.int32), h.astype(np.int32)
    L, T = 25, 275
    betas = O.beta_linear(0.1, 1.0, T)
    a = O.anneal(J, h, 0, 8, betas, 0.2, 1.0, L, 9, mh=(2.0, 2.0), trace=True)
    scale = np.array([2.0 ** max(0, k // L - 1) for k in range(T)], np.float32)
    b = O.anneal(J, h, 0, 8, betas * scale, 0.2, 1.0, L, 9, mh=(1.0, 1.0), trace=True)
    assert np.all(a.lam == 2.0 ** 9) and np.all(b.lam == 1.0)
    for f in ("x", "v", "bestE", "Etrace", "mhtrace", "acc"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert 0 < a.acc.sum() < a.dec.sum()


def test_mh_lambda_follows_outcomes(O):
    J, h = _c1()
    betas = O.beta_linear(0.5, 3.0, 400)
    run = O.anneal(J, h, 0, 8, betas, 0.3, 1.0, 40, 5, mh=(2.0, 0.5))
    expo = 2 * run.acc.astype(np.int64) - run.dec
    assert np.all(np.abs(expo) <= 10)
    assert np.array_equal(run.lam, (2.0 ** expo).astype(np.float32))
    assert np.all(run.dec == 8)  # decisions at k = 80, ..., 360 (k = 40 takes the first)


def test_mh_power_of_two_scaling_and_resume(O):
    Jf, hf = inst.sk_gauss_fixed(24, 3, frac_bits=4)
    J = np.rint(Jf * 16).astype(np.int32)
    h = np.rint(hf * 16).astype(np.int32)
    betas = O.beta_linear(0.5, 3.0, 300)
    a = O.anneal(J, h, 4, 4, betas, 0.3, 1.0, 20, 8, mh=(1.25, 0.8), trace=True)
    b = O.anneal(J * 8, h * 8, 7, 4, betas, 0.3, 1.0, 20, 8, mh=(1.25, 0.8), trace=True)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.mhtrace, b.mhtrace)
    assert np.array_equal(a.lam, b.lam) and 0 < a.acc.sum() < a.dec.sum()
    c = O.anneal(J, h, 4, 4, betas, 0.3, 1.0, 20, 8, k1=40, mh=(1.25, 0.8))
    for k0, k1 in ((40, 137), (137, 300)):
        O.anneal(J, h, 4, 4, betas, 0.3, 1.0, 20, 8, k0=k0, k1=k1, run=c, mh=(1.25, 0.8))
    for f in ("x", "v", "bestE", "bestS", "lam", "acc", "dec"):
        assert np.array_equal(getattr(a, f), getattr(c, f)), f
