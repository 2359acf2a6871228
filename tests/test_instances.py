"""Host-side checks of the seeded instance generators (no oracle, no GPU)."""
import numpy as np
import pytest

from paper_2407_10205_amd import instances as inst


@pytest.mark.parametrize("name", inst.TABLE2_FAMILIES)
def test_table2_families(name):
    """Generators of the Table 2 families: symmetric, zero diagonal, values
    on the stated sets and grid; cubic graphs have degree 3."""
    N = 24
    J, h = inst.table2_family(name, N, 5)
    assert J.shape == (N, N) and h.shape == (N,)
    assert np.array_equal(J, J.T) and np.all(np.diag(J) == 0)
    off = J[np.triu_indices(N, 1)]
    if name in ("maxcut_dense", "maxcut_d3", "sk_bool"):
        assert set(np.unique(off)) <= {0.0, -1.0}
    if name == "maxcut_d3":
        assert np.all((J != 0).sum(axis=1) == 3)
    if name == "sk_ising":
        assert set(np.unique(off)) == {-1.0, 1.0}
    if name == "sk_uniform":
        assert np.all(off <= 0) and np.all(off >= -1) and np.all(off * 64 == np.rint(off * 64))
        assert 0.3 < np.mean(off == 0) < 0.7
    if name == "spin_model":
        assert np.all(np.abs(off) <= 1) and np.all(np.abs(h) <= 1)
        assert np.all(off * 64 == np.rint(off * 64)) and np.all(h * 64 == np.rint(h * 64))
    if name == "nae_3_sat":
        assert np.all(off == np.rint(off)) and np.any(off != 0)
    if name != "spin_model":
        assert np.all(h == 0)


def _clause_energy(C, s):
    """Sum over clauses of 3 (literals all equal) or -1 (not all equal),
    counted clause by clause from the literal values."""
    E = 0
    for cl in C:
        lit = cl[:, 1] * s[cl[:, 0]]
        E += 3 if lit[0] == lit[1] == lit[2] else -1
    return E


def test_nae_3_sat_reduction_pins(O):
    """NAE-3-SAT through the clause-to-triangle reduction: Eq. 2 of the
    instance equals the clause count formula (3 per all-equal clause, -1
    per NAE-satisfied one) on random states; planted instances (N <= 16,
    2 N clauses) have exhaustive ground energy -M, reached by the hidden
    assignment; the four sign patterns of one variable triple that together
    exclude all eight assignments leave one clause violated (ground 0)."""
    rs = np.random.default_rng(0)
    for N, seed in ((6, 1), (9, 2), (12, 3), (16, 4)):
        J, h, M, z, C = inst.nae_3_sat(N, seed)
        Ji, hi = J.astype(np.int32), h.astype(np.int32)
        for _ in range(20):
            s = rs.choice([-1, 1], size=N).astype(np.int8)
            assert O.energy(Ji, hi, s) == _clause_energy(C, s)
        Eg, sg = O.bruteforce(Ji, hi)
        assert Eg == -M
        assert O.energy(Ji, hi, z.astype(np.int8)) == -M
        assert _clause_energy(C, sg) == -M
    C = np.array([[[0, 1], [1, 1], [2, 1]], [[0, 1], [1, 1], [2, -1]],
                  [[0, 1], [1, -1], [2, 1]], [[0, -1], [1, 1], [2, 1]]])
    J = np.zeros((3, 3), np.int32)
    for cl in C:
        for a in range(3):
            for b in range(a + 1, 3):
                J[cl[a, 0], cl[b, 0]] -= cl[a, 1] * cl[b, 1]
                J[cl[b, 0], cl[a, 0]] -= cl[a, 1] * cl[b, 1]
    assert O.bruteforce(J, np.zeros(3, np.int32))[0] == 0


def test_bench_exhaustive_ground_energy_matches_oracle(O):
    """The time-to-target sweep's exhaustive targets (numpy enumeration in
    bench.py) equal the oracle's brute force on every Table 2 family."""
    import bench
    for name in inst.TABLE2_FAMILIES:
        J, h = inst.table2_family(name, 12, 3)
        Ji = np.rint(J * 64).astype(np.int32)
        hi = np.rint(h * 64).astype(np.int32)
        assert bench.ground_energy_exhaustive(Ji, hi) == O.bruteforce(Ji, hi)[0]


def test_tts99_definition():
    """Eq. 9 with the success probability of a launch of R replicas."""
    import math
    import bench
    assert bench.tts99(2.0, 0.0, 100) == float("inf")
    assert bench.tts99(2.0, 0.5, 100) == 2.0
    p = 1 - (1 - 0.001) ** 64
    assert abs(bench.tts99(1.0, 0.001, 64) - math.log(0.01) / math.log(1 - p)) < 1e-12


def test_cpu_baseline_fields():
    """The benchmark's CPU leg (the oracle timed on the host) reports the
    fields its result line carries: a positive rate, the thread count it
    used, kind "oracle", the sample it timed, the single-thread rate and the
    host CPU; the sample grows its replica count (up to the workload's) when
    the whole schedule fits the budget."""
    import bench
    sched = dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=25)
    insts = [inst.sk_pm1(24, 1), inst.regular3_pm1(30, 2)]
    r = bench.cpu_baseline_instances(insts, 64, 40, sched, 0.5, "two instances")
    cores = bench.host_cpu()["threads"]
    assert r["kind"] == "oracle" and r["unit"] == "spin-updates/s" and r["cores"] == cores
    assert r["value"] > 0 and r["single_thread"]["value"] > 0
    assert "steps 0..39" in r["sample"] and "two instances" in r["sample"]
    reps = int(r["sample"].split("replicas 0..")[1].split(",")[0]) + 1
    assert reps >= cores and reps % cores == 0 and reps <= max(64, cores)
    for key in ("cpu_model", "nproc", "cpus_allowed"):
        assert key in r
    J, h = inst.sk_pm1(20, 3)
    w = dict(R=8, T=30, sched=dict(sched))
    r = bench.cpu_baseline(J, h, w, 0.3)
    assert r["kind"] == "oracle" and r["value"] > 0 and r["single_thread"]["value"] > 0
    assert "steps 0..29" in r["sample"] and r["cores"] == cores
