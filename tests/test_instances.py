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
    if name != "spin_model":
        assert np.all(h == 0)


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
