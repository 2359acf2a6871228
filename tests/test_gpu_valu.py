"""GPU parity of the VALU sweeps (k_sweep_valu) against the CPU oracle.

Two forms besides the FP32 plain sweep: the ELL path (sparse rows, spin
gathers) and the int8 dot-product sweep that the I8 path takes with few
replicas, where J.s is a matrix-vector product per replica.  Both compute the
same exact integer field as every other path, so x, v, records, record steps
and energy traces must be bit-identical to the oracle's.
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


class Forced:
    """PHIA_GEOMETRY for the anneals started inside the block."""

    def __init__(self, spec):
        self.spec = spec

    def __enter__(self):
        if self.spec:
            os.environ["PHIA_GEOMETRY"] = self.spec

    def __exit__(self, *exc):
        os.environ.pop("PHIA_GEOMETRY", None)


def int_units(J, h, f):
    return (np.rint(J * 2**f).astype(np.int32), np.rint(h * 2**f).astype(np.int32))


def run_both(P, O, J, h, f, path, R, T, seed, rows=None, geometry=None, eps=0.2, gamma=1.0, b0=0.1, b1=3.0, L=37,
             deriv="tanh", trace=True):
    say(f"case N={J.shape[0]} R={R} T={T} path={path} geometry={geometry} seed={seed} deriv={deriv}")
    prob = P.Problem(J, h, frac_bits=f, path=path)
    if trace:
        prob.set_trace(True)
    with Forced(geometry):
        prob.anneal(R, T, eps, gamma, beta0=b0, beta1=b1, refresh_L=L, seed=seed, deriv=deriv)
    E, S, K = prob.replica_best()
    x, v, k = prob.get_state()
    dev = dict(E=E, S=S, K=K, x=x, v=v, info=prob.info(), trace=prob.trace(T) if trace else None,
               best_exact=prob.best_exact(), best=prob.best())
    prob.close()
    Ji, hi = int_units(J, h, f)
    betas = O.beta_linear(b0, b1, T)
    runs = {r: O.anneal(Ji, hi, f, 1, betas, eps, gamma, L, seed, r0=r, trace=trace, deriv=deriv)
            for r in (range(R) if rows is None else rows)}
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


# ------------------------------------------------------------------ ELL ----
@pytest.mark.parametrize("geometry", [None, "valu,1", "valu,4"])
def test_ell_regular3_parity(P, O, geometry):
    """Sparse random 3-regular +-1 graph with h in {-1, 0, 1} (the sparse half
    of the uneven-N batch), ragged N = 202 (Np = 256), R = 9 (a ragged block
    of 4), both rows-per-workgroup variants."""
    J, h = inst.regular3_pm1(202, 5)
    dev, runs = run_both(P, O, J, h, 0, "ell", 9, 257, 31, geometry=geometry)
    assert dev["info"]["path_name"] == "ell" and dev["info"]["sweep_kernel"] == 4
    if geometry:
        assert dev["info"]["rows_per_block"] == int(geometry.split(",")[1])
    assert_parity(dev, runs)


def test_ell_uneven_degree_16bit_parity(P, O):
    """Erdos-Renyi rows of uneven degree (D = the largest), couplings up to
    2^14 units on a 2^-9 grid and nonzero fields, POLY2 kick: slots past a
    row's last nonzero hold zero and change nothing."""
    rs = np.random.default_rng(8)
    N = 150
    A = np.triu((rs.random((N, N)) < 0.05) * rs.integers(-2**14, 2**14, (N, N)), 1)
    J = (A + A.T).astype(np.float64) / 2**9
    h = rs.integers(-300, 300, N).astype(np.float64) / 2**9
    dev, runs = run_both(P, O, J, h, 9, "ell", 5, 203, 7, deriv="poly2", eps=0.05, b0=0.01, b1=0.3)
    assert_parity(dev, runs)


def test_ell_largest_n_sampled(P, O):
    """N = 4096 (16 columns per thread), 3-regular: sampled replicas."""
    J, h = inst.regular3_pm1(4096, 2)
    dev, runs = run_both(P, O, J, h, 0, "ell", 6, 41, 3, rows=[0, 5], trace=False)
    assert dev["info"]["Np"] == 4096
    assert_parity(dev, runs)


@pytest.mark.parametrize("path,kind,N,R,geometry", [
    ("fp32", "fixed", 700, 7, None), ("fp32", "fixed", 1500, 5, None), ("ell", "reg3", 700, 5, "valu,1"),
    ("ell", "reg3", 1500, 6, "valu,4"), ("ell", "er16", 1100, 3, None)])
def test_wide_workgroup_forms_parity(P, O, path, kind, N, R, geometry):
    """The FP32 and ELL forms in 1024-thread workgroups (Np > 256): one and
    two columns per thread, ragged replica blocks of four, and uneven 16-bit
    ELL rows with the POLY2 factor; every replica bit-identical to the
    oracle."""
    deriv, f = "tanh", 0
    if kind == "fixed":
        J, h = inst.sk_gauss_fixed(N, 11, frac_bits=5, bits=8)
        f = 5
    elif kind == "reg3":
        J, h = inst.regular3_pm1(N, 12)
    else:
        rs = np.random.default_rng(13)
        A = np.triu((rs.random((N, N)) < 0.01) * rs.integers(-2**14, 2**14, (N, N)), 1)
        J = (A + A.T).astype(np.float64) / 2**9
        h = rs.integers(-300, 300, N).astype(np.float64) / 2**9
        f, deriv = 9, "poly2"
    dev, runs = run_both(P, O, J, h, f, path, R, 61, 21, geometry=geometry, deriv=deriv,
                         b0=0.01 if f == 9 else 0.1, b1=0.3 if f == 9 else 3.0)
    assert dev["info"]["path_name"] == path and dev["info"]["sweep_kernel"] == 4
    if geometry:
        assert dev["info"]["rows_per_block"] == int(geometry.split(",")[1])
    assert_parity(dev, runs)


def test_ell_matches_other_paths(P):
    """Same instance, same seed: ELL, int8 and FP32 give identical results."""
    J, h = inst.er_maxcut(300, 0.06, 4, signed=True)
    out = {}
    for path in ("ell", "i8", "fp32"):
        say(f"cross-path {path}")
        p = P.Problem(J, h, path=path)
        p.anneal(40, 300, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=50, seed=77)
        E, S, K = p.replica_best()
        x, v, _ = p.get_state()
        out[path] = (E, S, K, x.view(np.uint32), v.view(np.uint32))
        p.close()
    for path in ("i8", "fp32"):
        for a, b in zip(out["ell"], out[path]):
            assert np.array_equal(a, b), path


# ----------------------------------------------- int8, few replicas ----
@pytest.mark.parametrize("R", [1, 4, 16])
@pytest.mark.parametrize("geometry", ["valu,1", "valu,2"])
def test_i8_valu_few_replicas_parity(P, O, R, geometry):
    """Max-cut G(300, 0.06) with +-1 weights, ragged N (Np = 320, two column
    passes for the first 64 threads): R = 1, 4, 16 on the int8 dot-product
    sweep, both rows-per-workgroup variants."""
    J, h = inst.er_maxcut(300, 0.06, 1, signed=True)
    dev, runs = run_both(P, O, J, h, 0, "i8", R, 230, 5 + R, geometry=geometry)
    assert dev["info"]["sweep_kernel"] == 4
    assert_parity(dev, runs)


def test_i8_valu_c1_and_argmin(P, O):
    """SK N = 16 (Np = 64, most threads own no column), 3 replicas: parity,
    and the final argmin over the replicas equals the oracle's."""
    J, h = inst.sk_pm1(16, 0)
    dev, runs = run_both(P, O, J, h, 0, "i8", 3, 1000, 1234, geometry="valu,2", L=50)
    assert_parity(dev, runs)
    Es = np.array([runs[r].bestE[0] for r in range(3)])
    r_star = int(np.argmin(Es))
    E_units, _, r_dev = dev["best_exact"]
    assert E_units == Es[r_star] and r_dev == r_star
    assert np.array_equal(dev["best"][1], runs[r_star].bestS[0][:16])


def test_i8_valu_n2000_sampled(P, O):
    """Dense fixed-point SK N = 2000 with 8-bit couplings, R = 2, sampled: 8
    column passes per thread."""
    J, h = inst.sk_gauss_fixed(2000, 11, frac_bits=5, bits=8)
    dev, runs = run_both(P, O, J, h, 5, "i8", 2, 31, 9, rows=[1], geometry="valu,2", trace=False)
    assert_parity(dev, runs)


def test_i8_auto_takes_valu_below_crossover(P):
    """Default geometry: the VALU sweep at R <= phia_valu_crossover(Np), a
    matrix-core sweep above it."""
    J, h = inst.er_maxcut(200, 0.06, 2)
    p = P.Problem(J, h, path="i8")
    Np = p.info()["Np"]
    rx = P.valu_crossover(Np)
    say(f"crossover Np={Np}: {rx}")
    for R in sorted({1, max(rx, 1), rx + 1, 64}):
        p.start(R, 20, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=10, seed=1)
        p.run(20)
        p.sync()
        k = p.info()["sweep_kernel"]
        assert (k == 4) == (R <= rx), (R, rx, k)
    p.close()


def test_i8_valu_chunked_and_noalloc(P):
    """The VALU sweep run in chunks, and phia_anneal_noalloc with the same
    geometry, equal one whole anneal."""
    import torch
    J, h = inst.er_maxcut(180, 0.08, 3, signed=True)
    R, T = 3, 150
    with Forced("valu,2"):
        a = P.Problem(J, h, path="i8")
        a.anneal(R, T, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=20, seed=4)
        E0, S0, K0 = a.replica_best()
        x0, v0, _ = a.get_state()
        b = P.Problem(J, h, path="i8")
        b.start(R, T, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=20, seed=4)
        for k in (7, 64, 65, T):
            b.run(k)
        b.sync()
        assert b.info()["sweep_kernel"] == 4
        E1, S1, K1 = b.replica_best()
        x1, v1, _ = b.get_state()
        Np = a.info()["Np"]
        dev = torch.device("cuda:0")
        bufs = dict(x=torch.empty(R, Np, dtype=torch.float32, device=dev),
                    v=torch.empty(R, Np, dtype=torch.float32, device=dev),
                    bestE=torch.empty(R, dtype=torch.int64, device=dev),
                    bestS=torch.empty(R, Np, dtype=torch.int8, device=dev),
                    bestStep=torch.empty(R, dtype=torch.int64, device=dev))
        a.anneal_noalloc(R, T, 0.2, 1.0, *(bufs[k].data_ptr() for k in ("x", "v", "bestE", "bestS", "bestStep")),
                         beta0=0.1, beta1=3.0, refresh_L=20, seed=4)
        torch.cuda.synchronize()
    assert np.array_equal(E0, E1) and np.array_equal(K0, K1) and np.array_equal(S0, S1)
    assert np.array_equal(x0.view(np.uint32), x1.view(np.uint32))
    assert np.array_equal(v0.view(np.uint32), v1.view(np.uint32))
    N = x0.shape[1]
    same_E = np.array_equal(bufs["bestE"].cpu().numpy(), E0)
    same_x = np.array_equal(bufs["x"].cpu().numpy()[:, :N].view(np.uint32), x0.view(np.uint32))
    assert same_E and same_x
    a.close()
    b.close()


# ------------------------------------------------- initial kick ----
def run_ikick(P, O, J, h, f, path, R, T, seed, L, geometry=None, chunks=(), deriv="tanh", rows=None):
    say(f"ikick N={J.shape[0]} R={R} T={T} L={L} path={path} geometry={geometry} chunks={chunks}")
    prob = P.Problem(J, h, frac_bits=f, path=path)
    prob.set_trace(True)
    with Forced(geometry):
        prob.start(R, T, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=L, seed=seed, deriv=deriv, ikick=True)
    for k in tuple(chunks) + (T,):
        prob.run(k)
    prob.sync()
    E, S, K = prob.replica_best()
    x, v, _ = prob.get_state()
    dev = dict(E=E, S=S, K=K, x=x, v=v, info=prob.info(), trace=prob.trace(T))
    prob.close()
    Ji, hi = int_units(J, h, f)
    betas = O.beta_linear(0.1, 3.0, T)
    runs = {r: O.anneal(Ji, hi, f, 1, betas, 0.2, 1.0, L, seed, r0=r, trace=True, deriv=deriv, ikick=True)
            for r in (range(R) if rows is None else rows)}
    return dev, runs


@pytest.mark.parametrize("path,geometry", [("fp32", None), ("i8", "valu,1"), ("i8", "valu,2"), ("ell", None)])
def test_initial_kick_parity(P, O, path, geometry):
    """Initial-kick variant (Table 3, state 2) on every VALU form: ragged
    N = 150 fixed-point couplings for FP32 and int8, a 3-regular graph for
    ELL; refresh period 23 that does not divide T = 201."""
    if path == "ell":
        J, h = inst.regular3_pm1(150, 9)
        f = 0
    else:
        J, h = inst.sk_gauss_fixed(150, 4, frac_bits=5, bits=8)
        f = 5
    dev, runs = run_ikick(P, O, J, h, f, path, 7, 201, 21, 23, geometry=geometry)
    assert dev["info"]["sweep_kernel"] == 4
    assert_parity(dev, runs)
    # the variant changes the trajectories
    o0 = O.anneal(*int_units(J, h, f), f, 1, O.beta_linear(0.1, 3.0, 201), 0.2, 1.0, 23, 21, r0=0)
    assert not np.array_equal(o0.x[0], runs[0].x[0])


def test_initial_kick_chunked_poly2_and_large_n(P, O):
    """Launch boundaries inside and at trajectory starts leave the results
    unchanged (the half kick recomputes its field); POLY2 factor; the int8
    form with J streamed (N = 600, no LDS copy) sampled."""
    J, h = inst.er_maxcut(200, 0.05, 6, signed=True)
    dev, runs = run_ikick(P, O, J, h, 0, "i8", 5, 120, 3, 20, chunks=(20, 33, 40, 100), deriv="poly2")
    assert_parity(dev, runs)
    J, h = inst.er_maxcut(600, 0.05, 7, signed=True)
    dev, runs = run_ikick(P, O, J, h, 0, "i8", 3, 60, 4, 25, rows=[2])
    assert dev["info"]["j_in_lds"] == 0
    assert_parity(dev, runs)


def test_initial_kick_noalloc_and_refusals(P):
    """phia_anneal_noalloc with the initial kick equals phia_anneal; BF16
    hi/lo (no VALU form) refuses it with PHIA_ERANGE, metropolis with
    PHIA_EINVAL, and batch plans refuse it."""
    import torch
    J, h = inst.er_maxcut(130, 0.1, 8, signed=True)
    R, T = 4, 90
    a = P.Problem(J, h, path="i8")
    a.anneal(R, T, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=30, seed=2, ikick=True)
    E0, S0, K0 = a.replica_best()
    x0, _, _ = a.get_state()
    Np = a.info()["Np"]
    d = torch.device("cuda:0")
    bufs = [torch.empty(R, Np, dtype=torch.float32, device=d), torch.empty(R, Np, dtype=torch.float32, device=d),
            torch.empty(R, dtype=torch.int64, device=d), torch.empty(R, Np, dtype=torch.int8, device=d),
            torch.empty(R, dtype=torch.int64, device=d)]
    a.anneal_noalloc(R, T, 0.2, 1.0, *(b.data_ptr() for b in bufs), beta0=0.1, beta1=3.0, refresh_L=30, seed=2,
                     ikick=True)
    torch.cuda.synchronize()
    same = (np.array_equal(bufs[2].cpu().numpy(), E0) and
            np.array_equal(bufs[0].cpu().numpy()[:, :x0.shape[1]].view(np.uint32), x0.view(np.uint32)))
    assert same
    with pytest.raises(P.PhiaError) as e:
        a.start(R, T, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=30, seed=2, ikick=True, mh=(1.0, 1.0))
    assert e.value.code == -1
    a.close()
    b = P.Problem(J * 300 / 128, h, path="bf16hilo", frac_bits=7, quantize=True)
    with pytest.raises(P.PhiaError) as e:
        b.start(R, T, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=30, seed=2, ikick=True)
    assert e.value.code == -4
    b.close()
    c = P.Problem(J, h, path="i8")
    c.start(R, T, 0.2, 1.0, beta0=0.1, beta1=3.0, refresh_L=30, seed=2)
    c.sync()
    with pytest.raises(P.PhiaError) as e:
        P.Batch([c], [R], [T], [dict(eps=0.2, gamma=1.0, beta0=0.1, beta1=3.0, refresh_L=30, ikick=True)])
    assert e.value.code == -1
    c.close()
