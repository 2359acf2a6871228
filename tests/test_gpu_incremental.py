"""GPU parity of the flip-incremental field update against the full product
and the CPU oracle, through the C ABI.

Between consecutive steps only the spins whose sign changed alter the field
I = J s + h of Eq. 6, so I(k) = I(k-1) + J (s(k) - s(k-1)).  The sweep keeps
J s in int32 registers and adds the product over the 16-spin column blocks
that changed, or recomputes it in full when too many did.  Both are exact
integer arithmetic, so every output must be bit-identical with the setting
on and off, and to the oracle (which recomputes J s every step).
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


def run(P, J, h, f, geometry, inc, R, T, b0, b1, L, seed, trace=False, chunk=None, path="i8", mh=None):
    say(f"case N={J.shape[0]} path={path} geometry={geometry} inc={inc} R={R} T={T} chunk={chunk} trace={trace} "
        f"mh={mh}")
    os.environ["PHIA_GEOMETRY"] = geometry
    try:
        p = P.Problem(J, h, frac_bits=f, path=path)
        p.set_incremental(inc)
        if trace:
            p.set_trace(True)
        if chunk is None:
            p.anneal(R, T, 0.2, 1.0, beta0=b0, beta1=b1, refresh_L=L, seed=seed, mh=mh)
        else:
            p.start(R, T, 0.2, 1.0, beta0=b0, beta1=b1, refresh_L=L, seed=seed, mh=mh)
            for k in range(chunk, T + chunk, chunk):
                p.run(min(k, T))
            p.sync()
    finally:
        del os.environ["PHIA_GEOMETRY"]
    E, S, K = p.replica_best()
    x, v, _ = p.get_state()
    out = dict(E=E, S=S, K=K, x=x, v=v, info=p.info(), stats=p.incremental_stats(),
               trace=p.trace(T) if trace else None, mhc=p.replica_mh() if mh is not None else None)
    p.close()
    say("  info", out["info"]["group"], out["info"]["incremental"], "stats", out["stats"])
    return out


def same(a, b):
    if a["mhc"] is not None:
        for u, w in zip(a["mhc"], b["mhc"]):
            assert np.array_equal(u, w), "accept/reject counts"
    for key in ("E", "S", "K", "x", "v", "trace"):
        if a[key] is None:
            continue
        u, w = a[key], b[key]
        if u.dtype.kind == "f":
            u, w = u.view(np.uint32), w.view(np.uint32)
        assert np.array_equal(u, w), key


def oracle_check(O, dev, J, h, f, T, b0, b1, L, seed, rows, trace=False, mh=None):
    Ji, hi = int_units(J, h, f)
    betas = O.beta_linear(b0, b1, T)
    for r in rows:
        o = O.anneal(Ji, hi, f, 1, betas, 0.2, 1.0, L, seed, r0=r, trace=trace, mh=mh)
        if mh is not None:
            assert (dev["mhc"][0][r], dev["mhc"][1][r]) == (o.acc[0], o.dec[0]), f"accept/reject replica {r}"
        assert np.array_equal(dev["x"][r].view(np.uint32), o.x[0].view(np.uint32)), f"x replica {r}"
        assert np.array_equal(dev["v"][r].view(np.uint32), o.v[0].view(np.uint32)), f"v replica {r}"
        assert dev["E"][r] == o.bestE[0] and dev["K"][r] == o.bestStep[0], f"record replica {r}"
        assert np.array_equal(dev["S"][r], o.bestS[0]), f"bestS replica {r}"
        if trace:
            assert np.array_equal(dev["trace"][r], o.Etrace[0]), f"trace replica {r}"


PATHS = {"i8": (5, 8), "bf16hilo": (12, 16)}  # path: (frac_bits, coupling bits) of the SK instances


@pytest.mark.parametrize("path", sorted(PATHS))
@pytest.mark.parametrize("geometry", ["1,8,0,1", "1,8,0,2", "1,4,0,2", "1,2,0,2,0"])
def test_incremental_equals_full_and_oracle(P, O, geometry, path):
    """Ragged N (20 column blocks over the group), ragged R (last block 8 of
    16 rows), energy traces on; a schedule that ends cold, so that early steps
    take the full product and late ones the incremental one.  BF16 hi/lo with
    16-bit couplings, both planes non-zero."""
    f, bits = PATHS[path]
    J, h = inst.sk_gauss_fixed(300, 21, frac_bits=f, bits=bits)
    R, T, b0, b1, L, seed = 40, 400, 0.05 * 2.0 ** (f - 5), 3.0 * 2.0 ** (f - 5), 25, 17
    on = run(P, J, h, f, geometry, True, R, T, b0, b1, L, seed, trace=True, path=path)
    off = run(P, J, h, f, geometry, False, R, T, b0, b1, L, seed, trace=True, path=path)
    assert on["info"]["path_name"] == path
    assert on["info"]["incremental"] == 1 and off["info"]["incremental"] == 0
    n_inc, n_full, n_kb = on["stats"]
    blocks = (R + 15) // 16
    assert n_inc + n_full == blocks * T
    assert n_inc > 0 and n_full >= blocks, "both products must run"
    assert n_kb < n_inc * (320 // 64), "incremental steps use fewer k blocks than the full product"
    assert off["stats"] == (0, 0, 0)
    same(on, off)
    oracle_check(O, on, J, h, f, T, b0, b1, L, seed, rows=(0, 17, 39), trace=True)


def test_incremental_chunked_launches(P, O):
    """Launch boundaries (every launch starts with the full product) do not
    change anything."""
    J, h = inst.sk_gauss_fixed(500, 3, frac_bits=4, bits=8)
    R, T, b0, b1, L, seed = 64, 300, 0.05, 2.5, 20, 5
    one = run(P, J, h, 4, "1,8,0,2", True, R, T, b0, b1, L, seed)
    chunked = run(P, J, h, 4, "1,8,0,2", True, R, T, b0, b1, L, seed, chunk=37)
    off = run(P, J, h, 4, "1,8,0,2", False, R, T, b0, b1, L, seed, chunk=37)
    same(one, chunked)
    same(one, off)
    n_inc, n_full, _ = chunked["stats"]
    launches = -(-T // 37)
    assert n_full >= launches * (R // 16) and n_inc > 0
    oracle_check(O, one, J, h, 4, T, b0, b1, L, seed, rows=(0, 63))


@pytest.mark.parametrize("path", sorted(PATHS))
def test_incremental_sk2000_shape(P, O, path):
    """The SK N = 2000 shape (32 k blocks of 64) with the group of its
    workloads (8 members, member m of every group on XCD m), 8- and 16-bit
    couplings, sampled against the oracle."""
    f, bits = PATHS[path]
    J, h = inst.sk_gauss_fixed(2000, 0, frac_bits=f, bits=bits)
    R, T, b0, b1, L, seed = 32, 600, 0.02 * 2.0 ** (f - 5), 3.0 * 2.0 ** (f - 5), 25, 11
    on = run(P, J, h, f, "1,8,0,2,0", True, R, T, b0, b1, L, seed, path=path)
    off = run(P, J, h, f, "1,8,0,2,0", False, R, T, b0, b1, L, seed, path=path)
    same(on, off)
    n_inc, n_full, n_kb = on["stats"]
    assert on["info"]["incremental"] == 1 and n_inc > 0 and n_kb < n_inc * 32
    oracle_check(O, on, J, h, f, T, b0, b1, L, seed, rows=(0, 31))


@pytest.mark.parametrize("path,N_max,N_off", [("i8", 4864, 4928), ("bf16hilo", 2496, None)])
def test_incremental_size_limit(P, O, path, N_max, N_off):
    """The largest instance whose LDS holds the incremental bookkeeping: int8
    N = 4864 (64 spins more fall back to the full product), BF16 hi/lo up to
    its path limit 2496."""
    f, bits = PATHS[path]
    for N, want in ((N_max, 1), (N_off, 0)):
        if N is None:
            continue
        J, h = inst.sk_gauss_fixed(N, 1, frac_bits=f, bits=bits)
        R, T, b0, b1, L, seed = 16, 40, 0.05 * 2.0 ** (f - 5), 3.0 * 2.0 ** (f - 5), 10, 2
        geo = "1,32,0,2" if path == "i8" else "1,16,0,2"
        on = run(P, J, h, f, geo, True, R, T, b0, b1, L, seed, path=path)
        assert on["info"]["incremental"] == want
        if want:
            off = run(P, J, h, f, geo, False, R, T, b0, b1, L, seed, path=path)
            same(on, off)
            oracle_check(O, on, J, h, f, T, b0, b1, L, seed, rows=(15,))


def test_incremental_several_blocks_per_group(P, O):
    """More replica blocks than concurrent groups (G = 64 leaves room for 4
    groups on 256 CUs, 80 replicas make 5 blocks): a group's second block
    starts from a full product again."""
    J, h = inst.sk_gauss_fixed(1024, 7, frac_bits=5, bits=8)
    R, T, b0, b1, L, seed = 80, 200, 0.05, 3.0, 25, 9
    on = run(P, J, h, 5, "1,64,0,2", True, R, T, b0, b1, L, seed)
    off = run(P, J, h, 5, "1,64,0,2", False, R, T, b0, b1, L, seed)
    assert on["info"]["group"] == 64 and on["info"]["incremental"] == 1
    same(on, off)
    n_inc, n_full, _ = on["stats"]
    assert n_inc + n_full == (R // 16) * T and n_inc > 0
    oracle_check(O, on, J, h, 5, T, b0, b1, L, seed, rows=(0, 64, 79))


@pytest.mark.parametrize("path", sorted(PATHS))
def test_incremental_with_accept_reject(P, O, path):
    """The accept/reject step returns the rejected replicas to their
    trajectory start, a change of many signs at once; the incremental update
    (asked for explicitly: the default leaves it off with this step) sees it
    like any other change.  Adaptive beta multiplier, ragged R."""
    f, bits = PATHS[path]
    J, h = inst.sk_gauss_fixed(300, 5, frac_bits=f, bits=bits)
    R, T, b0, b1, L, seed, mh = 40, 300, 0.05 * 2.0 ** (f - 5), 3.0 * 2.0 ** (f - 5), 20, 3, (1.05, 0.95)
    on = run(P, J, h, f, "1,4,0,2", True, R, T, b0, b1, L, seed, path=path, mh=mh, trace=True)
    off = run(P, J, h, f, "1,4,0,2", False, R, T, b0, b1, L, seed, path=path, mh=mh, trace=True)
    dflt = run(P, J, h, f, "1,4,0,2", None, R, T, b0, b1, L, seed, path=path, mh=mh, trace=True)
    assert on["info"]["incremental"] == 1 and off["info"]["incremental"] == 0
    assert dflt["info"]["incremental"] == 0, "the default leaves it off with the accept/reject step"
    same(on, off)
    same(on, dflt)
    n_inc, n_full, _ = on["stats"]
    assert n_inc > 0 and n_full > 0
    assert on["mhc"][1].max() > 0, "decisions were taken"
    oracle_check(O, on, J, h, f, T, b0, b1, L, seed, rows=(0, 39), trace=True, mh=mh)
