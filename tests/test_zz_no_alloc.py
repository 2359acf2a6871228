"""The allocation-free anneal (phia_anneal_noalloc) against phia_anneal.

phia_anneal_noalloc takes the replica state and records in caller-owned
device buffers and keeps the kernels' scratch in a fixed device array.  Its
results must be bit-identical to phia_anneal's with the same arguments, on
two calls in a row with the second one smaller (the scratch keeps the first
call's contents), on every sweep kernel.
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


SCHED = dict(beta0=0.05, beta1=2.0, refresh_L=23)


def _noalloc(P, p, R, T, seed):
    import torch
    Np = p.info()["Np"]
    dev = torch.device("cuda", 0)
    x = torch.full((R, Np), float("nan"), dtype=torch.float32, device=dev)
    v = torch.full((R, Np), float("nan"), dtype=torch.float32, device=dev)
    bE = torch.full((R,), 7, dtype=torch.int64, device=dev)
    bS = torch.full((R, Np), 5, dtype=torch.int8, device=dev)
    bK = torch.full((R,), 7, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    E, r = p.anneal_noalloc(R, T, 0.2, 1.0, x.data_ptr(), v.data_ptr(), bE.data_ptr(), bS.data_ptr(), bK.data_ptr(),
                            seed=seed, **SCHED)
    N = p.N
    out = dict(E=bE.cpu().numpy(), S=bS.cpu().numpy(), K=bK.cpu().numpy(), x=x.cpu().numpy(), v=v.cpu().numpy(),
               best=(E, r))
    assert np.all(out["S"][:, N:] == 0) and np.all(out["x"][:, N:] == 0) and np.all(out["v"][:, N:] == 0)
    out["S"], out["x"], out["v"] = out["S"][:, :N], out["x"][:, :N], out["v"][:, :N]
    return out


def _plain(p, R, T, seed):
    p.anneal(R, T, 0.2, 1.0, seed=seed, **SCHED)
    E, S, K = p.replica_best()
    x, v, _ = p.get_state()
    e, _, r = p.best_exact()
    return dict(E=E, S=S, K=K, x=x, v=v, best=(e, r))


def _same(a, b, what):
    for key in ("E", "S", "K"):
        assert np.array_equal(a[key], b[key]), (what, key)
    for key in ("x", "v"):
        assert np.array_equal(a[key].view(np.uint32), b[key].view(np.uint32)), (what, key)
    assert a["best"] == b["best"], what


@pytest.mark.parametrize("path,geometry", [("i8", None), ("fp32", None), ("ell", None), ("bf16hilo", None), ("i8", "pp,3"),
                                           ("i8", "pp4,3"), ("i8", "ppg,3"), ("i8", "1,3,1"), ("i8", "1,4,0")])
def test_noalloc_equals_anneal_twice(P, path, geometry):
    """Two calls in a row, the second with fewer replicas and steps, each
    bit-identical to phia_anneal; the problem's own anneal is untouched."""
    J, h = inst.er_maxcut(300, 0.05, 4)
    if path == "bf16hilo":
        J, h = inst.sk_gauss_fixed(300, 4, frac_bits=12, bits=16)
    say(f"noalloc path={path} geometry={geometry}")
    if geometry:
        os.environ["PHIA_GEOMETRY"] = geometry
    try:
        p = P.Problem(J, h, path=path)
        ref1 = _plain(p, 256, 300, 11)
        info = p.info()
        say("geometry", info)
        if geometry:
            assert info["group"] == int(geometry.split(",")[1])
        got1 = _noalloc(P, p, 256, 300, 11)
        _same(ref1, got1, "first call")
        ref2 = _plain(p, 100, 120, 12)
        got2 = _noalloc(P, p, 100, 120, 12)
        _same(ref2, got2, "second call, smaller")
        # phia_anneal_noalloc leaves the problem's own anneal as it was
        E, S, K = p.replica_best()
        assert np.array_equal(E, ref2["E"]) and np.array_equal(S, ref2["S"])
    finally:
        os.environ.pop("PHIA_GEOMETRY", None)
    p.close()


def test_noalloc_rejects_what_does_not_fit(P):
    import torch
    J, h = inst.sk_pm1(40, 1)
    p = P.Problem(J, h, path="i8")
    Np = p.info()["Np"]
    bufs = [torch.zeros((4, Np), dtype=t, device="cuda") for t in (torch.float32, torch.float32)]
    bE = torch.zeros(4, dtype=torch.int64, device="cuda")
    bS = torch.zeros((4, Np), dtype=torch.int8, device="cuda")
    bK = torch.zeros(4, dtype=torch.int64, device="cuda")
    ptrs = [b.data_ptr() for b in bufs] + [bE.data_ptr(), bS.data_ptr(), bK.data_ptr()]
    with pytest.raises(P.PhiaError) as e:  # 4 bytes per step of scratch: 9e6 steps do not fit 32 MiB
        p.anneal_noalloc(4, 9_000_000, 0.2, 1.0, *ptrs, seed=1, **SCHED)
    assert e.value.code == -4
    with pytest.raises(P.PhiaError) as e:
        p.anneal_noalloc(4, 10, 0.2, 1.0, 0, 0, 0, 0, 0, seed=1, **SCHED)
    assert e.value.code == -1
    E, r = p.anneal_noalloc(4, 50, 0.2, 1.0, *ptrs, seed=1, **SCHED)
    ref = _plain(p, 4, 50, 1)
    assert (E, r) == ref["best"]
    p.close()
