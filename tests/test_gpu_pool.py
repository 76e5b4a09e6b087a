"""Continuous-batching pool: admission by memory budget, requests joining
while others run, and every result identical to the same case run alone."""
import numpy as np
import pytest

from conftest import say
from paper_1806_10241_amd import inputs as I

pytestmark = pytest.mark.gpu


def requests():
    return [
        (I.annulus_convection(Nr=48, Nz=64, Ra=1e4, seed=61), "f32"),
        (I.rotating_lid_cylinder(Nr=40, Nz=80, Re=200.0, Ri=0.2, seed=62), "f16"),
        (I.annulus_convection(Nr=96, Nz=80, Ra=1e5, radius_ratio=3.0, seed=63), "f32"),
        (I.couette_poiseuille_conduction(Nr=30, Nz=8), "bf16"),
        (I.rotating_lid_cylinder(Nr=64, Nz=64, Re=400.0, Ri=0.0, seed=64), "f32"),
    ]


def pool_layout(storage):
    """The layout the pool gives a request of this storage."""
    return "ab2" if storage == "f32" else "aa"


def test_pool_results_equal_alone(gpu):
    say("pool vs alone")
    from paper_1806_10241_amd import axlb
    reqs = requests()
    sizes = [axlb.state_bytes(c["Nr"], c["Nz"], st, pool_layout(st)) for c, st in reqs]
    pool = axlb.Pool(budget_bytes=sizes[0] + sizes[1] + sizes[2])
    ids = [pool.submit(c, st, tol=0.0, max_steps=300) for c, st in reqs[:2]]
    assert pool.tick() == (2, 0)
    ids += [pool.submit(c, st, tol=0.0, max_steps=300) for c, st in reqs[2:]]
    peak = 0
    for _ in range(20):
        run, queued = pool.tick()
        peak = max(peak, run)
        if run == 0 and queued == 0:
            break
    assert peak <= 3
    for rid, (c, st) in zip(ids, reqs):
        state, steps, _ = pool.status(rid)
        assert state == axlb.REQ_DONE and steps == 300
        got, nu = pool.result(rid)
        lat = axlb.Lattice(c, storage=st, layout=pool_layout(st))
        lat.step(300)
        ref = lat.fields()
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (rid, k)
    pool.close()


def test_pool_retires_on_residual(gpu):
    say("pool residual retirement")
    from paper_1806_10241_amd import axlb
    pool = axlb.Pool(budget_bytes=1 << 30)
    c = I.couette_poiseuille_conduction(Nr=30, Nz=8)
    rid = pool.submit(c, "f32", tol=1e-6, max_steps=10 ** 6)
    for _ in range(2000):
        run, queued = pool.tick()
        if run == 0:
            break
    state, steps, res = pool.status(rid)
    assert state == axlb.REQ_DONE and res < 1e-6 and steps < 10 ** 6
    F, nu = pool.result(rid)
    assert abs(nu[0] - 1 / np.log(4)) < 0.04


def test_pool_rejects_requests_above_the_budget(gpu):
    say("pool budget")
    from paper_1806_10241_amd import axlb
    pool = axlb.Pool(budget_bytes=1 << 20)
    with pytest.raises(axlb.AxlbError) as e:
        pool.submit(I.annulus_convection(Nr=256, Nz=256), "f32")
    assert e.value.code == axlb.ENOMEM


def test_pool_smallest_first_with_node_window(gpu):
    """SMALLEST_FIRST admits the least Nr*Nz*max_steps first, the node
    window keeps the rest queued, and a request larger than the window runs
    once it is alone; FIFO keeps arrival order."""
    say("pool policy")
    from paper_1806_10241_amd import axlb
    big = I.annulus_convection(Nr=96, Nz=96, Ra=1e4, seed=71)
    mid = I.annulus_convection(Nr=64, Nz=64, Ra=1e4, seed=72)
    small = I.annulus_convection(Nr=32, Nz=48, Ra=1e4, seed=73)
    for order, first in (("smallest", "small"), ("fifo", "big")):
        pool = axlb.Pool(budget_bytes=1 << 30, order=order, node_window=64 * 64 + 32 * 48)
        ids = {name: pool.submit(c, "f32", tol=0.0, max_steps=200)
               for name, c in (("big", big), ("mid", mid), ("small", small))}
        pool.tick()
        running = {n for n, rid in ids.items() if pool.status(rid)[0] == axlb.REQ_RUNNING}
        if order == "smallest":
            assert running == {"small", "mid"}
        else:
            assert running == {"big"}          # the head blocks, and exceeds the window alone
        for _ in range(40):
            run, queued = pool.tick()
            if run == 0 and queued == 0:
                break
        for name, rid in ids.items():
            assert pool.status(rid)[0] == axlb.REQ_DONE and pool.status(rid)[1] == 200, name
            pool.result(rid)
        with pytest.raises(axlb.AxlbError):
            pool.set_policy("fifo", -1)
        pool.close()
