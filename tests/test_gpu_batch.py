"""Batched stepping: uneven lattices in one fused launch per step must give
every member exactly the result it gets alone."""
import numpy as np
import pytest

from conftest import say
from paper_1806_10241_amd import inputs as I

pytestmark = pytest.mark.gpu


def members():
    cases = [I.annulus_convection(Nr=48 + 17 * k, Nz=50 + 23 * k, Ra=10 ** (3 + 0.5 * k),
                                  radius_ratio=1.5 + 0.5 * k, seed=40 + k) for k in range(4)]
    cases.append(I.rotating_lid_cylinder(Nr=37, Nz=61, Re=300.0, Ri=0.3, seed=45))
    cases.append(I.couette_poiseuille_conduction(Nr=30, Nz=8))
    return cases


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_batch_equals_alone(gpu, storage):
    say("batch vs alone", storage)
    from paper_1806_10241_amd import axlb
    cases = members()
    alone = [axlb.Lattice(c, storage=storage) for c in cases]
    batched = [axlb.Lattice(c, storage=storage) for c in cases]
    # members may join with different phases
    alone[1].step(1)
    batched[1].step(1)
    b = axlb.Batch(batched)
    for tile, blocks in ((0, 0), (3, 0), (5, 2048), (7, 64)):
        b.set_schedule(tile, blocks)
        b.step(113)
    b.sync()
    for lat in alone:
        lat.step(4 * 113)
    for la, lb in zip(alone, batched):
        assert lb.steps == la.steps
        assert la.save() == lb.save()
        fa, fb = la.fields(), lb.fields()
        for k in fa:
            assert np.array_equal(fa[k], fb[k])
    b.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_whole_members_equal_alone(gpu, storage):
    """Members of at most WHOLE_MAX_NODES nodes run one per workgroup, a
    bundle per launch with a workgroup barrier per step, beside a member too
    large for the mode on the work-list: after bundles, single steps and an
    odd count every member equals stepping alone bit for bit, also when the
    mode is switched mid-run, and a member joins with the other phase."""
    say("whole members", storage)
    from paper_1806_10241_amd import axlb
    cases = members()
    cases.append(I.annulus_convection(Nr=300, Nz=260, Ra=1e4, seed=49))  # 78000 nodes
    cases.append(I.couette_poiseuille_conduction(Nr=2, Nz=3))
    alone = [axlb.Lattice(c, storage=storage) for c in cases]
    batched = [axlb.Lattice(c, storage=storage) for c in cases]
    alone[2].step(1)
    batched[2].step(1)
    b = axlb.Batch(batched)
    b.set_whole(axlb.WHOLE_MAX_NODES)
    small = sum(c["Nr"] * c["Nz"] <= axlb.WHOLE_MAX_NODES for c in cases)
    assert b.whole() == (axlb.WHOLE_MAX_NODES, small) and small == len(cases) - 1
    b.step(237)
    b.set_whole(0)
    assert b.whole() == (0, 0)
    b.step(3)
    b.set_whole(5000)
    b.step(101)
    b.sync()
    for lat in alone:
        lat.step(341)
    for la, lb in zip(alone, batched):
        assert lb.steps == la.steps
        assert la.save() == lb.save()
    lib = axlb.load()
    assert lib.axlb_batch_set_whole(b._h, axlb.WHOLE_MAX_NODES + 1) == axlb.EINVAL
    assert lib.axlb_batch_set_whole(b._h, -1) == axlb.EINVAL
    b.close()


def test_cache_groups_on_two_streams_equal_alone(gpu):
    """Members whose states exceed one cache group: a bundle splits them into
    groups that alternate between two streams; every member still ends
    bit-identical to stepping alone (two bundles and a partial one)."""
    say("batch groups on two streams")
    from paper_1806_10241_amd import axlb
    cases = [I.annulus_convection(Nr=640, Nz=512, Ra=10 ** (3 + 0.4 * k), seed=70 + k)
             for k in range(6)]
    assert sum(axlb.state_bytes(c["Nr"], c["Nz"]) for c in cases) > 3 * (80 << 20) // 2
    alone = [axlb.Lattice(c) for c in cases]
    batched = [axlb.Lattice(c) for c in cases]
    b = axlb.Batch(batched)
    b.step(237)
    b.sync()
    for lat in alone:
        lat.step(237)
    for la, lb in zip(alone, batched):
        assert la.save() == lb.save()
    b.close()


def test_batch_autotune_restores_state_and_members_are_locked(gpu):
    say("batch autotune")
    from paper_1806_10241_amd import axlb
    cases = members()
    a = [axlb.Lattice(c) for c in cases]
    ref = [axlb.Lattice(c) for c in cases]
    b = axlb.Batch(a)
    tile, blocks, ms = b.autotune(steps_per_trial=4)
    assert (tile, blocks) == b.schedule()
    assert np.all(ms > 0)
    lib = axlb.load()
    assert lib.axlb_step(a[0].handle, 1) == axlb.ESTATE
    assert lib.axlb_set_fields(a[0].handle, None, None, None, None, None) == axlb.ESTATE
    b.step(150)
    b.sync()
    for lat in ref:
        lat.step(150)
    for x, y in zip(a, ref):
        assert x.save() == y.save()
    m, nodes = b.size()
    assert m == len(cases) and nodes == sum(c["Nr"] * c["Nz"] for c in cases)
    b.close()
    a[0].step(1)  # released from the batch


def test_step_each_matches_single_lattices(gpu):
    say("step_each")
    from paper_1806_10241_amd import axlb
    cases = members()[:3]
    a = [axlb.Lattice(c) for c in cases]
    ref = [axlb.Lattice(c) for c in cases]
    axlb.step_each(a, 37)
    for lat in ref:
        lat.step(37)
    for x, y in zip(a, ref):
        assert x.save() == y.save()


def test_batched_workload_members_match_oracle(gpu, orc):
    """The 256-instance batched workload stepped 1000 times in one fused
    launch per step (100-step graph bundles): 8 sampled members against the
    FP64 oracle (the 8 smallest, so that the oracle finishes in seconds), to
    the FP32 parity bars."""
    from test_gpu_parity import TOL, TOL_DRHO, assert_parity, field_errors
    say("batched workload vs oracle")
    from paper_1806_10241_amd import axlb
    cases = I.batched_annuli(256, seed=4)
    lats = [axlb.Lattice(c) for c in cases]
    b = axlb.Batch(lats)
    b.step(1000)
    b.sync()
    sample = sorted(range(len(cases)), key=lambda k: cases[k]["Nr"] * cases[k]["Nz"])[:8]
    for k in sample:
        c = cases[k]
        ref = orc.Lattice(c, deriv_mode=orc.DERIV_PREVIOUS, fields=c["fields"]())
        ref.step(1000)
        got, want = lats[k].fields(), ref.fields()
        say("  member %d (%d x %d): %s" % (k, c["Nr"], c["Nz"], {
            f: "%.2e" % e for f, (e, _) in field_errors(got, want).items()}))
        assert_parity(got, want, TOL["f32"], "member %d" % k, TOL_DRHO["f32"])
    b.close()


def test_batch_with_degenerate_members_equals_alone(gpu):
    """Members with one or two rows or columns next to ordinary ones."""
    say("batch with degenerate members")
    from paper_1806_10241_amd import axlb
    cases = [I.couette_poiseuille_conduction(Nr=65, Nz=1, r_inner=5.0),
             I.couette_poiseuille_conduction(Nr=2, Nz=3, r_inner=5.0),
             I.rotating_lid_cylinder(Nr=3, Nz=2, Re=50.0, Ri=0.5),
             I.annulus_convection(Nr=70, Nz=66, Ra=1e4, seed=81)]
    alone = [axlb.Lattice(c) for c in cases]
    batched = [axlb.Lattice(c) for c in cases]
    b = axlb.Batch(batched)
    b.step(150)
    b.sync()
    for lat in alone:
        lat.step(150)
    for la, lb in zip(alone, batched):
        assert la.save() == lb.save()
    b.close()


def test_destroying_a_batched_member_is_refused(gpu):
    """A batch keeps stepping its members' memory: destroying a member while
    the batch lives is refused (nothing released), and the member keeps
    stepping with the batch; after the batch is gone it can be closed."""
    say("destroy a batched member")
    from paper_1806_10241_amd import axlb
    cases = members()[:3]
    a = [axlb.Lattice(c) for c in cases]
    ref = axlb.Lattice(cases[0])
    b = axlb.Batch(a)
    lib = axlb.load()
    assert lib.axlb_destroy(a[0].handle) == axlb.ESTATE
    assert b"batch" in lib.axlb_last_error(a[0].handle)
    with pytest.raises(axlb.AxlbError) as e:
        a[0].close()
    assert e.value.code == axlb.ESTATE
    assert a[0].handle and a[0]._buf is not None
    b.step(120)
    b.sync()
    ref.step(120)
    assert a[0].save() == ref.save()
    b.close()
    for lat in a:
        lat.close()
    assert not a[0].handle


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_two_step_batch_equals_alone(gpu, storage):
    """A batch of AB2 members (two steps per launch over all members) gives
    every member the result it gets alone, through graph bundles, plain
    pairs and odd single steps, members joining with either buffer current;
    degenerate members included."""
    say("two-step batch vs alone", storage)
    from paper_1806_10241_amd import axlb
    cases = members() + [I.couette_poiseuille_conduction(Nr=65, Nz=1, r_inner=5.0),
                         I.rotating_lid_cylinder(Nr=3, Nz=2, Re=50.0, Ri=0.5)]
    alone = [axlb.Lattice(c, storage=storage, layout="ab2") for c in cases]
    batched = [axlb.Lattice(c, storage=storage, layout="ab2") for c in cases]
    alone[1].step(1)
    batched[1].step(1)
    b = axlb.Batch(batched)
    for n in (101, 100, 3, 2, 1):
        b.step(n)
    b.sync()
    for lat in alone:
        lat.step(207)
    for la, lb in zip(alone, batched):
        assert lb.steps == la.steps
        assert la.save() == lb.save()
    with pytest.raises(axlb.AxlbError):
        b.set_schedule(0, 0)
    b.close()


def test_two_step_batched_workload_members_match_oracle(gpu, orc):
    """The 256-instance batched workload as AB2 members, 1000 steps: 8
    sampled members against the FP64 oracle at the FP32 parity bars."""
    from test_gpu_parity import TOL, TOL_DRHO, assert_parity, field_errors
    say("two-step batched workload vs oracle")
    from paper_1806_10241_amd import axlb
    cases = I.batched_annuli(256, seed=4)
    lats = [axlb.Lattice(c, layout="ab2") for c in cases]
    b = axlb.Batch(lats)
    b.step(1000)
    b.sync()
    sample = sorted(range(len(cases)), key=lambda k: cases[k]["Nr"] * cases[k]["Nz"])[:8]
    for k in sample:
        c = cases[k]
        ref = orc.Lattice(c, deriv_mode=orc.DERIV_PREVIOUS, fields=c["fields"]())
        ref.step(1000)
        got, want = lats[k].fields(), ref.fields()
        say("  member %d (%d x %d): %s" % (k, c["Nr"], c["Nz"], {
            f: "%.2e" % e for f, (e, _) in field_errors(got, want).items()}))
        assert_parity(got, want, TOL["f32"], "member %d" % k, TOL_DRHO["f32"])
    b.close()


def test_batch_members_share_one_layout(gpu):
    from paper_1806_10241_amd import axlb
    cases = members()[:2]
    lats = [axlb.Lattice(cases[0], layout="aa"), axlb.Lattice(cases[1], layout="ab2")]
    with pytest.raises(axlb.AxlbError):
        axlb.Batch(lats)
    with pytest.raises(axlb.AxlbError):
        axlb.Batch([axlb.Lattice(cases[0], layout="ab")])


def test_two_step_batch_groups_on_two_streams_equal_alone(gpu):
    """AB2 members whose states exceed one cache group: the bundle's 50
    two-step launches run group by group on two streams; every member
    still ends bit-identical to stepping alone (two bundles and a partial
    one)."""
    say("two-step batch groups on two streams")
    from paper_1806_10241_amd import axlb
    cases = [I.annulus_convection(Nr=640, Nz=512, Ra=10 ** (3 + 0.4 * k), seed=90 + k)
             for k in range(5)]
    assert sum(axlb.state_bytes(c["Nr"], c["Nz"], layout="ab2") for c in cases) > 2 * (80 << 20)
    alone = [axlb.Lattice(c, layout="ab2") for c in cases]
    batched = [axlb.Lattice(c, layout="ab2") for c in cases]
    b = axlb.Batch(batched)
    b.step(237)
    b.sync()
    for lat in alone:
        lat.step(237)
    for la, lb in zip(alone, batched):
        assert la.save() == lb.save()
    b.close()
