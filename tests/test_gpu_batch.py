"""Batched stepping of independent systems (GPU tests, called through the C ABI).

Every system of a batch must compute exactly what it computes alone: states are
compared bit for bit with single-system runs of the same workloads, under several
launch configurations, the autotuner and graph launches.  Single-system parity
with the oracle is covered by test_gpu_parity.py.
"""
import numpy as np
import pytest

from synth import ic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_16791_amd as m
    m.lib()
    return m


def uneven_workloads():
    """Six systems of uneven size and kind: embryo disks with and without gas, a
    two-giant system with its own time step, and a disk big enough for many tiles."""
    ws = [ic.embryo_disk(seed=11, n_small=1500, n_emb=2),
          ic.embryo_disk(seed=12, n_small=4096, n_emb=8),
          ic.two_giants(seed=13, n_small=700),
          ic.embryo_disk(seed=14, n_small=257, n_emb=5, gas=False),
          ic.embryo_disk(seed=15, n_small=9000, n_emb=3),
          ic.embryo_disk(seed=16, n_small=64, n_emb=4)]
    return ws


def single_runs(mx, ws, steps):
    out = []
    for w in ws:
        s = mx.System.from_workload(w)
        s.step(steps)
        s.sync()
        x, u = s.get_dh()
        out.append((x, u, s.encounters(), s.energy()[0], s.step_index()))
        s.close()
    return out


def assert_batch_equals(b, ref, steps):
    for k, (x, u, enc, E, idx) in enumerate(ref):
        v = b.system(k)
        xb, ub = v.get_dh()
        assert np.array_equal(xb, x) and np.array_equal(ub, u), f"system {k} differs"
        assert np.array_equal(v.encounters(), enc), f"system {k} encounter list differs"
        assert v.energy()[0] == E
        assert v.step_index() == idx == steps


def test_batch_equals_single_systems(mx):
    ws = uneven_workloads()
    steps = 12
    ref = single_runs(mx, ws, steps)
    b = mx.Batch.from_workloads(ws)
    b.step(steps)
    b.sync()
    assert_batch_equals(b, ref, steps)
    # some system had encounters, so the planner and integrator ran batched
    assert sum(len(r[2]) for r in ref) > 0


@pytest.mark.parametrize("cfg", [(64, 1, 1), (128, 3, 7), (512, 8, 2), (256, 64, 1024)])
def test_batch_launch_shapes_bitwise_identical(mx, cfg):
    ws = uneven_workloads()
    steps = 8
    ref = single_runs(mx, ws, steps)
    b = mx.Batch.from_workloads(ws)
    b.set_config(*cfg)
    assert b.config() == cfg
    b.step(steps)
    b.sync()
    assert_batch_equals(b, ref, steps)


def test_batch_with_big_components_and_long_lists(mx):
    """Systems whose encounter lists take the general plan (big-big pairs; more
    than 256 pairs) next to systems on the common plan, in one launch: each must
    still compute exactly what it computes alone."""
    from test_gpu_parity import _planets_with_cloud
    ws = [ic.embryo_disk(seed=21, n_small=900, n_emb=3),
          _planets_with_cloud(n_far=60, k=40, close_pair=True),
          ic.embryo_disk(seed=22, n_small=300, n_emb=2),
          _planets_with_cloud(n_far=20, k=320, close_pair=False)]
    steps = 3
    ref = single_runs(mx, ws, steps)
    for cfg in [(128, 1, 4), (256, 2, 1)]:
        b = mx.Batch.from_workloads(ws)
        b.set_config(*cfg)
        b.step(steps)
        b.sync()
        assert_batch_equals(b, ref, steps)
        b.close()
    assert max(len(r[2]) for r in ref) > 256
    assert any(np.any(np.asarray(r[2])[:, 1] < 3) for r in ref if len(r[2]))


def test_batch_autotune_and_graph_launch(mx):
    ws = uneven_workloads()
    b = mx.Batch.from_workloads(ws)
    taken, cfg, ms = b.autotune(steps_per_candidate=1)
    assert taken == 1 + 16 + 2 * 4 and ms > 0.0
    assert cfg[0] in (64, 128, 256, 512) and cfg[2] in (8, 16, 32, 64) and b.config() == cfg
    b.set_launch_mode("graph", steps_per_graph=4)
    b.step(10)       # two graph replays and two eager steps
    b.step(4)        # one replay of the same graph
    b.sync()
    ref = single_runs(mx, ws, taken + 14)
    assert_batch_equals(b, ref, taken + 14)


def test_batch_member_steps_alone_and_errors(mx):
    ws = uneven_workloads()[:3]
    b = mx.Batch.from_workloads(ws)
    v = b.system(1)
    v.step(5)        # a member can be advanced on its own with the same kernels
    v.sync()
    v.close()        # closing a view leaves the member to the batch
    ref = single_runs(mx, [ws[1]], 5)[0]
    xb, ub = b.system(1).get_dh()
    assert np.array_equal(xb, ref[0]) and np.array_equal(ub, ref[1])
    b.step(2)
    b.sync()
    assert b.system(1).step_index() == 7 and b.system(0).step_index() == 2
    with pytest.raises(mx.MxError):
        b.set_config(100, 1, 1)
    with pytest.raises(mx.MxError):
        b.system(3)
    keep = b.system(2)
    b.close()             # views of a closed batch refuse to run
    with pytest.raises(mx.MxError):
        keep.step(1)
    del keep
    big = ic.self_gravitating(seed=0, n_pl=4, n_pls=100)  # 104 massive bodies
    with pytest.raises(mx.MxError) as e:
        mx.Batch.from_workloads([ws[0], big])
    assert e.value.code == -1


def test_full_batch_members_match_oracle(mx, orc):
    """The 256-system ensemble the benchmark runs (3.2 M bodies), at the autotuned
    launch shape: its smallest, median and largest members against the oracle, per
    step from the same state, for three steps."""
    from parity_helpers import compare_pairs, relerr_per_body, step_close
    ws = ic.batch(seed=0, n_sys=256)
    sizes = np.array([w.n for w in ws])
    order = np.argsort(sizes, kind="stable")
    picks = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    keep = {k: ws[k] for k in picks}
    b = mx.Batch.from_workloads(ws)
    del ws
    b.autotune(steps_per_candidate=1)
    ors = {k: orc.OracleSystem.from_workload(keep[k]) for k in picks}
    for step in range(3):
        before = {k: b.system(k).get_dh() for k in picks}
        idx = b.system(picks[0]).step_index()
        b.step(1)
        b.sync()
        for k in picks:
            o = ors[k]
            x, u = before[k]
            o.set_dh(x, u, idx)
            o.step(1)
            v = b.system(k)
            xg, ug = v.get_dh()
            xo, uo = o.get_dh()
            nb = keep[k].params["n_big"]
            excluded, n_border, big = compare_pairs(o, v.encounters(), o.encounters(), xo, nb)
            assert not big
            ex, eu, bad_x, bad_u = step_close(xg, ug, xo, uo, excluded)
            print(f"[parity] batch member {k} (n={xo.shape[1]}) step {step}: pairs "
                  f"{len(o.encounters())}, borderline {n_border}, max rel err x {ex:.2e} u {eu:.2e}")
            assert bad_x.size == 0 and bad_u.size == 0, (k, step, ex, eu)
