"""Host-side helpers of the experiments and of bench.py, on the CPU: block
means of the precision report, the settling time and curvature of the
gradient-formation summary, the Poiseuille profile error of the boundary
comparison, and the digest of counter runs into HBM bytes per launch."""
import csv
import json

import numpy as np
import pytest

import bench
from paper_1307_4703_amd import experiments as E


def test_block_means_fluid_only():
    a = np.arange(16 * 16, dtype=float).reshape(16, 16)
    fluid = np.ones_like(a, bool)
    fluid[:8, :8] = False          # one block without fluid
    fluid[8, 8] = False            # one node out of another block
    m = E.block_means(a, fluid)
    assert m.shape == (2, 2)
    assert np.isnan(m[0, 0])
    blk = a[8:16, 8:16].copy()
    assert m[1, 1] == pytest.approx((blk.sum() - a[8, 8]) / 63)
    assert m[0, 1] == pytest.approx(a[:8, 8:].mean())


def test_time_to_settle_and_curvature():
    t = np.linspace(0.0, 4.0, 401)
    c = np.where(t < 2.0, 1 - np.exp(-t / 0.2), np.exp(-(t - 2.0) / 0.5))
    # 90 % of the rise after t = 0: 0.2 ln 10 hours (to the sample spacing)
    assert E.time_to_settle(t, c, 0.0, 1.99) == pytest.approx(0.2 * np.log(10), abs=0.011)
    # the fall after the swap at 2 h, measured to the value at the last
    # sample before t_to (exp(-3.98), not 0)
    end = np.exp(-1.98 / 0.5)
    goal = 1.0 + 0.9 * (end - 1.0)
    assert E.time_to_settle(t, c, 2.0, 3.99) == pytest.approx(-0.5 * np.log(goal), abs=0.011)
    assert E.time_to_settle(t, np.ones_like(t), 0.0, 2.0) is None
    assert E.curvature([1.0, 0.75, 0.5, 0.25, 0.0]) == pytest.approx(0.0)
    assert E.curvature([1.0, 0.4, 0.25, 0.1, 0.0]) == pytest.approx(-0.25)


def test_poiseuille_error_of_an_exact_parabola():
    """A profile that is the parabola of the pressure gradient it sits in
    has no error, and the centre speed follows G H^2 / (8 nu rho)."""
    H, nu, nx = 30, 0.1, 101
    G = 1e-6
    s = np.arange(1, H + 1) - 0.5
    u = G * s * (H - s) / (2 * nu)
    x = np.arange(nx)
    rho = 1.0 - 3 * G * (x - nx // 2)          # p = rho / 3 falls by G per cell
    rho = np.broadcast_to(rho[None, :], (H + 2, nx)).copy()
    ux = np.zeros((H + 2, nx))
    ux[1:-1, :] = u[:, None]
    err, umax = E._poiseuille_error(rho, ux, H, nu, nx // 2)
    assert err < 1e-12
    assert umax == pytest.approx(G * H * H / (8 * nu), rel=1e-12)


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, grid, value in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                        "Counter_Value": value})


def test_digest_scales_counters_by_the_copy_kernel(tmp_path):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of each leg are scaled by
    what they read for the copy kernel of known size in the same run,
    averaged over the dispatches of the kernel (and grid) the leg's
    manifest names, and set against the manifest's algorithmic bytes."""
    copy_grid = 1024                               # 1024 lanes x 16 B each way
    nbytes = copy_grid * 16
    pf = tmp_path / "lattices_fetch"
    pw = tmp_path / "lattices_write"
    pf.mkdir()
    pw.mkdir()
    kern = "void gg::(anonymous namespace)::k_tile2<double, false, 14, false, false>(x)"
    other = "void gg::(anonymous namespace)::k_tile2<double, false, 14, false, false>(x)"
    # the copy reads half of its bytes per FETCH_SIZE unit, writes all
    _counter_csv(pf / "fetch_counter_collection.csv", "FETCH_SIZE",
                 [("gg::k_copy(y)", copy_grid, nbytes / 1024 / 2),
                  (kern, 647168, 1000.0), (kern, 647168, 1200.0), (other, 1024, 9.0)])
    _counter_csv(pw / "write_counter_collection.csv", "WRITE_SIZE",
                 [("gg::k_copy(y)", copy_grid, nbytes / 1024),
                  (kern, 647168, 500.0), (kern, 647168, 500.0), (other, 1024, 9.0)])
    (tmp_path / "counters_lattices.json").write_text(json.dumps(
        {"straight_f64": {"kernel": "k_tile2<double, false, 14,", "grid": 647168,
                          "units": 2000, "bytes_per_update": 225}}))
    out = tmp_path / "traffic.json"
    d = bench.digest_counters(str(tmp_path), str(out))
    leg = d["legs"]["lattices"]
    assert leg["fetch_scale"] == pytest.approx(2.0) and leg["write_scale"] == pytest.approx(1.0)
    w = d["workloads"]["straight_f64"]
    assert w["fetch_bytes_per_launch"] == round(1100.0 * 1024 * 2)
    assert w["write_bytes_per_launch"] == 500 * 1024
    assert w["algorithmic_bytes_per_launch"] == 2000 * 225
    assert w["bytes_per_launch"] == round(1100.0 * 1024 * 2) + 500 * 1024
    assert json.loads(out.read_text())["kernel_sha"] == bench.kernel_hash()


def test_digest_sums_the_kernels_of_a_pass(tmp_path):
    """sum_kernels: a pass of two kernels (interior and boundary tiles, one
    launch each per pass) counts the sum of their per-dispatch means."""
    copy_grid = 1024
    nbytes = copy_grid * 16
    (tmp_path / "batch_fetch").mkdir()
    (tmp_path / "batch_write").mkdir()
    k1 = "void gg::(anonymous namespace)::k_tile4<float, false, 6, true>(x)"
    k2 = "void gg::(anonymous namespace)::k_tile4<float, true, 2, true>(x)"
    _counter_csv(tmp_path / "batch_fetch" / "f_counter_collection.csv", "FETCH_SIZE",
                 [("gg::k_copy(y)", copy_grid, nbytes / 1024), (k1, 7680, 100.0), (k1, 7680, 300.0),
                  (k2, 512, 10.0), (k2, 512, 30.0)])
    _counter_csv(tmp_path / "batch_write" / "w_counter_collection.csv", "WRITE_SIZE",
                 [("gg::k_copy(y)", copy_grid, nbytes / 1024), (k1, 7680, 50.0), (k1, 7680, 50.0),
                  (k2, 512, 5.0), (k2, 512, 5.0)])
    (tmp_path / "counters_batch.json").write_text(json.dumps(
        {"batch64": {"kernel": "k_tile4<float,", "grid": None, "sum_kernels": True,
                     "units": 100, "bytes_per_update": 113}}))
    d = bench.digest_counters(str(tmp_path), str(tmp_path / "t.json"))
    w = d["workloads"]["batch64"]
    assert w["fetch_bytes_per_launch"] == (200 + 20) * 1024
    assert w["write_bytes_per_launch"] == (50 + 5) * 1024


def test_bench_alignment_steps():
    # the timed region starts where a run of two-step passes can start
    for t in range(0, 13):
        a = bench.align_steps(t)
        assert 0 <= a < 4 and (t + a) % 4 == 0


def test_monitor_interval_ends_on_the_last_step():
    assert bench.monitor_interval(0, 1024) == 0
    assert bench.monitor_interval(20, 1024) == 20
    assert bench.monitor_interval(4000, 1024) == 1000
    assert bench.monitor_interval(4096, 1024) == 1024
    for steps in (1025, 3000, 5000, 12345, 20000):
        m = bench.monitor_interval(steps, 1024)
        assert 1 <= m <= 1024
        if any(steps % d == 0 for d in range(512, 1025)):
            assert steps % m == 0 and m >= 512


def _fake_run(nf, steps, event_ms, prof):
    return {"nf": nf, "steps": steps, "event_ms": event_ms, "prof": prof}


def test_bench_roofline_pass_and_single():
    prof = {"n_pass": 10, "ms_pass": 1.0, "n_single": [0, 0], "ms_single": [0.0, 0.0],
            "n_graph": 0, "ms_graph": 0.0, "graph_passes": 0, "graph_singles": 0,
            "pass_fluid": 1000000, "fuse": 3}
    r = _fake_run(1100000, 20, 2.0, prof)
    out = bench.roofline(r, "f16", traffic=None)
    # two updates of 57 B per fluid node of the pass's tiles per launch
    assert out["algorithmic_bytes_per_launch"] == 2 * 1000000 * 57
    assert out["kernel_ms"] == pytest.approx(0.1)
    assert out["achieved"] == pytest.approx(2 * 1000000 * 57 / 1e-4 / 1e9, rel=1e-3)
    assert out["frac"] == pytest.approx(out["achieved"] / 8000.0, rel=1e-3)
    assert "traffic_frac" not in out
    out = bench.roofline(r, "f16", traffic=60000000)
    assert out["traffic_gbs"] == pytest.approx(60000000 / 1e-4 / 1e9, rel=1e-3)
    assert out["traffic_per_algorithmic_single_trip"] == pytest.approx(60 / 57, rel=1e-3)
    prof = {"n_pass": 0, "ms_pass": 0.0, "n_single": [3, 2], "ms_single": [0.3, 0.2],
            "n_graph": 0, "ms_graph": 0.0, "graph_passes": 0, "graph_singles": 0,
            "pass_fluid": 0, "fuse": 1}
    out = bench.roofline(_fake_run(500000, 5, 1.0, prof), "f32", traffic=None)
    assert out["algorithmic_bytes_per_launch"] == 500000 * 113
    assert out["kernel_ms"] == pytest.approx(0.1)
    # graph replays: their duration over the passes they hold
    prof = {"n_pass": 2, "ms_pass": 0.2, "n_single": [0, 0], "ms_single": [0.0, 0.0],
            "n_graph": 1, "ms_graph": 0.8, "graph_passes": 8, "graph_singles": 0,
            "pass_fluid": 1000000, "fuse": 3}
    out = bench.roofline(_fake_run(1100000, 20, 2.0, prof), "f16", traffic=None)
    assert out["launches_timed"] == 10 and out["launches_in_graph_replays"] == 8
    assert out["kernel_ms"] == pytest.approx(0.1)
    # every pass inside graph replays (the driver's 20 steps): still one
    # trip per pass launch
    prof = {"n_pass": 0, "ms_pass": 0.0, "n_single": [0, 0], "ms_single": [0.0, 0.0],
            "n_graph": 1, "ms_graph": 1.0, "graph_passes": 10, "graph_singles": 0,
            "pass_fluid": 1000000, "fuse": 3}
    out = bench.roofline(_fake_run(1100000, 20, 2.0, prof), "f16", traffic=60000000)
    assert out["traffic_per_algorithmic_single_trip"] == pytest.approx(60 / 57, rel=1e-3)
    # the four-step pass: four updates of its tiles' nodes per launch, and
    # one trip through memory for them
    prof = dict(prof, steps_per_pass=4, fuse=5)
    out = bench.roofline(_fake_run(1100000, 20, 2.0, prof), "f32", traffic=120000000)
    assert out["algorithmic_bytes_per_launch"] == 4 * 1000000 * 113
    assert out["kernel"].startswith("four-step")
    assert out["traffic_per_algorithmic_single_trip"] == pytest.approx(120 / 113, rel=1e-3)


def test_bench_refuses_several_gpus():
    with pytest.raises(SystemExit) as e:
        bench.main(["--gpus", "2"])
    assert e.value.code == 2


def test_snapshot_slots_follow_both_layouts():
    """The snapshot reader of the tests: the element of population i of a
    node in each layout (paired: f_i, g_i side by side for i < 5, f5..f8 in
    planes 10..13), and the planes gathered back in population order."""
    from tests.parity_util import snapshot_planes, snapshot_slot, SNAP_DATA
    plane = 8
    for pairs in (0, 1):
        h = {"pairs": pairs, "plane": plane}
        slots = {(i, n): snapshot_slot(h, i, n) for i in range(14) for n in range(plane // 2)}
        assert len(set(slots.values())) == len(slots)  # no two share an element
        assert all(0 <= v < 14 * plane for v in slots.values())
        if pairs:
            for i in range(5):
                assert slots[(9 + i, 3)] == slots[(i, 3)] + 1
        hdr = (b"GGLBMSNP" + np.array([2, 4, 1, 1, pairs, 0], np.int32).tobytes()
               + np.array([8, plane, 0], np.int64).tobytes())
        assert len(hdr) == SNAP_DATA
        data = np.zeros(14 * plane, np.float32)
        for (i, n), v in slots.items():
            data[v] = 100 * i + n
        got = snapshot_planes(hdr + data.tobytes(), np.float32)
        for (i, n) in slots:
            assert got[i, n] == 100 * i + n
