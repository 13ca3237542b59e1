"""bench.py under the arguments the benchmark driver passes (and an odd
combination): one JSON line with the roofline block, the timed steps all
accounted for, and the monitor reductions inside the timed region."""
import json

import pytest

import bench

pytestmark = pytest.mark.gpu


def _run(capsys, argv):
    out = bench.main(argv)
    lines = [l for l in capsys.readouterr().out.splitlines() if l.strip()]
    assert len(lines) == 1
    line = json.loads(lines[0])
    assert line == json.loads(json.dumps(out))
    return line


@pytest.mark.parametrize("argv, workload", [
    (["--gpus", "1", "--steps", "20", "--warmup", "5"], "gradient_generator_8192x4096"),
    (["--gpus", "1", "--steps", "7", "--warmup", "3", "--workload", "gg2048_f32"],
     "gradient_generator_2048x1024"),
])
def test_bench_line(capsys, argv, workload):
    line = _run(capsys, argv + ["--no-extra", "--no-cpu-baseline"])
    steps = int(argv[argv.index("--steps") + 1])
    assert line["steps"] == steps and line["n_gpus"] == 1
    assert line["config"]["workload"] == workload
    assert line["value"] > 0 and line["ms_per_step"] > 0
    launches = line["config"]["launches"]
    # every timed step is a step of a pass (two per launch, four with the
    # four-step pass, whose leftover runs of four steps go in two-step
    # passes counted apart) or a single step, plain or inside a graph
    # replay of the timed steps rounded down to 4 (to 8 with the four-step
    # pass)
    spp = launches["steps_per_pass"]
    q = 2 * spp
    assert (spp * launches["pass_kernel"] + 2 * launches["two_step_pass_beside_four_step"] +
            launches["single_even"] + launches["single_odd"] +
            launches["single_in_graph_replays"]) == steps
    assert launches["pass_kernel"] == steps // q * 2
    assert launches["pass_kernel_in_graph_replays"] == steps // q * 2
    assert line["config"]["graph_chunk"] == steps // q * q
    assert spp == (4 if workload == "gradient_generator_2048x1024" else 2)
    assert line["config"]["warmup_steps_run"] % 4 == 0
    rf = line["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["achieved"] > 0 and rf["frac"] == pytest.approx(rf["achieved"] / 8000.0, rel=1e-3)
    assert line["config"]["monitor_reductions"] >= 1
    d = line["diagnostics"]
    assert d["n_nonfinite"] == 0 and d["mass"] > 0
