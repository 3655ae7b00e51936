"""CPU checks of the launch plan: host builds of the library's layout code."""
import model_build


def test_segment_test_queue_holds_every_append():
    """Every accepted segment-test tile shape (64 x mark_words pixels by mark_rows):
    each wave's pre-test queue segment holds the most pixels the wave can append."""
    exe = model_build.build("lds_capacity", ["lds_capacity.cpp"])
    res = model_build.run(exe)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip() == "ok 244"


SCENARIOS = ["tuner_c2", "tuner_cell0", "tuner_c3", "bench_legs", "served", "test_shapes",
             "scratch"]


def test_launch_model_every_launch_in_bounds():
    """The library's host code (of_api.cpp), built for the host with AddressSanitizer and
    UndefinedBehaviorSanitizer, drives a model of every kernel launch: the tuner's trial
    sequence on one resident workspace, every benchmark leg, served batches of mixed
    sizes and the GPU tests' shapes.  Every block's global and LDS accesses (at the
    extremes the data can reach) stay inside their buffers and regions, every tile is
    taken once per launch, and each call leaves the state the next call expects."""
    exe = model_build.build(
        "launch_model", ["launch_model.cpp", "../../paper_2506_07164_amd/csrc/of_api.cpp"],
        extra=["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer"])
    import os
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    import subprocess
    res = subprocess.run([exe, *SCENARIOS], capture_output=True, text=True, timeout=900, env=env)
    assert res.returncode == 0, res.stdout[-4000:] + res.stderr[-4000:]
    for s in SCENARIOS:
        assert f"{s}: ok" in res.stdout, res.stdout
