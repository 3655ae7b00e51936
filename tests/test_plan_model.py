"""CPU checks of the launch plan: host builds of the library's layout code."""
import model_build


def test_segment_test_queue_holds_every_append():
    """Every accepted segment-test tile shape (64 x mark_words pixels by mark_rows):
    each wave's pre-test queue segment holds the most pixels the wave can append."""
    exe = model_build.build("lds_capacity", ["lds_capacity.cpp"])
    res = model_build.run(exe)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip() == "ok 244"
