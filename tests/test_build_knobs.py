"""The build's tile knobs: tuned.json (written by the autotuner) holds a
point of the tuner's grid, the build passes every knob explicitly, and the
build id that keys the stored counter readings follows the knobs."""
import json

from paper_2503_19925_amd import build, tune


def test_tuned_knobs_are_a_grid_point():
    rec = json.load(open(build.TUNED))
    knobs = build.tuned_knobs()
    assert set(knobs) == set(build.KNOBS) == set(tune.GRID)
    for k, v in knobs.items():
        assert v in tune.GRID[k]
        assert rec["knobs"][k] == v
    # the record names the chosen variant among the timed ones
    assert tune.tag(knobs) in [row[0] for row in rec["table"]]


def test_defines_and_build_id_follow_the_knobs():
    base = build.tuned_knobs()
    assert build.defines(base) == ["-D%s=%d" % (k, base[k]) for k in sorted(base)]
    other = dict(base, EXACT_VIEW_BATCH=2 if base["EXACT_VIEW_BATCH"] != 2 else 4)
    assert build.build_id(other) != build.build_id(base)
    assert build.build_id(base) == build.build_id()


def test_tuner_grid_holds_the_defaults():
    assert tune.tag(tune.DEFAULT) in {tune.tag(k) for k in tune.variants()}
    assert len(list(tune.variants())) == 36
