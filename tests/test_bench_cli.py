"""bench.py refuses, before it touches torch or a GPU, the runs it does not
measure: more than one GPU, dense mixing or another model shape outside the
13,824-atom evaluation, the training step at shapes whose double backward
is not built, and dense mixing combined with another model shape."""

import pytest

import bench


@pytest.mark.parametrize("argv", [
    ["--gpus", "2"],
    ["--gpus", "8", "--config", "B"],
    ["--config", "D", "--model", "fm512"],
    ["--config", "E", "--mixing", "dense"],
    ["--config", "C", "--model", "lmax3"],
    ["--config", "C", "--mixing", "dense"],
    ["--config", "C", "--model", "fm512", "--mixing", "dense"],
    ["--config", "B", "--model", "fm512", "--mixing", "dense"],
])
def test_refused_runs_exit_with_status_2(argv, capsys):
    assert bench.main(argv) == 2
    err = capsys.readouterr().err
    assert "not supported" in err or "measured on" in err


def test_unknown_choices_are_argument_errors():
    with pytest.raises(SystemExit):
        bench.main(["--model", "fm1024"])
    with pytest.raises(SystemExit):
        bench.main(["--mixing", "full"])
