"""The ensemble runner (`python -m paper_2304_09180_amd.ensemble`) on a few members,
eager and replayed as graphs: one JSON line, every member converged, the same
iteration counts either way."""
import json

import pytest

pytestmark = pytest.mark.gpu


def run(capsys, *extra):
    from paper_2304_09180_amd import ensemble
    assert ensemble.main(["--members", "4", "--steps", "3", *extra]) == 0
    return json.loads(capsys.readouterr().out.strip().splitlines()[-1])


def test_ensemble_runner_eager_and_graph(capsys):
    eager = run(capsys)
    graph = run(capsys, "--graph")
    print(eager, graph, flush=True)
    for r in (eager, graph):
        assert r["members"] == 4 and r["status"] == ["OK"] and r["ms_per_step"] > 0
        assert r["cell_timesteps_per_s"] == pytest.approx(r["cells"] * 1e3 / r["ms_per_step"], rel=1e-3)   # ms rounded
    assert graph["graph"] and not eager["graph"]
    assert eager["solver"] == graph["solver"]
