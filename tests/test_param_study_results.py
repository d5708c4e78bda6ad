"""The committed parameter-influence study of Sec. 3.1.2 at the paper's grid
(dx = 0.02, dt = 1e-8, t = 0.22; written by `python -m
paper_2101_03055_amd.param_study --out ...` on the GPU) satisfies the trends
the section states and the exact invariants (same checks as the GPU test)."""
import json
import os

from tests.test_gpu_param_study import check

HERE = os.path.dirname(os.path.abspath(__file__))
DATA = os.path.join(os.path.dirname(HERE), "paper_2101_03055_amd", "data", "chemotaxis_parameter_study.json")


def test_committed_study_satisfies_the_stated_trends():
    with open(DATA) as fh:
        out = json.load(fh)
    assert out["dx"] == 0.02 and out["dt"] == 1e-8 and out["t"] == 0.22 and len(out["cases"]) == 14
    check(out)
