"""Influence of alpha, beta and delta on the chemotaxis-fluid system
(Sec. 3.1.2): the fourteen cases of the section, batched, FP64, to t = 0.22.
The paper's figures are not in the text, so the run is checked against the
trends its text states and against exact invariants.  The run uses the
paper's dx = 0.02 (50 rows) and dt = 1e-8: 22 million steps of all fourteen
cases in one batch, ~150 s, with a progress line per million steps.  (At
twice the spacing, dx = 0.04, the beta = 40 oxygen profile crosses the
beta = 20 one in the upper half: the steep layer under the surface is not
resolved there.)  The committed study,
paper_2101_03055_amd/data/chemotaxis_parameter_study.json, is this run's
output and passes the same checks (tests/test_param_study_results.py)."""
import numpy as np
import pytest

from paper_2101_03055_amd import param_study as PS

pytestmark = pytest.mark.gpu


def check(out):
    for c in out["cases"]:
        # bacteria: no-flux walls, no bacteria source -> the total is conserved
        assert abs(c["n_total_rel_change"]) < 1e-11, c["label"]
        # data and lattice are mirror symmetric about x = 0
        assert c["mirror_asymmetry"] < 1e-9, c["label"]
    s = PS.statements(out)
    inc = lambda v: bool(np.all(np.diff(v) > 0))
    dec = lambda v: bool(np.all(np.diff(v) < 0))
    # alpha up: bacteria gather near the surface, leave the lower part, consume less oxygen there
    assert inc(s["alpha_n_top"]) and dec(s["alpha_n_lower_half"]) and inc(s["alpha_c_lower_half"])
    # beta up: oxygen lower at every height, more bacteria swim up to the surface
    assert np.all(np.diff(np.asarray(s["beta_c_profiles"]), axis=0) < 0)
    assert inc(s["beta_n_surface"])
    # delta up: oxygen fills the domain, bacteria stay in the lower part, fewer swim up
    assert inc(s["delta_c_mean"]) and inc(s["delta_n_lower_half"]) and dec(s["delta_n_top"])
    # base case: below the cut-off level c* = 0.3 the bacteria increase towards the bottom
    assert s["base_c_bottom"] < 0.3
    assert dec(s["base_n_lower"])


def test_parameter_influence_trends():
    out = PS.run()
    for c in out["cases"]:
        print({k: round(c[k], 4) for k in ("n_top", "n_surface", "n_lower_half", "c_mean", "c_lower_half")},
              c["label"], flush=True)
    check(out)
