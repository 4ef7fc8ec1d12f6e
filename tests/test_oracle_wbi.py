"""The oracle against the paper's Weibel/filamentation production runs (CPU).

The growing eigenmode varies only in y, and the loading is quiet (pairs at the cells' y
centres, uniform in x and z), so a mesh reduced to 4 x 32 x 4 with one pair per cell
follows the same y dynamics as the paper's 32^3 run with 25 pairs per cell.  Its fitted
growth rates must equal the two rates the paper prints, to all nine printed digits.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from oracle import closed_forms as CF
from paper_2609_36383_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "wbi_runs.json")))


def _run(run, **cfg_over):
    g = GOLD[run]
    w = W.spec("wbi", n=(4, 32, 4), ppc=2, dt=g["dt"], eig_gamma=CF.gamma_weibel(1.0, 0.9, math.pi / 16))
    x, u, q = W.particles(w)
    A0, U0 = W.potentials(w)
    sim = O.OracleSim(O.config_from_dict(W.config_dict(w), gl_order=8, **cfg_over))
    sim.load_particles(x, u, q)
    sim.load_potentials(A0, U0)
    sim.initialize()
    ts, amps, diags, outer = [0.0], [sim.mode_amplitude("B", 2, (0, 1, 0))], [], []
    win = GOLD["fit_window"]
    for _ in range(int(round(win["t1"] / g["dt"]))):
        _, rep = sim.step()
        outer.append(rep["outer_iters"])
        diags.append(sim.diagnostics())
        ts.append(diags[-1]["t"])
        amps.append(sim.mode_amplitude("B", 2, (0, 1, 0)))
    return w, ts, amps, diags, outer


@pytest.mark.parametrize("run", ["WBI-0.2", "WBI-0.04"])
def test_wbi_fitted_growth_rate_equals_printed(run):
    w, ts, amps, diags, _ = _run(run)
    assert abs(amps[0] - w["B0"] / 2) <= 1e-15  # |B_z-hat(k_y)| / N_g of B0 sin(k_y y)
    win = GOLD["fit_window"]
    fit = CF.fit_growth(ts, amps, win["t0"], win["t1"])
    # the printed rate has nine significant digits: the fit must round to it
    assert abs(fit - GOLD[run]["fitted_rate"]) <= 5e-10, fit
    G = CF.gamma_weibel(1.0, 0.9, math.pi / 16)
    assert abs(abs(fit / G - 1) - GOLD[run]["fitted_rate_rel_err"]) < 0.01e-3
    assert max(abs(d["energy_rel"]) for d in diags) < 1e-13
    assert max(d["gauss_rms"] for d in diags) < 1e-18
    assert max(d["lorenz_rms"] for d in diags) < 1e-18


def test_wbi_anderson_outer_counts_within_printed_maximum():
    """With the paper's Anderson settings (beta = 0.5) the outer counts of the first steps
    of WBI-0.2 stay within the printed maximum, and the fit is unchanged."""
    w, ts, amps, diags, outer = _run("WBI-0.2", outer_scheme=1, beta=0.5)
    assert max(outer) <= GOLD["WBI-0.2"]["outer_max"]
    assert min(outer) >= 5
    fit = CF.fit_growth(ts, amps, 0.0, 1.6)
    assert abs(fit - GOLD["WBI-0.2"]["fitted_rate"]) <= 5e-10
