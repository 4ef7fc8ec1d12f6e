"""The oracle against the paper's two-stream production runs (CPU).

The growing mode depends only on x and the loading is quiet (pairs evenly along x within a
cell, cell centre across), so the run reduces exactly to 1D: 32 cells on [-4 pi, 4 pi]
with the paper's 10 pairs per cell.  Its fitted growth rates must equal the two rates the
paper prints, to all seven printed digits.
"""
import json
import math
import os

import pytest

import oracle as O
from oracle import closed_forms as CF
from paper_2609_36383_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tsi_runs.json")))
GTS = CF.gamma_two_stream(0.25, 0.9, math.pi / 4)


@pytest.mark.parametrize("run", ["TSI-0.1", "TSI-0.3"])
def test_tsi_fitted_growth_rate_equals_printed(run):
    g = GOLD[run]
    w = W.spec("tsi", dim=1, n=(32,), lo=(-4.0 * math.pi,), length=(8.0 * math.pi,), dt=g["dt"], eig_gamma=GTS)
    x, u, q = W.particles(w)
    sim = O.OracleSim(O.config_from_dict(W.config_dict(w), gl_order=8))
    sim.load_particles(x, u, q)
    sim.initialize()
    # grid charge density alpha cos(k x') gives |E_x-hat(k)| / N_g = alpha / (2 k)
    a0 = sim.mode_amplitude("E", 0, (1, 0, 0))
    assert abs(a0 - w["alpha"] / (2 * 0.25)) <= 1e-6 * a0
    win = GOLD["fit_window"]
    ts, amps, drift = [0.0], [a0], 0.0
    for _ in range(int(math.ceil(win["t1"] / g["dt"] - 1e-9))):
        sim.step()
        d = sim.diagnostics()
        drift = max(drift, abs(d["energy_rel"]))
        ts.append(d["t"])
        amps.append(sim.mode_amplitude("E", 0, (1, 0, 0)))
    fit = CF.fit_growth(ts, amps, win["t0"], win["t1"])
    # the printed rate has seven significant digits: the fit must round to it
    assert abs(fit - g["fitted_rate"]) <= 5e-9, fit
    assert abs(abs(fit / GTS - 1) - g["fitted_rate_rel_err"]) < 0.01e-3
    assert drift < 1e-12


def test_tsi_0p3_anderson_outer_counts_match_printed():
    """TSI-0.3 through T = 60 with the paper's Anderson settings: the outer iterations as
    the paper's algorithm counts them (accepted updates plus one) average within 5% of
    the printed mean, and their maximum equals the printed one."""
    g = GOLD["TSI-0.3"]
    w = W.spec("tsi", dim=1, n=(32,), lo=(-4.0 * math.pi,), length=(8.0 * math.pi,), dt=g["dt"], eig_gamma=GTS)
    x, u, q = W.particles(w)
    sim = O.OracleSim(O.config_from_dict(W.config_dict(w), gl_order=8, outer_scheme=1, beta=0.5))
    sim.load_particles(x, u, q)
    sim.initialize()
    counts = []
    for _ in range(int(round(g["end_time"] / g["dt"]))):
        _, rep = sim.step()
        counts.append(rep["outer_updates"] + 1)
    mean = sum(counts) / len(counts)
    assert abs(mean / g["outer_mean"] - 1) < 0.05, mean
    assert max(counts) == g["outer_max"]
    # the amplitude at T = 60 (nonlinear trapping) equals the printed one
    assert abs(sim.mode_amplitude("E", 0, (1, 0, 0)) - g["amp_T60"]) <= 5e-8
