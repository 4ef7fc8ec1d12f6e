"""Pin the closed-form linear theory to the constants the paper prints."""
import json
import math
import os

import pytest

from oracle import closed_forms as CF


@pytest.fixture(scope="module")
def consts(golden_dir):
    with open(os.path.join(golden_dir, "paper_constants.json")) as f:
        return json.load(f)


def _agree(val, ref, digits):
    # printed with `digits` significant digits: agree to half a unit in the last place
    scale = 10.0 ** (math.floor(math.log10(abs(ref))) - digits + 1)
    return abs(val - ref) <= 0.5 * scale + 1e-15


def test_gamma0(consts):
    c = consts["gamma0"]
    assert _agree(CF.gamma0(c["v0"]), c["value"], c["digits"])


def test_two_stream_constants(consts):
    c = consts["tsi"]
    assert _agree(CF.chi(c["k"], c["dx"]) ** 2, c["chi2_sq"], c["chi2_sq_digits"])
    assert _agree(CF.gamma_two_stream(c["k"], c["v0"], c["dx"]), c["Gamma_TS"], c["Gamma_TS_digits"])


def test_weibel_constants(consts):
    c = consts["weibel"]
    A, Cc = CF.weibel_coeffs(c["k"], c["v0"], c["dx"])
    assert _agree(CF.chi(c["k"], c["dx"]) ** 2, c["chi2_sq"], c["digits"])
    assert _agree(A, c["A"], c["digits"])
    assert _agree(Cc, c["C"], c["digits"])
    assert _agree(CF.gamma_weibel(c["k"], c["v0"], c["dx"]), c["Gamma_W"], c["digits"])


def test_two_stream_root_solves_dispersion():
    # the closed-form root makes the dispersion function vanish at w = i Gamma
    k, v0, dx = 0.5, CF.v_of_u(1.0), 4 * math.pi / 64
    G = CF.gamma_two_stream(k, v0, dx)
    g0 = CF.gamma0(v0)
    w = 1j * G
    f = 1 - CF.omega_p_h2(k, dx) / (2 * g0 ** 3) * ((w - k * v0) ** -2 + (w + k * v0) ** -2)
    assert abs(f) < 1e-12
    # cutoff: a stable long-wavelength-complement mode returns zero
    assert CF.gamma_two_stream(1.0, v0, dx) == 0.0


def test_weibel_root_solves_dispersion():
    k, v0, dx = 1.3, CF.v_of_u(0.5), 0.2
    G = CF.gamma_weibel(k, v0, dx)
    g0 = CF.gamma0(v0)
    w2 = -G * G
    wp2 = CF.omega_p_h2(k, dx)
    f = w2 * w2 - (k * k + wp2 / g0 ** 3) * w2 - k * k * wp2 * v0 * v0 / g0
    assert abs(f) < 1e-13


def test_outer_vector_sizes(consts):
    c = consts["outer_vector"]
    ng = c["mesh"] ** 3
    assert 3 * ng == c["outer_components"]
    assert 3 * ng * 2 * c["tsi_pairs_per_cell"] == c["tsi_velocity_components"]
    assert 3 * ng * 2 * c["wbi_pairs_per_cell"] == c["wbi_velocity_components"]
