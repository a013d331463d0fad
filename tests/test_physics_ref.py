"""Pins of the independent physics references against textbook values."""
import json
import os

import pytest

import physics_ref as P

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "textbook_constants.json")))


def test_sod_star_state_matches_textbook():
    g = GOLD["sod_gamma_1p4"]
    WL, WR = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    ps, us = P.exact_star(WL, WR, 1.4)
    assert ps == pytest.approx(g["p_star"], abs=g["tol"])
    assert us == pytest.approx(g["u_star"], abs=g["tol"])
    rl = P.exact_sample(WL, WR, 1.4, us - 1e-9)[0]
    rr = P.exact_sample(WL, WR, 1.4, us + 1e-9)[0]
    assert rl == pytest.approx(g["rho_star_left"], abs=g["tol"])
    assert rr == pytest.approx(g["rho_star_right"], abs=g["tol"])
    assert P.shock_speed_right(WR, ps, 1.4) == pytest.approx(g["shock_speed"], abs=g["tol"])


def test_exact_riemann_limits():
    # identical states: no waves; far left/right of the fan: initial states
    W = (0.7, 0.3, 2.0)
    ps, us = P.exact_star(W, W, 1.4)
    assert ps == pytest.approx(2.0, rel=1e-12) and us == pytest.approx(0.3, rel=1e-12)
    WL, WR = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    assert P.exact_sample(WL, WR, 1.4, -10.0) == (1.0, 0.0, 1.0)
    assert P.exact_sample(WL, WR, 1.4, 10.0) == (0.125, 0.0, 0.1)


def test_sedov_constants_match_textbook():
    g = GOLD["sedov_spherical"]
    assert P.sedov_xi0(1.4) == pytest.approx(g["xi0_gamma_1p4"], abs=g["tol"])
    assert P.sedov_xi0(5.0 / 3.0) == pytest.approx(g["xi0_gamma_5over3"], abs=g["tol"])
