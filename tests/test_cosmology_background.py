"""The expansion history behind the device-resident comoving runs: for a
flat matter + Lambda background, a(t) = (om/ol)^(1/3) sinh(3/2 sqrt(ol) H0 t)^(2/3)
(ol > 0) and a(t) = (3/2 H0 t)^(2/3) (Einstein-de Sitter) solve the
Friedmann equation (adot/a)^2 = H0^2 (om/a^3 + ol) with a(0) = 0.  Pinned
against a direct numerical integration of that equation; a planted wrong
exponent fails.  The GPU tests compare the device's a(t) and H with this
reference."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp


def flat_lcdm(t, H0, om, ol, expo=2.0 / 3.0):
    """a(t) and H(a(t)), in the device code's order of operations."""
    if ol > 0.0:
        a = np.cbrt(om / ol) * np.power(np.sinh(1.5 * np.sqrt(ol) * H0 * t), expo)
    else:
        a = np.power(1.5 * H0 * t, expo)
    return a, H0 * np.sqrt(om / (a * a * a) + ol)


def integrated(t_eval, H0, om, ol, t0=1e-6):
    a0 = flat_lcdm(t0, H0, om, ol)[0]  # a ~ t^(2/3) at early times, either way
    sol = solve_ivp(lambda t, a: a * H0 * np.sqrt(om / a ** 3 + ol), (t0, t_eval[-1]), [a0], t_eval=t_eval,
                    rtol=1e-12, atol=0.0, method="DOP853")
    return sol.y[0]


@pytest.mark.parametrize("H0,om,ol", [(2.0 / 3.0, 1.0, 0.0), (2.0 / 3.0, 0.3, 0.7), (1.0, 0.05, 0.95)])
def test_closed_form_solves_the_friedmann_equation(H0, om, ol):
    t = np.linspace(0.2, 3.0, 8)
    a_ode = integrated(t, H0, om, ol)
    a, H = flat_lcdm(t, H0, om, ol)
    assert np.max(np.abs(a - a_ode) / a_ode) < 1e-9
    # H is adot / a of the closed form (central differences)
    h = 1e-6
    ap, am = flat_lcdm(t + h, H0, om, ol)[0], flat_lcdm(t - h, H0, om, ol)[0]
    assert np.max(np.abs((ap - am) / (2 * h) / a - H) / H) < 1e-8
    # a planted wrong exponent is off the solution
    bad = flat_lcdm(t, H0, om, ol, expo=0.5)[0]
    assert np.max(np.abs(bad - a_ode) / a_ode) > 1e-2
