"""The closed-form central differences that the device source of the cut
torus uses for the second-order compensation (the differences over rho at
a +- h of 1/rho^2, 1/(rho q) and 1/q^2, q = R + rho cos th) against the
difference quotients themselves, in 50-digit arithmetic."""
import mpmath as mp
import pytest


@pytest.mark.parametrize("th", [0.1, 1.3, 2.9, 4.0, 3.14159])
@pytest.mark.parametrize("R,a,h", [(1.0, 0.45, 1e-2), (1.0, 0.45, 1e-3), (2.5, 0.7, 0.05)])
def test_written_out_differences_equal_the_quotients(th, R, a, h):
    mp.mp.dps = 50
    R, a, h = mp.mpf(R), mp.mpf(a), mp.mpf(h)
    c, s = mp.cos(th), mp.sin(th)
    utt, ut, uss = mp.mpf("1.7"), mp.mpf("-0.6"), mp.mpf("2.3")

    def L(rho):
        q = R + rho * c
        return utt / rho ** 2 - s * ut / (rho * q) + uss / q ** 2
    m1 = -(L(a + h) - L(a - h)) / (2 * h)
    m2 = -(L(a + h) - 2 * L(a) + L(a - h)) / h ** 2
    q0 = R + a * c
    e, g = a * a - h * h, q0 * q0 - h * h * c * c
    d1_r2, d2_r2 = -2 * a / e ** 2, (6 * a * a - 2 * h * h) / (a * a * e ** 2)
    d1_q2 = -2 * q0 * c / g ** 2
    d2_q2 = (6 * q0 * q0 - 2 * h * h * c * c) * c * c / (q0 * q0 * g ** 2)
    d1_rq = (-1 / e + c * c / g) / R
    d2_rq = (2 / (a * e) - 2 * c ** 3 / (q0 * g)) / R
    B = -s * ut
    assert abs(m1 + (utt * d1_r2 + B * d1_rq + uss * d1_q2)) < mp.mpf(10) ** -40 * (1 + abs(m1))
    assert abs(m2 + (utt * d2_r2 + B * d2_rq + uss * d2_q2)) < mp.mpf(10) ** -38 * (1 + abs(m2))
