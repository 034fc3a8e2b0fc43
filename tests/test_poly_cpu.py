"""Host side of the Chebyshev time step: the library's Bessel weights
(Miller's backward recurrence) against scipy's J_k through the oracle, and
against identities that hold for the exact functions."""
import numpy as np
import pytest

import oracle

mpk = pytest.importorskip("paper_2405_12525_amd")


@pytest.mark.parametrize("dt", [1e-6, 0.01, 0.5, 1.0, 2.5, 7.3, 20.0, 55.5, -3.0])
@pytest.mark.parametrize("M", [1, 4, 30, 200])
def test_weights_match_oracle(dt, M):
    a, b, g, wa, wb = mpk.cheb_time_coefficients(M, dt)
    oa, ob, og, owa, owb = oracle.cheb_time_coefficients(M, dt)
    assert np.array_equal(a, oa) and np.array_equal(b, ob) and np.array_equal(g, og)
    # (-i)^k: even weights real, odd weights imaginary, the other part exactly 0
    assert not wa[1::2].any() and not wb[0::2].any()
    ref = np.abs(owa) + np.abs(owb)
    d = np.abs(wa - owa) + np.abs(wb - owb)
    assert d.max() <= 1e-13 * ref.max()
    # relative accuracy in the decaying tail as well (k > |dt|, not underflowed)
    k = np.arange(M + 1)
    tail = (k > abs(dt) + 2) & (ref > 1e-280)
    if tail.any():
        assert (d[tail] / ref[tail]).max() <= 1e-12


@pytest.mark.parametrize("dt", [0.3, 4.0, 37.0, 400.0])
def test_weights_satisfy_bessel_identities(dt):
    # J_0 + 2 sum J_2k = 1 and J_0^2 + 2 sum J_k^2 = 1, with M past the decay
    M = int(dt) + 80
    _, _, _, wa, wb = mpk.cheb_time_coefficients(M, dt)
    Jk = np.empty(M + 1)
    Jk[0] = wa[0]
    for k in range(1, M + 1):
        re, im = ((1, 0), (0, -1), (-1, 0), (0, 1))[k % 4]   # (-i)^k
        Jk[k] = wa[k] / (2.0 * re) if re else wb[k] / (2.0 * im)
    assert abs(Jk[0] + 2.0 * Jk[2::2].sum() - 1.0) <= 1e-14 * max(1.0, dt)
    assert abs(Jk[0] ** 2 + 2.0 * (Jk[1:] ** 2).sum() - 1.0) <= 1e-14 * max(1.0, dt)


def test_argument_errors():
    with pytest.raises(mpk.MPKError):
        mpk.cheb_time_coefficients(0, 1.0)
    with pytest.raises(mpk.MPKError):
        mpk.cheb_time_coefficients(5, float("nan"))
    # dt = 0: the identity step
    _, _, _, wa, wb = mpk.cheb_time_coefficients(6, 0.0)
    assert wa[0] == 1.0 and not wa[1:].any() and not wb.any()
