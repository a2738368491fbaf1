"""Host logic of the update-scheme decision (Sec. 4.4 final update scheme,
Sec. 4.5 adaptive maximum level), the function mls2mc_run uses: no device
work, so it runs on the CPU."""
import pytest

import paper_1709_09763_amd as P

ITU, LU, DONE, NEED = P.DECIDE_ITU, P.DECIDE_LU, P.DECIDE_DONE, P.DECIDE_NEED_CV
MLS, MLB = P.SCHEME_MLS2MC, P.SCHEME_MLB


@pytest.mark.parametrize("beta,l,lmax,prev,scheme,cv,tau_lu,tau_min,want", [
    (1.0, 6, 6, 0, MLS, -1, 1.0, 0.0, DONE),       # finished
    (1.0, 6, 6, 0, MLS, 0.5, 1.0, 0.01, DONE),
    (1.0, 4, 6, 0, MLS, -1, 1.0, 0.0, LU),         # beta = 1: bridge the remaining levels
    (1.0, 4, 6, 1, MLS, -1, 1.0, 0.0, LU),
    (1.0, 4, 6, 0, MLS, -1, 1.0, 0.001, NEED),     # u': the look-ahead decides
    (1.0, 4, 6, 0, MLS, 0.0005, 1.0, 0.001, DONE),
    (1.0, 4, 6, 0, MLS, 0.002, 1.0, 0.001, LU),
    (1.0, 4, 6, 0, MLB, -1, 1.0, 0.0, LU),         # multilevel bridging at beta = 1
    (0.3, 4, 6, 1, MLS, -1, 1.0, 0.0, ITU),        # after a level update (or first): tempering
    (0.0, 3, 6, 1, MLS, -1, 1.0, 0.0, ITU),
    (0.3, 6, 6, 0, MLS, -1, 1.0, 0.0, ITU),        # finest level: tempering
    (0.3, 4, 6, 0, MLB, -1, 1.0, 0.0, ITU),        # multilevel bridging below beta = 1
    (0.3, 4, 6, 0, MLS, -1, 1.0, 0.0, NEED),       # otherwise cv^LU decides
    (0.3, 4, 6, 0, MLS, 0.99, 1.0, 0.0, ITU),
    (0.3, 4, 6, 0, MLS, 1.0, 1.0, 0.0, LU),
    (0.3, 4, 6, 0, MLS, 3.0, 1.0, 0.0, LU),
    (0.3, 4, 6, 0, MLS, 3.0, 1.0, 0.5, LU),        # tau_min applies at beta = 1 only
])
def test_decision_table(beta, l, lmax, prev, scheme, cv, tau_lu, tau_min, want):
    assert P.mls2mc_decide(beta, l, lmax, prev, scheme, cv, tau_lu, tau_min) == want


@pytest.mark.parametrize("beta,l,lmax,scheme", [(1.2, 3, 6, MLS), (-0.1, 3, 6, MLS), (0.5, 7, 6, MLS),
                                                (0.5, 3, 6, 9)])
def test_bad_arguments(beta, l, lmax, scheme):
    assert P.mls2mc_decide(beta, l, lmax, 0, scheme, 0.5, 1.0, 0.0) == -1
