"""First-emission pins of the splitting kernels the other Sudakov pins leave
out, in every form of the competition (max-veto, retained trials,
generate-select, veto-max):

* FF g -> g g and g -> q qbar, and q -> q g with a gluon spectator, on an
  e+e- -> q qbar g configuration (appendix B.2);
* the initial-state gluon families C (g <- g) and D (g <- q) at an IF and an
  II end, and FI q -> q g with an incoming gluon spectator, on two NLO
  q g -> Z q events (one where the FI end weighs most, one where family D
  does; appendices B.3-B.5);
* the heavy-quark measure dt/(t - m^2) with the factor (t - m^2)/t of appendix
  A.2, on c cbar -> Z and b bbar -> Z Born events.

The integrands are written independently in tests/sudakov_pins.py."""
import pytest

from tests import sudakov_pins as P

FORM = pytest.mark.parametrize("form", P.FORMS)


@pytest.mark.slow
@FORM
def test_ff_gluon_kernels_qqg(oracles, form):
    P.check_ff_qqg(oracles["ee"], form)


@pytest.mark.slow
@FORM
@pytest.mark.parametrize("pick", ["fi", "is"])
def test_is_gluon_families_and_fi_quark(oracles, cfgs, form, pick):
    P.check_h_gluon(oracles["nlo"], P.PDF(cfgs["nlo"]["pdf"]), form, pick)


@pytest.mark.slow
@FORM
@pytest.mark.parametrize("flavour", [4, 5], ids=["charm", "bottom"])
def test_heavy_quark_measure(oracles, cfgs, form, flavour):
    P.check_heavy_born(oracles["lo"], P.PDF(cfgs["lo"]["pdf"]), form, flavour)
