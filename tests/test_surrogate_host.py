"""Host logic of the warm start (no GPU): rebuilding c+- from a predicted
charge density (Boltzmann product c+ c- = A^2, both contents equal to the
gap volume), including predictions the ions cannot carry."""
import numpy as np

from paper_1701_02005_amd.surrogate import ions_from_charge


def _grid(n=64):
    yn = np.tanh(1.5 * np.linspace(-1, 1, n + 1)) / np.tanh(1.5)
    return np.diff(yn), 0.5 * (yn[1:] + yn[:-1])


def test_feasible_charge_is_kept():
    dn, yc = _grid()
    rho = 3.0 * np.sinh(4 * yc) / np.sinh(4.0)
    rho0 = rho - np.sum(rho * dn) / np.sum(dn)
    info = {}
    cp, cm, A = ions_from_charge(rho, dn, info)
    assert info["scale"] == 1.0
    np.testing.assert_allclose(cp - cm, rho0, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(cp * cm, A * A, rtol=1e-12)
    assert abs(np.sum(cp * dn) - 2.0) < 1e-10 and abs(np.sum(cm * dn) - 2.0) < 1e-10


def test_strong_layer_minority_species_without_cancellation():
    """rho up to 400 with A ~ 1e-3: the minority concentration (~2.5e-9) is
    still exact to the Boltzmann product."""
    dn, yc = _grid(128)
    rho = 400.0 * np.sign(yc) * np.exp(-(1 - np.abs(yc)) / 0.01)
    cp, cm, A = ions_from_charge(rho, dn)
    assert np.all(cp > 0) and np.all(cm > 0)
    np.testing.assert_allclose(cp * cm, A * A, rtol=1e-12)


def test_infeasible_charge_is_scaled_to_the_content():
    """A predicted |rho| integrating to more than the ions' total content has
    no Boltzmann reconstruction with A > 0: it is scaled to 99% of it, and
    both species stay positive with the right contents."""
    dn, yc = _grid()
    rho = 5.0 * np.sign(yc) * np.ones_like(yc)  # integral of |rho| = 10 > 4
    info = {}
    cp, cm, A = ions_from_charge(rho, dn, info)
    assert 0 < info["scale"] < 1 and A > 0
    assert np.all(cp > 0) and np.all(cm > 0)
    np.testing.assert_allclose(np.sum(np.abs(cp - cm) * dn), 0.99 * 4.0, rtol=1e-12)
    assert abs(np.sum(cp * dn) - 2.0) < 1e-10 and abs(np.sum(cm * dn) - 2.0) < 1e-10
