"""Pins of the oracle's design chain (§3.3): Heaviside projection, p-norm
objective of the element-averaged temperature, volume constraint, and the
full adjoint gradient through filter and projection."""
import numpy as np
import pytest

from oracle.assemble import Material
from oracle.design import (heaviside, heaviside_deriv, pnorm, pnorm_chain, volume,
                           element_average)
from oracle.grid import Grid

MAT = Material()
PATCH = [(0, 0.5, 0.2)]


def test_heaviside_closed_forms():
    for beta in (1.0, 8.0, 32.0):
        assert heaviside(0.0, beta, 0.5) == pytest.approx(0.0, abs=1e-15)
        assert heaviside(1.0, beta, 0.5) == pytest.approx(1.0, abs=1e-15)
        assert heaviside(0.5, beta, 0.5) == pytest.approx(0.5, abs=1e-15)
    # eta != 0.5: H(eta) = tanh(b eta) / (tanh(b eta) + tanh(b (1 - eta)))
    b, e = 6.0, 0.3
    assert heaviside(e, b, e) == pytest.approx(np.tanh(b * e) / (np.tanh(b * e) + np.tanh(b * (1 - e))))
    # beta = 32: close to a step away from the threshold
    assert heaviside(0.4, 32.0, 0.5) < 2e-3 and heaviside(0.6, 32.0, 0.5) > 1 - 2e-3


def test_heaviside_derivative_matches_central_difference():
    x = np.linspace(0.0, 1.0, 41)
    for beta, eta in [(1.0, 0.5), (32.0, 0.5), (6.0, 0.3)]:
        h = 1e-6
        fd = (heaviside(x + h, beta, eta) - heaviside(x - h, beta, eta)) / (2 * h)
        assert np.max(np.abs(fd - heaviside_deriv(x, beta, eta))) <= 1e-7 * max(1.0, beta)


def test_pnorm_uniform_field_and_euler_identity():
    g = Grid(3, 4, 5, 0.3, 0.2)
    c = 0.7
    phi, grad = pnorm(g, np.full(g.n_nodes, c), 20.0)
    assert phi == pytest.approx(g.n_elems ** (1 / 20.0) * c, rel=1e-14)
    # phi is positively homogeneous of degree 1: s . grad phi = phi
    s = np.random.default_rng(1).uniform(0.1, 1.0, g.n_nodes)
    phi, grad = pnorm(g, s, 20.0)
    assert np.dot(s, grad) == pytest.approx(phi, rel=1e-13)
    # element average of a nodal constant is that constant
    assert np.allclose(element_average(g, np.full(g.n_nodes, 2.5)), 2.5)


def test_pnorm_gradient_matches_central_difference():
    g = Grid(3, 3, 2, 0.3, 0.5)
    s = np.random.default_rng(2).uniform(0.2, 1.0, g.n_nodes)
    _, grad = pnorm(g, s, 8.0)
    for a in (0, 5, 17, g.n_nodes - 1):
        h = 1e-6
        sp_, sm_ = s.copy(), s.copy()
        sp_[a] += h
        sm_[a] -= h
        fd = (pnorm(g, sp_, 8.0)[0] - pnorm(g, sm_, 8.0)[0]) / (2 * h)
        assert fd == pytest.approx(grad[a], rel=1e-7, abs=1e-12)


def test_volume_closed_form():
    g = Grid(4, 4, 6, 0.25, 1 / 6)
    chi, d = volume(g, np.full((4, 4), 0.15), 0.3)       # time-constant field
    assert chi == pytest.approx(0.15 / 0.3 - 1.0, rel=1e-14)
    assert d.sum() == pytest.approx(1 / 0.3, rel=1e-14)
    chi, _ = volume(g, np.full((6, 4, 4), 0.6), 0.3)      # time-varying field
    assert chi == pytest.approx(1.0, rel=1e-14)


@pytest.mark.parametrize("tv,filt,beta", [(True, 1.5, 4.0), (False, 1.5, 8.0), (True, None, None)])
def test_pnorm_chain_gradient_matches_central_difference(tv, filt, beta):
    g = Grid(4, 4, 3, 0.25, 1 / 3)
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.1, 0.9, (3, 4, 4) if tv else (4, 4))
    kw = dict(P=8.0, r_elems=filt, beta=beta, vf=0.3)
    o = pnorm_chain(g, MAT, rho, PATCH, **kw)
    for e in (0, 7, rho.size - 1):
        h = 1e-6
        rp, rm = rho.copy().ravel(), rho.copy().ravel()
        rp[e] += h
        rm[e] -= h
        fp = pnorm_chain(g, MAT, rp.reshape(rho.shape), PATCH, with_grad=False, **kw)
        fm = pnorm_chain(g, MAT, rm.reshape(rho.shape), PATCH, with_grad=False, **kw)
        # FD rounding: ~1e-16 |phi| / h = 1e-10 absolute
        assert (fp["phi"] - fm["phi"]) / (2 * h) == pytest.approx(o["grad"].ravel()[e], rel=1e-6, abs=1e-9)
        assert (fp["chi"] - fm["chi"]) / (2 * h) == pytest.approx(o["dchi"].ravel()[e], rel=1e-6, abs=1e-9)
