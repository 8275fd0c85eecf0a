"""Pins of the oracle's 1-D operators against closed forms and independent characterisations."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle.basis import Ops1D, gauss_points, interpolation_1d, projection_1d


@pytest.mark.parametrize("P", range(0, 7))
def test_gauss_rule_exact(P):
    x, w = gauss_points(P)
    for k in range(2 * P + 2):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14


@pytest.mark.parametrize("P", range(0, 7))
def test_derivative_and_extrapolation_exact_on_polynomials(P):
    o = Ops1D(P)
    for m in range(P + 1):
        f = o.x ** m
        df = m * o.x ** (m - 1) if m > 0 else 0.0 * o.x
        assert np.max(np.abs(o.D @ f - df)) < 1e-12
        assert abs(o.lm @ f - (-1.0) ** m) < 1e-13
        assert abs(o.lp @ f - 1.0) < 1e-13


def test_radau_closed_forms():
    # g_R = (L_{P+1} + L_P)/2 written out: P=0: (x+1)/2; P=1: (3x^2+2x-1)/4; P=2: (5x^3+3x^2-3x-1)/4
    x1 = gauss_points(1)[0]
    assert np.allclose(Ops1D(1).gR, (3 * x1 + 1) / 2, atol=1e-15)
    x2 = gauss_points(2)[0]
    assert np.allclose(Ops1D(2).gR, (15 * x2 ** 2 + 6 * x2 - 3) / 4, atol=1e-14)
    assert np.allclose(Ops1D(0).gR, [0.5])
    for P in range(0, 6):
        o = Ops1D(P)
        assert np.allclose(o.gL, -o.gR[::-1], atol=1e-13)


@pytest.mark.parametrize("P", range(0, 7))
def test_radau_correction_is_dg_lifting(P):
    """With Gauss points, g_DG recovers nodal DG: g_R'(x_i) = l_i(1)/w_i and g_L'(x_i) = -l_i(-1)/w_i."""
    o = Ops1D(P)
    assert np.max(np.abs(o.gR - o.lp / o.w)) < 1e-11 * max(1.0, np.max(np.abs(o.gR)))
    assert np.max(np.abs(o.gL + o.lm / o.w)) < 1e-11 * max(1.0, np.max(np.abs(o.gL)))


@pytest.mark.parametrize("Pf,Pc", [(1, 0), (2, 1), (2, 0), (3, 2), (3, 1), (4, 2), (4, 3), (5, 3)])
def test_transfer_pins(Pf, Pc):
    R1 = projection_1d(Pf, Pc)
    I1 = interpolation_1d(Pc, Pf)
    xf, wf = gauss_points(Pf)
    xc, wc = gauss_points(Pc)
    # projection after interpolation is the identity on the coarse space
    assert np.max(np.abs(R1 @ I1 - np.eye(Pc + 1))) < 1e-14
    # exact on polynomials of degree <= Pc
    for m in range(Pc + 1):
        assert np.max(np.abs(R1 @ xf ** m - xc ** m)) < 1e-13
    # the reference-element mean is preserved
    rng = np.random.default_rng(3)
    u = rng.standard_normal(Pf + 1)
    assert abs(wc @ (R1 @ u) - wf @ u) < 1e-14
    # Galerkin orthogonality: u - I P u is orthogonal to P_Pc under the exact fine quadrature
    r = u - I1 @ (R1 @ u)
    for k in range(Pc + 1):
        assert abs(np.sum(wf * r * npleg.legval(xf, np.eye(k + 1)[k]))) < 1e-14
