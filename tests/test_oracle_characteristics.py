"""Pins of the characteristic-curve oracle (Sec. 4: pendulum flow with
exponential memory, and its equilibrium average at finite temperature).

Each test reaches the same number by another route: the Esaki-Tsu and Tucker
closed forms and the Jacobi-Anger continuum trace at B = 0, the
finite-difference BTE oracle with Richardson extrapolation in dphi at B != 0,
exact symmetries of the flow, and convergence in the quadrature parameters.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle



@pytest.mark.parametrize("mu", [None, 116.0])
@pytest.mark.parametrize("E", [0.5, 1.0, 6.0])
def test_esaki_tsu(mu, E):
    """B = 0, constant field: every point drifts uniformly in phi_x, and the
    memory integral gives (I1/I0) E/(1+E^2) (I1/I0 -> 1 at zero temperature)."""
    _, v = oracle.characteristic_v(E, 0.0, 1.0, 0.0, mu)
    ratio = 1.0 if mu is None else sp.ive(1, mu) / sp.ive(0, mu)
    # next Euler-Maclaurin term: h^4/720 * E^3 ~ 3e-9 at E = 6, h = 0.01
    assert abs(v[0] - ratio * E / (1 + E * E)) < 1e-8


@pytest.mark.parametrize("E_dc,E_w,omega", [(6.0, 0.1, 2.0), (5.0, 1.0, 1.0), (0.0, 0.5, 3.0)])
def test_b0_trace_and_tucker(E_dc, E_w, omega):
    """B = 0, ac field: the whole periodic trace v(t) equals (I1/I0) Im u(t)
    of the Jacobi-Anger continuum state, and A equals the Tucker sum for any
    temperature (A carries I0/I1)."""
    mu = 116.0
    t, v = oracle.characteristic_v(E_dc, E_w, omega, 0.0, mu)
    ratio = sp.ive(1, mu) / sp.ive(0, mu)
    ref = ratio * oracle.continuum_u(E_dc, E_w, omega, t).imag
    # fourth-order quadrature in tau at h = 0.01: a few 1e-9
    np.testing.assert_allclose(v, ref, rtol=0, atol=1e-8)
    ref_A = oracle.tucker_absorption(E_dc, E_w, omega)
    for m in (None, mu):
        A = oracle.characteristic_absorption(E_dc, E_w, omega, 0.0, m)
        assert abs(A - ref_A) < 1e-8 * max(1.0, abs(ref_A)), (m, A, ref_A)


def test_origin_at_rest():
    """Zero temperature, no field: the point stays at the stable equilibrium."""
    _, v = oracle.characteristic_v(0.0, 0.0, 1.0, 4.0, None)
    assert v[0] == 0.0


def test_symmetries():
    """phi -> -phi maps the flow for E to the flow for -E (v odd in E);
    phi_y -> -phi_y maps B to -B (v even in B); f0 is even in both."""
    for mu in (None, 116.0):
        _, vp = oracle.characteristic_v(3.0, 0.5, 2.0, 4.0, mu, nodes=8)
        _, vm = oracle.characteristic_v(-3.0, -0.5, 2.0, 4.0, mu, nodes=8)
        _, vb = oracle.characteristic_v(3.0, 0.5, 2.0, -4.0, mu, nodes=8)
        np.testing.assert_allclose(vm, -vp, rtol=0, atol=1e-15)
        np.testing.assert_allclose(vb, vp, rtol=0, atol=1e-15)
        assert np.abs(vp).max() > 1e-2


def test_converges_in_nodes_steps_and_memory():
    """The B != 0 ac result is converged in the node count (to ~1e-5 of A: with
    the drive, neighbouring orbits dephase over the memory time and the
    node sum converges slowly, not spectrally), fourth order in the step
    (halving h changes it by about 1/16 of the previous change) and
    insensitive to the memory cut-off beyond e^{-36}."""
    args = (6.0, 0.1, 2.0, 4.0, 116.0)
    A = {(n, h, tm): oracle.characteristic_absorption(*args, nodes=n, h=h, tau_max=tm)
         for n, h, tm in ((8, 0.01, 36.0), (12, 0.01, 36.0), (16, 0.01, 36.0),
                          (12, 0.02, 36.0), (12, 0.04, 36.0), (12, 0.01, 30.0))}
    ref = A[(12, 0.01, 36.0)]
    assert abs(A[(8, 0.01, 36.0)] - ref) < 2e-5 * abs(ref)
    assert abs(A[(16, 0.01, 36.0)] - ref) < 2e-5 * abs(ref)
    assert abs(A[(12, 0.01, 30.0)] - ref) < 1e-12
    d1 = abs(A[(12, 0.04, 36.0)] - A[(12, 0.02, 36.0)])
    d2 = abs(A[(12, 0.02, 36.0)] - ref)
    assert d2 < d1 / 8 or d2 < 1e-12, (d1, d2)


def test_finite_temperature_matches_finite_difference_bte():
    """B = 4, E = 6, mu = 116 (the static point of the Fig. 4b parameters): the
    BTE oracle's steady drift velocity on two phi_y grids converges at second
    order in dphi, and its Richardson extrapolation equals the characteristic
    solution.  This ties the flow's signs and the equilibrium average to the
    Fourier equations of Sec. 2."""
    E, B, mu = 6.0, 4.0, 116.0
    _, vc = oracle.characteristic_v(E, 0.0, 1.0, B, mu)
    got = {}
    for cells in (800, 600):          # dphi = 5/800 and 5/600 on [-4, 1]
        pb = oracle.Problem(nx=100, ny=cells + 1, phiy_min=-4.0, phiy_max=1.0, E_dc=E,
                            E_w=0.0, omega=1.0, B=B, mu=mu, dt=2e-3)
        got[cells] = oracle.run(pb, 10000).v
    r = (800 / 600) ** 2
    e1, e2 = got[800] - vc[0], got[600] - vc[0]
    # both errors are small, of one sign, and in the ratio of dphi^2
    assert 0 < abs(e1) < 1e-5 and abs(e2 / e1 - r) < 0.1, (e1, e2)
    extrap = got[800] + (got[800] - got[600]) / (r - 1)
    assert abs(extrap - vc[0]) < 1e-7, (extrap, vc[0])
