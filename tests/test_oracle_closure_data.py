"""Pins of the oracle's closure-sample pipeline (filter, strain, target,
features) against closed forms."""
import math

import numpy as np
import pytest

from oracle import closure_ref as cr


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                          indexing="ij")
    return x, y, z


def test_linear_shear_recovers_the_fine_eddy_viscosity():
    """u = (a y, 0, 0), fine nu_t = nu0: every coarse cell has Sb_xy = a (a
    coarse cell spans two fine cells, so the coarse velocity gradient is 2a),
    the subfilter stress tau_xy = -nu0 a and tau_xx = a^2/4 (the variance over
    the block), and the fitted viscosity is nu0/2 (viscosity in coarse
    lattice units is half the fine-unit value)."""
    nx, ny, nz, a, nu0, tau0, h = 8, 10, 6, 3e-3, 2e-4, 0.5005, 5.0
    x, y, z = _grid(nx, ny, nz)
    u = np.zeros((3, nz, ny, nx))
    u[0] = a * y
    nut = np.full((nz, ny, nx), nu0)
    lad = np.linspace(0, 0.4, ny // 2)
    X, t, ex = cr.samples(u, nut, tau0, h, lad)
    np.testing.assert_allclose(ex["Sb"][0, 1], a, rtol=1e-12)
    np.testing.assert_allclose(ex["tau"][0, 1], -nu0 * a, rtol=1e-12)
    np.testing.assert_allclose(ex["tau"][0, 0], a * a / 4, rtol=1e-12)
    np.testing.assert_allclose(t, nu0 / 2, rtol=1e-12)
    p = -2.0 * (tau0 + 1.5 * nu0) * a
    np.testing.assert_allclose(X[:, 0], 0.0, atol=1e-18)
    np.testing.assert_allclose(X[:, 1], 2 * p * p, rtol=1e-12)
    np.testing.assert_allclose(X[:, 2], 0.0, atol=1e-18)
    np.testing.assert_allclose(X[:, 3], 0.0, atol=1e-18)
    np.testing.assert_allclose(X[:, 4], p * p, rtol=1e-12)
    np.testing.assert_allclose(X[:, 5], math.sqrt(2) * abs(p), rtol=1e-12)
    cy = ny // 2
    np.testing.assert_allclose(X[:, 6].reshape(nz // 2, cy, nx // 2)[0, :, 0],
                               (np.arange(cy) + 0.5) / h)
    np.testing.assert_allclose(X[:, 7].reshape(nz // 2, cy, nx // 2)[0, :, 0], lad)
    assert np.all(X[:, 8] == 1.0)


def test_uniform_flow_has_no_subfilter_stress():
    u = np.zeros((3, 4, 6, 8))
    u[0], u[1], u[2] = 0.05, -0.01, 0.02
    X, t, ex = cr.samples(u, np.full(u.shape[1:], 1e-4), 0.52, 3.0, np.zeros(3))
    assert np.all(t == 0.0)
    np.testing.assert_allclose(ex["tau"], 0.0, atol=1e-18)
    assert np.all(X[:, :6] == 0.0)


def test_periodic_central_difference_of_a_sine():
    nx = 16
    x, y, z = _grid(nx, 4, 4)
    k = 2 * math.pi / nx
    u = np.zeros((3, 4, 4, nx))
    u[1] = np.sin(k * x)
    g = cr.grad(u)
    np.testing.assert_allclose(g[1, 0], np.cos(k * x) * math.sin(k), atol=1e-15)
    np.testing.assert_allclose(g[0], 0.0)


def test_box_filter_of_a_trilinear_field_is_the_block_centre_value():
    x, y, z = _grid(6, 4, 8)
    f = 1 + 2 * x - 3 * y + 0.5 * z + 0.1 * x * y * z
    b = cr.box(f)
    X, Y, Z = _grid(3, 2, 4)
    centre = 1 + 2 * (2 * X) - 3 * (2 * Y) + 0.5 * (2 * Z)
    # the xyz term averages to the centre value plus zero (odd deviations cancel)
    np.testing.assert_allclose(b, centre + 0.1 * (2 * X) * (2 * Y) * (2 * Z), rtol=1e-13)
