"""Pins of the oracle's wall-fraction streaming (the continuous form of the
half-way bounce-back that the wall-layout gradient differentiates).

* with phi in {0, 1} it is the masked step, bit for bit (channel, duct and
  scattered solid nodes, both lattices, both attractor forms);
* mass is conserved for fractional phi;
* a uniform fraction c in a periodic box reverses the fraction c of the
  post-collision momentum every step: for a uniform state j(n+1) =
  (1 - 2c)(j(n) + F), a closed form, with j = sum fbar e;
* it is affine in phi for fixed post-collision populations (so the complex
  step in phi is exact).
"""
import numpy as np
import pytest

import lbm_inputs as inp
from oracle import collision, lbm
from oracle.lattice import D3Q15, D3Q27


def _geometries(shape):
    nz, ny, nx = shape
    yield "channel", inp.channel_mask(nx, ny, nz)
    yield "duct", inp.duct_mask(nx, ny, nz)
    rng = np.random.default_rng(4)
    yield "scattered", rng.random(shape) < 0.15


@pytest.mark.parametrize("per_mass", [False, True])
@pytest.mark.parametrize("lat", [D3Q27, D3Q15], ids=str)
def test_binary_fraction_is_the_masked_step(lat, per_mass):
    shape = (6, 7, 8)
    rng = np.random.default_rng(1)
    om = list(rng.uniform(0.6, 1.9, lat.Q - 4))
    F = inp.gaussian_force(shape, 1e-4, 2)
    for name, solid in _geometries(shape):
        u0 = 0.05 * rng.uniform(-1, 1, (3,) + shape)
        f = lbm.initial_state(lat, 1 + 0.01 * rng.standard_normal(shape), u0, F, solid)
        phi = solid.astype(float)
        a = lbm.step_wall_fraction(lat, f, F, om, phi, per_mass)
        b = lbm.step(lat, f, F, om, solid, per_mass)
        assert np.array_equal(a, b), name


@pytest.mark.parametrize("lat", [D3Q27, D3Q15], ids=str)
def test_mass_conserved_with_fractional_walls(lat):
    shape = (5, 6, 7)
    rng = np.random.default_rng(2)
    om = list(rng.uniform(0.6, 1.9, lat.Q - 4))
    F = inp.gaussian_force(shape, 1e-4, 3)
    phi = np.where(rng.random(shape) < 0.3, rng.uniform(0, 1, shape), 0.0)
    phi[0] = 1.0
    f = lbm.initial_state(lat, np.ones(shape), 0.05 * rng.uniform(-1, 1, (3,) + shape), F, phi == 1)
    m0 = f.sum()
    for _ in range(3):
        f = lbm.step_wall_fraction(lat, f, F, om, phi)
    assert abs(f.sum() / m0 - 1) <= 1e-14
    assert np.all(f[:, phi == 1] == 0)


@pytest.mark.parametrize("c", [0.0, 0.1, 0.35])
@pytest.mark.parametrize("lat", [D3Q27, D3Q15], ids=str)
def test_uniform_fraction_momentum_closed_form(lat, c):
    shape = (3, 4, 5)
    F = np.array([2e-4, -1e-4, 5e-5])
    om = [1.7] * 5 + [1.0] * (lat.Q - 9)
    u0 = np.broadcast_to(np.array([0.02, -0.01, 0.005])[:, None, None, None], (3,) + shape)
    f = lbm.initial_state(lat, np.ones(shape), np.ascontiguousarray(u0), F)
    phi = np.full(shape, c)
    j = (f.reshape(lat.Q, -1).T @ lat.E).mean(axis=0)
    for _ in range(4):
        f = lbm.step_wall_fraction(lat, f, F, om, phi)
        jn = (f.reshape(lat.Q, -1).T @ lat.E)
        assert np.abs(jn - jn.mean(axis=0)).max() <= 1e-15       # the state stays uniform
        j = (1 - 2 * c) * (j + F)
        assert np.abs(jn.mean(axis=0) - j).max() <= 1e-15


def test_streaming_is_affine_in_the_fraction():
    lat = D3Q27
    shape = (4, 5, 6)
    rng = np.random.default_rng(9)
    post = rng.uniform(0, 0.1, (lat.Q,) + shape)
    p0 = np.where(rng.random(shape) < 0.5, rng.uniform(0, 0.9, shape), 0.0)
    p1 = np.where(rng.random(shape) < 0.5, rng.uniform(0, 0.9, shape), 0.0)
    s0, s1 = lbm.stream_wall_fraction(lat, post, p0), lbm.stream_wall_fraction(lat, post, p1)
    for t in (0.25, 0.5):
        st = lbm.stream_wall_fraction(lat, post, (1 - t) * p0 + t * p1)
        assert np.abs(st - ((1 - t) * s0 + t * s1)).max() <= 1e-16
