"""The oracle's process-pool step (oracle/pool.py) is the oracle's step: the
per-node collisions split over worker processes give bit-identical states,
real and complex, with walls and a force field; and the committed decay
goldens start as the oracle's plain run does."""
import json
import os

import numpy as np
import pytest

import lbm_inputs as inp
from oracle import lbm
from oracle.lattice import D3Q15, D3Q27
from oracle.pool import Pool

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def pool():
    with Pool(2) as p:
        yield p


@pytest.mark.parametrize("lat", [D3Q27, D3Q15], ids=str)
def test_pool_step_is_the_oracle_step(pool, lat):
    n = 10
    u0 = inp.random_spectrum_velocity(n, seed=3, shells=(1, 3))
    F = inp.gaussian_force((n, n, n), 1e-5, 1)
    solid = inp.channel_mask(n, n, n)
    om = list(np.random.default_rng(0).uniform(0.5, 1.9, lat.Q - 4))
    f = lbm.initial_state(lat, np.ones((n, n, n)), u0, F, solid)
    assert np.array_equal(pool.step(lat, f, F, om, solid), lbm.step(lat, f, F, om, solid))
    Fc = F.astype(complex)
    Fc[0, 3, 3, 3] += 1e-30j
    fc = f.astype(complex)
    a = pool.step(lat, fc, Fc, om, solid, per_mass=True)
    b = lbm.step(lat, fc, Fc, om, solid, per_mass=True)
    assert a.dtype == np.complex128 and np.array_equal(a, b)


@pytest.mark.parametrize("q", [15, 27])
def test_decay_golden_starts_as_the_oracle_run(pool, q):
    with open(os.path.join(HERE, "golden", f"decay32_d3q{q}.json")) as fh:
        g = json.load(fh)
    r = g["recipe"]
    lat = {15: D3Q15, 27: D3Q27}[q]
    n = r["n"]
    u0 = inp.random_spectrum_velocity(n, seed=r["field_seed"])
    F = np.zeros(3)
    f = lbm.initial_state(lat, np.ones((n, n, n)), u0, F)
    assert lbm.kinetic_energy(lat, f, F) == g["ke"][0]
    f = pool.run(lat, f, F, r["rates"], r["ke_every"])
    assert lbm.kinetic_energy(lat, f, F) == g["ke"][1]
