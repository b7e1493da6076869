"""The validation flows of Sec. 9 run on the GPU (FP64 storage and arithmetic)
against their closed forms, with the paper's parameters.

Geometry (fixed by the paper's quoted Reynolds and Womersley numbers): N nodes
across, one solid layer at each end, half-way bounce-back walls, so the
half-width is a = (N - 2)/2.  Viscosity nu = (1/omega - 1/2)/3 (end of Sec. 7).

* Plates, 3 x 3 x 45, omega 1.818, F_x = 2, 4, 6e-7 (Re 3.6, 7.2, 10.7), both
  lattices; D3Q15 at F_x = 1e-6 with omega 1.923 and 1.961 (Re 111.8, 447.2).
* Grid convergence under diffusive scaling, 3 x 3 x N, F ~ 1/a^3 from
  F = 6.958e-6 at N = 13: the error against the parabola falls as N^-2.
* Womersley flow, 3 x 3 x 45, F_x = F_m cos(Omega t), F_m = 1e-5, T = 10000,
  omega 1.724 and 1.923 (Wo 3.3, 6.6), through the force-scale call, against
  the solution of the same momentum equation from rest.
* Square duct, 3 x 45 x 45, F_x = 1e-6, omega 1.923 (Re 65.7), against
  Eq. ductFourier.

Each flow first runs a few steps against the FP64 oracle at 1e-12 on the same
geometry, then long enough for the closed form to apply.
"""
import math

import numpy as np
import pytest

import lbm_inputs as inp
from gpu_helpers import gpu_initial, gpu_setup, shear_rates
from oracle import lbm
from oracle.lattice import LATTICES
from test_oracle_flows import duct_steady_paper, nu_of, womersley

pytestmark = pytest.mark.gpu

F64 = 0


def _oracle_parity(q, shape, omega, F, solid, steps, scales=None, per_mass=False):
    """`steps` GPU steps against the oracle (force scaled per step by `scales`)."""
    lat = LATTICES[q]
    om = shear_rates(q, omega)
    sim = gpu_setup(q, shape, F64, om, F, solid, per_mass)
    rho0, u0 = np.ones(shape), np.zeros((3,) + shape)
    s = (lambda n: 1.0) if scales is None else scales
    sim.set_force_scale(s(0))
    f_post, pre = gpu_initial(sim, rho0, u0)
    other = sim.populations()
    f = lbm.initial_state(lat, rho0, u0, F * s(0), solid)
    for n in range(steps):
        sim.set_force_scale(s(n))
        sim.step(f_post, other)
        f_post, other = other, f_post
        f = lbm.step(lat, f, F * s(n), om, solid, per_mass)
    sim.set_force_scale(s(steps))
    g = sim.gather(f_post, out=pre).cpu().numpy()
    fluid = ~solid
    assert np.abs(g[:, fluid] - f[:, fluid]).max() <= 1e-12 * np.abs(f[:, fluid]).max()


def _steady_run(q, shape, omega, F, solid, nsteps, per_mass=False):
    sim = gpu_setup(q, shape, F64, shear_rates(q, omega), F, solid, per_mass)
    f_post, _ = gpu_initial(sim, np.ones(shape), np.zeros((3,) + shape))
    f_last = sim.run(f_post, sim.populations(), nsteps)
    _, u = sim.macroscopic(f_last)
    return u.cpu().numpy()


def _plates_steps(a, nu, decades=16.0):
    # slowest start-up mode decays as exp(-nu (pi / 2a)^2 t)
    return int(decades / (nu * (math.pi / (2 * a)) ** 2)) + 1


@pytest.mark.parametrize("q,F,omega,Re", [(27, 2e-7, 1.818, 3.6), (27, 4e-7, 1.818, 7.2), (27, 6e-7, 1.818, 10.7),
                                          (15, 2e-7, 1.818, 3.6), (15, 4e-7, 1.818, 7.2), (15, 6e-7, 1.818, 10.7),
                                          (15, 1e-6, 1.923, 111.8), (15, 1e-6, 1.961, 447.2)])
def test_plates_poiseuille(q, F, omega, Re):
    print(f"case plates q{q} F{F} omega{omega}", flush=True)
    N = 45
    shape = (N, 3, 3)
    solid = inp.channel_mask(3, 3, N)
    Fv = np.array([F, 0.0, 0.0])
    _oracle_parity(q, shape, omega, Fv, solid, 8)
    a, nu = (N - 2) / 2, nu_of(omega)
    u = _steady_run(q, shape, omega, Fv, solid, _plates_steps(a, nu))
    z = np.arange(1, N - 1) - (N - 1) / 2
    ua = F * (a * a - z * z) / (2 * nu)
    un = u[0, 1:-1, 1, 1]
    err = np.linalg.norm(un - ua) / np.linalg.norm(ua)
    Re_c = un.max() * a / nu
    print(f"plates q{q} Re {Re} (closed form {ua.max() * a / nu:.2f}): computed Re {Re_c:.2f}, rel L2 {err:.3e}",
          flush=True)
    assert err < 5e-3
    assert abs(Re_c - Re) / Re < 0.015
    assert np.abs(u[1:]).max() < 1e-9 * un.max()


@pytest.mark.parametrize("q", [15, 27])
def test_plates_grid_convergence(q):
    # 3 x 3 x N, omega 1.818; F = 6.958e-6 at N = 13, scaled as 1/a^3 so that
    # Re = u0 a / nu is the same at every N.
    print(f"case grid convergence q{q}", flush=True)
    omega = 1.818
    nu = nu_of(omega)
    a13 = (13 - 2) / 2
    Ns = [13, 25, 49, 97]
    errs = []
    for N in Ns:
        a = (N - 2) / 2
        F = 6.958e-6 * (a13 / a) ** 3
        solid = inp.channel_mask(3, 3, N)
        u = _steady_run(q, (N, 3, 3), omega, np.array([F, 0.0, 0.0]), solid, _plates_steps(a, nu, 20.0))
        z = np.arange(1, N - 1) - (N - 1) / 2
        ua = F * (a * a - z * z) / (2 * nu)
        errs.append(np.linalg.norm(u[0, 1:-1, 1, 1] - ua) / np.linalg.norm(ua))
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    print(f"grid convergence q{q}: N {Ns} rel L2 {['%.3e' % e for e in errs]} slope {slope:.3f}", flush=True)
    assert -2.3 < slope < -1.7
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))


@pytest.mark.parametrize("omega,Wo", [(1.724, 3.3), (1.923, 6.6)])
def test_womersley(omega, Wo):
    print(f"case womersley Wo{Wo}", flush=True)
    N, q, Fm, T = 45, 15, 1e-5, 10000
    shape = (N, 3, 3)
    solid = inp.channel_mask(3, 3, N)
    Om = 2 * math.pi / T
    Fv = np.array([Fm, 0.0, 0.0])
    _oracle_parity(q, shape, omega, Fv, solid, 8, scales=lambda n: math.cos(Om * n * 1000))
    a, nu = (N - 2) / 2, nu_of(omega)
    assert abs(a * math.sqrt(Om / nu) - Wo) < 0.01
    sim = gpu_setup(q, shape, F64, shear_rates(q, omega), Fv, solid)
    sim.set_force_scale(1.0)
    f_post, _ = gpu_initial(sim, np.ones(shape), np.zeros((3,) + shape))
    other = sim.populations()
    z = np.arange(1, N - 1) - (N - 1) / 2
    checks = [2 * T + k * T // 8 for k in range(5)]          # first half of the third period
    errs = []
    n = 0
    for t_check in checks:
        while n < t_check:
            sim.set_force_scale(math.cos(Om * n))
            sim.step(f_post, other)
            f_post, other = other, f_post
            n += 1
        sim.set_force_scale(math.cos(Om * n))
        _, u = sim.macroscopic(f_post)
        un = u[0, 1:-1, 1, 1].cpu().numpy()
        ua = womersley(z, a, Fm, Om, nu, float(n))
        errs.append(np.abs(un - ua).max())
    scale = Fm / Om
    print(f"womersley Wo {Wo}: max |u - u_a| / (F_m/Omega) at t = {checks}: "
          f"{['%.2e' % (e / scale) for e in errs]}", flush=True)
    # half-way bounce-back with omega near 2 shifts the Stokes layer slightly:
    # 0.9% of F_m/Omega at Wo 6.6
    assert max(errs) < 1.5e-2 * scale


@pytest.mark.parametrize("q,per_mass", [(15, True), (27, False)])
def test_duct_reynolds_65_7(q, per_mass):
    # 3 x 45 x 45 (x periodic), F_x = 1e-6, omega 1.923.  The paper runs this
    # duct with D3Q15; with the literal factorized attractor that lattice grows
    # a cross-flow mode within ~10^3 steps (pinned on the oracle in
    # test_oracle_flows), so D3Q15 runs here with the per-unit-mass form, and
    # D3Q27 with the literal one.
    print(f"case duct Re 65.7 q{q} per_mass={per_mass}", flush=True)
    N, F, omega = 45, 1e-6, 1.923
    shape = (N, N, 3)
    solid = inp.duct_mask(3, N, N)
    Fv = np.array([F, 0.0, 0.0])
    _oracle_parity(q, shape, omega, Fv, solid, 4, per_mass=per_mass)
    a, nu = (N - 2) / 2, nu_of(omega)
    # slowest duct mode: exp(-2 nu (pi / 2a)^2 t)
    u = _steady_run(q, shape, omega, Fv, solid, int(16.0 / (2 * nu * (math.pi / (2 * a)) ** 2)) + 1, per_mass)
    c = np.arange(1, N - 1) - (N - 1) / 2
    Z, Y = np.meshgrid(c, c, indexing="ij")
    ua = duct_steady_paper(Y, Z, a, F, nu)
    un = u[0, 1:-1, 1:-1, 1]
    err = np.linalg.norm(un - ua) / np.linalg.norm(ua)
    Re_c = un.max() * a / nu
    print(f"duct q{q}: computed Re {Re_c:.2f} (paper 65.7), rel L2 vs Eq. ductFourier {err:.3e}", flush=True)
    assert np.isfinite(un).all()
    assert err < 1.5e-2
    assert abs(Re_c - 65.7) / 65.7 < 0.015
