"""Shared helpers of the GPU tests: run the HIP library and the oracle on the
same seeded inputs."""
import numpy as np
import torch

from oracle import lbm
from oracle.lattice import LATTICES


def lib():
    from paper_1202_6081_amd import cmlbm
    return cmlbm


def shear_rates(q, shear, others=1.0):
    return [shear] * 5 + [others] * (q - 9)


def gpu_setup(q, shape, precision, omega, F=None, solid=None, per_mass=False):
    """Create a Sim; F is None, a 3-vector or a (3, nz, ny, nx) array."""
    cm = lib()
    nz, ny, nx = shape
    sim = cm.Sim(q, nx, ny, nz, precision)
    sim.set_rates(omega)
    if per_mass:
        sim.set_attractor_per_mass(True)
    if F is not None:
        F = np.asarray(F, dtype=float)
        if F.ndim == 1:
            sim.set_force(F)
        else:
            sim.set_force(torch.from_numpy(F))
    if solid is not None:
        sim.set_mask(torch.from_numpy(np.asarray(solid, dtype=np.uint8)))
    return sim


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def gpu_initial(sim, rho0, u0):
    f_post, f_pre = sim.init_equilibrium(to_dev(rho0, sim.real), to_dev(u0, sim.real))
    return f_post, f_pre


def gpu_pre(sim, f_post):
    return sim.gather(f_post).double().cpu().numpy()


def oracle_run(q, rho0, u0, F, omega, nsteps, solid=None, per_mass=False):
    lat = LATTICES[q]
    Fo = np.zeros(3) if F is None else np.asarray(F, dtype=float)
    f = lbm.initial_state(lat, rho0, u0, Fo, solid)
    states = [f]
    for _ in range(nsteps):
        f = lbm.step(lat, f, Fo, omega, solid, per_mass)
        states.append(f)
    return states


def rel_err(a, b, fluid=None):
    if fluid is not None:
        a = a[..., fluid]
        b = b[..., fluid]
    return float(np.abs(a - b).max() / np.abs(b).max())


def velocity_l2(u_a, u_b, fluid=None):
    if fluid is not None:
        u_a = u_a[:, fluid]
        u_b = u_b[:, fluid]
    return float(np.linalg.norm(u_a - u_b) / np.linalg.norm(u_b))
