"""Whole-lattice reference step of the central-moment LBM (test infrastructure).

State: the paper's transformed pre-collision populations fbar(x, t), stored
as an array f[Q, nz, ny, nx] (x fastest, directions in the paper's order).

One time step (Eqs. cascadedcollision1 and cascadedstreaming1, Sec. 6):
    fbar~(x, t)          = collide(fbar(x, t))                  at fluid x
    fbar_a(x + e_a, t+1) = fbar~_a(x, t)                        periodic wrap
with half-way bounce-back (named in Sec. 9): when x + e_a is a solid node the
population returns to x reversed, fbar_abar(x, t+1) = fbar~_a(x, t).  Solid
nodes are never collided and their entries stay zero.

Initial condition (the paper gives none): fbar(x, 0) = f^eq(rho0, u0) - S/2,
the transformation fbar = f - S/2 of Sec. 4 applied to the equilibrium, so
that the velocity read back by Eq. velocitycalculation is u0.
"""
import numpy as np

from . import collision


def _nodes_last(f):
    return np.moveaxis(f, 0, -1)                     # (nz, ny, nx, Q)


def _force_field(F, shape):
    """Broadcast a uniform force (3,) or a field (3, nz, ny, nx) to (nz, ny, nx, 3)."""
    F = np.asarray(F)
    if F.ndim == 1:
        return np.broadcast_to(F, tuple(shape) + (3,))
    return np.moveaxis(F, 0, -1)


def fluid_mask(solid, shape):
    if solid is None:
        return np.ones(shape, dtype=bool)
    return ~np.asarray(solid, dtype=bool)


def collide_field(lat, f, F, omega, solid=None, per_mass=False):
    """Post-collision populations at every fluid node (solid entries 0)."""
    shape = f.shape[1:]
    fluid = fluid_mask(solid, shape)
    fn = _nodes_last(f)
    Fn = _force_field(F, shape)
    post = np.zeros(fn.shape, dtype=np.result_type(fn, Fn, np.asarray(omega)))
    post[fluid] = collision.collide(lat, fn[fluid], Fn[fluid], omega, per_mass)
    return np.moveaxis(post, -1, 0)


def stream(lat, post, solid=None):
    """Push streaming with periodic wrap and half-way bounce-back."""
    shape = post.shape[1:]
    fluid = fluid_mask(solid, shape)
    out = np.zeros_like(post)
    for a, (ex, ey, ez) in enumerate(lat.E):
        # value at x moves to x + e_a (np.roll with +e_a shift)
        out[a] = np.roll(post[a], shift=(ez, ey, ex), axis=(0, 1, 2))
    if solid is not None:
        for a, (ex, ey, ez) in enumerate(lat.E):
            target_solid = np.roll(~fluid, shift=(-ez, -ey, -ex), axis=(0, 1, 2))   # solid at x + e_a
            hit = fluid & target_solid
            out[lat.opp[a]][hit] = post[a][hit]
        out[:, ~fluid] = 0
    return out


def stream_wall_fraction(lat, post, phi):
    """Streaming with a wall fraction phi(x) in [0, 1] per node, a linear blend
    of plain streaming and the half-way bounce-back named in Sec. 9 (the paper
    has only whole walls; this continuous form exists to differentiate the loss
    with respect to the wall layout):

        fbar_a(x) = (1 - phi(x)) fbar~_a(x - e_a) + phi(x - e_a) fbar~_abar(x).

    A population leaving s towards t = s + e_a arrives at t with weight
    1 - phi(t) and returns to s, reversed, with weight phi(t), so mass is
    conserved.  Nodes with phi = 1 are solid: never collided, zero populations.
    With phi in {0, 1} this is ``stream(lat, post, solid=(phi == 1))`` exactly."""
    phi = np.asarray(phi)
    out = np.zeros(post.shape, dtype=np.result_type(post, phi))
    for a, (ex, ey, ez) in enumerate(lat.E):
        shift = (int(ez), int(ey), int(ex))
        pulled = np.roll(post[a], shift=shift, axis=(0, 1, 2))        # fbar~_a(x - e_a)
        phi_src = np.roll(phi, shift=shift, axis=(0, 1, 2))           # phi(x - e_a)
        out[a] = (1 - phi) * pulled + phi_src * post[lat.opp[a]]
    out[:, phi == 1] = 0
    return out


def step_wall_fraction(lat, f, F, omega, phi, per_mass=False):
    """One step with the wall-fraction streaming above; nodes with phi < 1
    collide."""
    solid = np.asarray(phi) == 1
    return stream_wall_fraction(lat, collide_field(lat, f, F, omega, solid, per_mass), phi)


def step(lat, f, F, omega, solid=None, per_mass=False):
    """One collide-and-stream step of the pre-collision state (per_mass: the
    attractor form, see collision.attractors)."""
    return stream(lat, collide_field(lat, f, F, omega, solid, per_mass), solid)


def run(lat, f, F, omega, nsteps, solid=None, callback=None, per_mass=False):
    for n in range(nsteps):
        f = step(lat, f, F, omega, solid, per_mass)
        if callback is not None:
            callback(n + 1, f)
    return f


def initial_state(lat, rho0, u0, F, solid=None):
    """fbar(x, 0) = f^eq(rho0, u0) - S(F, u0)/2 at fluid nodes.

    rho0: (nz, ny, nx), u0: (3, nz, ny, nx), F: (3,) or (3, nz, ny, nx)."""
    rho0 = np.asarray(rho0)
    shape = rho0.shape
    fluid = fluid_mask(solid, shape)
    u = np.moveaxis(np.asarray(u0), 0, -1)
    Fn = _force_field(F, shape)
    f = np.zeros(shape + (lat.Q,), dtype=np.result_type(float, rho0, u, Fn))
    feq = collision.equilibrium(lat, rho0[fluid], u[fluid])
    S = collision.source(lat, Fn[fluid], u[fluid])
    f[fluid] = feq - 0.5 * S
    return np.moveaxis(f, -1, 0)


def macroscopic_fields(lat, f, F, solid=None):
    """rho (nz, ny, nx) and u (3, nz, ny, nx); zero at solid nodes."""
    shape = f.shape[1:]
    fluid = fluid_mask(solid, shape)
    fn = _nodes_last(f)
    Fn = _force_field(F, shape)
    rho = np.zeros(shape)
    u = np.zeros(shape + (3,))
    r, v = collision.macroscopic(lat, fn[fluid], Fn[fluid])
    rho[fluid] = r
    u[fluid] = v
    return rho, np.moveaxis(u, -1, 0)


def totals(lat, f, F, solid=None):
    """(sum rho, sum rho u_x, sum rho u_y, sum rho u_z) over fluid nodes, with
    rho u = sum fbar e + F/2 (Eq. velocitycalculation)."""
    shape = f.shape[1:]
    fluid = fluid_mask(solid, shape)
    fn = _nodes_last(f)[fluid]
    Fn = _force_field(F, shape)[fluid]
    j = fn @ lat.E + 0.5 * Fn
    return np.array([fn.sum(), j[:, 0].sum(), j[:, 1].sum(), j[:, 2].sum()])


def kinetic_energy(lat, f, F, solid=None):
    """Mean kinetic energy (1/N) sum_x |rho u|^2 / (2 rho) over the N fluid nodes."""
    shape = f.shape[1:]
    fluid = fluid_mask(solid, shape)
    fn = _nodes_last(f)[fluid]
    Fn = _force_field(F, shape)[fluid]
    rho = fn.sum(axis=-1)
    j = fn @ lat.E + 0.5 * Fn
    return (0.5 * (j * j).sum(axis=-1) / rho).mean()
