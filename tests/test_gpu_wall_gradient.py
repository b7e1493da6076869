"""GPU parity of the wall-layout gradient (through the C ABI) against complex-step
derivatives of the FP64 oracle's wall-fraction step.

The wall fraction phi(x) in [0, 1] blends plain streaming and half-way
bounce-back, fbar_a(x) = (1 - phi(x)) fbar~_a(x - e_a) + phi(x - e_a)
fbar~_abar(x) (oracle/lbm.py, stream_wall_fraction); with phi in {0, 1} it is the
masked step.  cmlbm_wall_sensitivity (from the step's input, recomputing the
collision) and cmlbm_wall_sensitivity_post (from the collided state the
streaming moves) accumulate dL/dphi at every fluid node, evaluated at the
mask: one step's contribution against the oracle, and whole checkpointed runs
(torch.autograd through ``autograd.run(..., wall=phi)``, which uses the
second).
"""
import numpy as np
import pytest
import torch

import lbm_inputs as inp
from gpu_helpers import gpu_setup, shear_rates
from oracle import lbm
from oracle.lattice import LATTICES

pytestmark = pytest.mark.gpu

F64, F32 = 0, 1
H = 1e-30


def _walls(shape):
    solid = np.zeros(shape, dtype=bool)
    solid[0] = True
    solid[shape[0] // 2, shape[1] // 2, shape[2] // 3] = True
    solid[shape[0] // 2 + 1, 1:3, 5:9] = True
    return solid


def _fluid_direction(rng, solid):
    v = rng.standard_normal(solid.shape)
    v[solid] = 0.0
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("q,per_mass", [(27, False), (27, True), (15, False)])
def test_wall_sensitivity_one_step(q, per_mass):
    # d/de <mu, step(fbar; phi + e v)> at phi = mask, for random mu and v on
    # the fluid nodes, and at single fluid nodes next to a wall.
    print(f"case wall-sens step q{q} per_mass={per_mass}", flush=True)
    from paper_1202_6081_amd import cmlbm
    lat = LATTICES[q]
    shape = (6, 7, 67)
    rng = np.random.default_rng(41)
    om = list(rng.uniform(0.7, 1.9, q - 4))
    F = inp.gaussian_force(shape, 1e-4, 5)
    solid = _walls(shape)
    phi = solid.astype(float)
    sim = gpu_setup(q, shape, F64, om, F, solid, per_mass)
    rho0 = 1 + 0.01 * rng.standard_normal(shape)
    u0 = 0.05 * rng.uniform(-1, 1, (3,) + shape)
    x, _ = sim.init_equilibrium(torch.from_numpy(rho0).cuda(), torch.from_numpy(u0).cuda())
    x = sim.run(x, sim.populations(), 2)
    f_pre = sim.gather(x).cpu().numpy()
    mu = rng.standard_normal((q,) + shape)
    mu[:, solid] = 0.0
    mu_d = torch.from_numpy(mu).cuda()
    g = torch.zeros(shape, dtype=torch.float64, device="cuda")
    cmlbm.cmlbm_wall_sensitivity(sim.h, x, mu_d, g)
    g = g.cpu().numpy()
    assert np.all(g[solid] == 0.0)
    # the gather form, from the collided state the streaming moves
    x1 = sim.run(x, sim.populations(), 1)
    gp = torch.zeros(shape, dtype=torch.float64, device="cuda")
    cmlbm.cmlbm_wall_sensitivity_post(sim.h, x1, mu_d, gp)
    gp = gp.cpu().numpy()
    assert np.all(gp[solid] == 0.0)
    np.testing.assert_allclose(gp, g, rtol=1e-12, atol=1e-12 * np.abs(g).max())

    def L(p):
        return np.sum(mu * lbm.step_wall_fraction(lat, f_pre.astype(complex), F.astype(complex), om, p, per_mass))

    for k in range(2):
        v = _fluid_direction(rng, solid)
        ref = L(phi + 1j * H * v).imag / H
        got = float(np.sum(g * v))
        assert abs(got - ref) <= 1e-10 * abs(ref), (k, got, ref)
        got_post = float(np.sum(gp * v))
        assert abs(got_post - ref) <= 1e-10 * abs(ref), (k, got_post, ref)
    # single fluid nodes: beside the bottom wall, beside the obstacle, in the bulk
    for z, y, xx in [(1, 3, 10), (shape[0] // 2, shape[1] // 2, shape[2] // 3 + 1), (4, 5, 50)]:
        assert not solid[z, y, xx]
        e = np.zeros(shape)
        e[z, y, xx] = 1.0
        ref = L(phi + 1j * H * e).imag / H
        assert abs(g[z, y, xx] - ref) <= 1e-10 * abs(ref) + 1e-16, ((z, y, xx), g[z, y, xx], ref)
        assert abs(gp[z, y, xx] - ref) <= 1e-10 * abs(ref) + 1e-16, ((z, y, xx), gp[z, y, xx], ref)


def _oracle_loss(q, rho0, u0, F, om, nsteps, phi):
    lat = LATTICES[q]
    solid = np.asarray(phi) == 1
    f = lbm.initial_state(lat, rho0, u0, F, solid)
    for _ in range(nsteps):
        f = lbm.step_wall_fraction(lat, f, F, om, phi)
    return lbm.kinetic_energy(lat, f, F, solid)


@pytest.mark.parametrize("q,prec,schedule", [(27, F64, {"every": 2}), (27, F64, {"snapshots": 1}),
                                             (15, F64, {"every": 3}), (27, F32, {"every": 2})])
def test_wall_gradient_of_a_run(q, prec, schedule):
    # L = mean kinetic energy after N steps; dL/dphi of a whole checkpointed
    # run against the oracle's complex step along a random fluid direction.
    print(f"case wall-grad run q{q} p{prec} {schedule}", flush=True)
    from paper_1202_6081_amd import autograd as ag
    shape = (5, 6, 66)
    nsteps = 5
    rng = np.random.default_rng(43)
    om = np.array(rng.uniform(0.8, 1.9, q - 4))
    F = inp.gaussian_force(shape, 1e-4, 8)
    solid = _walls(shape)
    phi = solid.astype(float)
    rho0 = 1 + 0.01 * rng.standard_normal(shape)
    u0 = 0.05 * rng.uniform(-1, 1, (3,) + shape)
    u0[:, solid] = 0.0
    sim = gpu_setup(q, shape, prec, list(om))
    real = torch.float64 if prec == F64 else torch.float32
    Ft = torch.from_numpy(F).cuda().requires_grad_(True)
    wt = torch.from_numpy(om.copy()).requires_grad_(True)
    pt = torch.from_numpy(phi).cuda().requires_grad_(True)
    out = ag.run(sim, torch.from_numpy(rho0).cuda().to(real), torch.from_numpy(u0).cuda().to(real), Ft, wt,
                 nsteps, wall=pt, **schedule)
    ag.kinetic_energy(sim, out, Ft).backward()
    g = pt.grad.double().cpu().numpy()
    assert np.all(g[solid] == 0.0)
    for k in range(2):
        v = _fluid_direction(rng, solid)
        ref = _oracle_loss(q, rho0, u0, F, list(om), nsteps, phi + 1j * H * v).imag / H
        got = float(np.sum(g * v))
        tol = 1e-9 if prec == F64 else 1e-3   # FP32: the populations round to 2^-24 every step (measured 2.4e-4)
        print(f"wall-grad q{q} p{prec}: dir {k}: {got:.10e} vs oracle {ref:.10e}", flush=True)
        assert abs(got - ref) <= tol * abs(ref), (k, got, ref)


@pytest.mark.parametrize("q,prec,shape", [(27, F64, (19, 5, 70)), (15, F64, (17, 4, 64)), (27, F32, (9, 3, 300))])
def test_wall_sensitivity_forms_agree(q, prec, shape):
    # The gather form (taken in tiles of 8 planes, z fastest: several tiles and
    # a ragged last one here) against the scatter form with atomics, on walls
    # that cross tile boundaries; each fluid node's sum has the same terms.
    print(f"case wall forms q{q} p{prec} {shape}", flush=True)
    from paper_1202_6081_amd import cmlbm
    rng = np.random.default_rng(47)
    om = list(rng.uniform(0.7, 1.9, q - 4))
    F = inp.gaussian_force(shape, 1e-4, 9)
    solid = _walls(shape)
    solid[7:9, 2, 10:20] = True           # a block across the first tile boundary (z = 8)
    solid[-1] = True
    sim = gpu_setup(q, shape, prec, om, F, solid)
    real = torch.float64 if prec == F64 else torch.float32
    rho0 = 1 + 0.01 * rng.standard_normal(shape)
    u0 = 0.05 * rng.uniform(-1, 1, (3,) + shape)
    x, _ = sim.init_equilibrium(torch.from_numpy(rho0).cuda().to(real), torch.from_numpy(u0).cuda().to(real))
    x = sim.run(x, sim.populations(), 2)
    x1 = sim.run(x, sim.populations(), 1)
    mu = rng.standard_normal((q,) + shape)
    mu[:, solid] = 0.0
    mu_d = torch.from_numpy(mu).cuda().to(real)
    g = torch.zeros(shape, dtype=torch.float64, device="cuda")
    gp = torch.zeros(shape, dtype=torch.float64, device="cuda")
    cmlbm.cmlbm_wall_sensitivity(sim.h, x, mu_d, g)
    cmlbm.cmlbm_wall_sensitivity_post(sim.h, x1, mu_d, gp)
    g, gp = g.cpu().numpy(), gp.cpu().numpy()
    assert np.all(gp[solid] == 0.0) and np.any(gp != 0.0)
    # FP64: rounding order only; FP32: the stored state is the collision's
    # result rounded once, the recomputed one may fuse differently (2^-24 scale)
    tol = 1e-12 if prec == F64 else 1e-5
    np.testing.assert_allclose(gp, g, rtol=tol, atol=tol * np.abs(g).max())


def test_full_size_wall_term_sampled_nodes():
    # The wall-layout term of the benchmark's wall-bounded measurement (512^3
    # D3Q27 FP32, square duct, Kolmogorov force, shear rate 1.9), in the launch
    # configuration the benchmark times, at 384 sampled fluid nodes (beside the
    # walls, in the duct's corners and in the bulk) against the complex step of
    # the oracle's wall-fraction streaming on the 3x3x3 neighbourhood of each
    # node, whose post-collision populations are the oracle's collision of the
    # pre-collision state the GPU pulled.  (On a periodic 3-wide patch phi at
    # the centre enters exactly the terms it enters on the lattice.)
    from oracle import collision
    print("case wall term full512", flush=True)
    n, q = 512, 27
    lat = LATTICES[q]
    om = shear_rates(q, 1.9)
    solid = inp.duct_mask(n, n, n)
    sim = gpu_setup(q, (n, n, n), F32, om, None, solid)
    F = torch.from_numpy(inp.kolmogorov_force(n)).to("cuda", torch.float32)
    sim.set_force(F)
    g = torch.Generator(device="cuda").manual_seed(5)
    rho0 = torch.ones((n, n, n), device="cuda", dtype=torch.float32)
    u0 = 0.03 * (torch.rand((3, n, n, n), device="cuda", generator=g) - 0.5)
    sd = torch.from_numpy(solid).cuda()
    u0[:, sd] = 0.0
    x, pre = sim.init_equilibrium(rho0, u0)
    del rho0, u0
    x1 = sim.populations()
    sim.step(x, x1)
    pre = sim.gather(x, out=pre)                 # fbar at every node: what the step collided
    lam = torch.randn((q, n, n, n), device="cuda", generator=g)
    lam[:, sd] = 0.0
    dphi = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    sim.wall_sensitivity_post(x1, lam, dphi)
    del x, x1
    rng = np.random.default_rng(6)
    picks = [(1, 1, 0), (1, n - 2, n - 1), (n - 2, n - 2, 7), (1, 200, 31), (300, 1, 400), (n - 2, 100, 0)]
    picks += [tuple(int(v) for v in (rng.integers(1, 4), rng.integers(1, n - 1), rng.integers(0, n))) for _ in range(90)]
    picks += [tuple(int(v) for v in (rng.integers(1, n - 1), rng.integers(n - 4, n - 1), rng.integers(0, n))) for _ in range(90)]
    picks += [tuple(int(v) for v in (rng.integers(1, n - 1), rng.integers(1, n - 1), rng.integers(0, n))) for _ in range(192)]
    offs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    nodes = np.array([[((z + dz) % n) * n * n + ((y + dy) % n) * n + (xx + dx) % n for dz, dy, dx in offs]
                      for z, y, xx in picks])                                          # (samples, 27)
    flat = torch.from_numpy(nodes.reshape(-1)).to("cuda")
    f_in = pre.reshape(q, -1)[:, flat].double().cpu().numpy().T                        # (samples*27, q)
    Fs = F.reshape(3, -1)[:, flat].double().cpu().numpy().T
    lam_p = lam.reshape(q, -1)[:, flat].double().cpu().numpy().T.reshape(len(picks), 27, q)
    got = dphi.reshape(-1)[torch.from_numpy(nodes[:, 13]).to("cuda")].cpu().numpy()
    del pre, lam, dphi
    torch.cuda.empty_cache()
    solid_p = solid.reshape(-1)[nodes]                                                 # (samples, 27)
    fl = ~solid_p.reshape(-1)
    post = np.zeros((len(picks) * 27, q))          # solid nodes hold no populations
    post[fl] = collision.collide(lat, f_in[fl], Fs[fl], np.array(om))
    post = post.reshape(len(picks), 27, q)
    want = np.empty(len(picks))
    for k in range(len(picks)):
        phi = solid_p[k].reshape(3, 3, 3).astype(complex)
        assert phi[1, 1, 1] == 0
        phi[1, 1, 1] += 1j * H
        out = lbm.stream_wall_fraction(lat, post[k].T.reshape(q, 3, 3, 3).astype(complex), phi)
        want[k] = np.sum(lam_p[k].T.reshape(q, 3, 3, 3) * out).imag / H
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"wall term full512: rel err {err:.2e} over {len(picks)} nodes", flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("q", [27, 15])
@pytest.mark.parametrize("frac", [0.0, 0.2])
def test_one_nan_through_the_wall_term(q, frac):
    """Addressing of the gather form, row tiles included (20 planes: tiles of
    8, 8 and 4), on 130-node rows: dL/dphi(t) += sum_a x_a(s) (lam_abar(s) -
    lam_a(t)), s = t - e_a, terms from solid sources dropped.  A NaN in
    lam_b(m) enters the term of t = m (as lam_a(t), a = b) and of t = m - e_b
    (as lam_abar(s), s = m), both only when m and m - e_b are fluid; a NaN in
    x_a(s) enters the term of t = s + e_a only, when s and t are fluid.
    Exactly those entries of dL/dphi must be NaN."""
    lat = LATTICES[q]
    shape = (20, 6, 130)
    nz, ny, nx = shape
    rng = np.random.default_rng(41 + q + int(10 * frac))
    solid = rng.random(shape) < frac if frac else None
    fluid = np.ones(shape, dtype=bool) if solid is None else ~solid
    sim = gpu_setup(q, shape, F32, shear_rates(q, 1.6), [1e-4, 0, 0], solid)
    u0 = 0.04 * (rng.random((3,) + shape) - 0.5)
    if solid is not None:
        u0[:, solid] = 0.0
    x, _ = sim.init_equilibrium(torch.ones(shape, device="cuda"), torch.from_numpy(u0).to("cuda", torch.float32))
    x_h = sim.export_populations(x).cpu().numpy()
    lam_base = torch.from_numpy(rng.standard_normal((q,) + shape)).to("cuda", torch.float32)

    def wrap(p):
        return (p[0] % nz, p[1] % ny, p[2] % nx)

    def shifted(p, b, sign):
        ex, ey, ez = (int(c) for c in lat.E[b])
        return wrap((p[0] + sign * ez, p[1] + sign * ey, p[2] + sign * ex))

    def run(lam, xbuf):
        d = torch.zeros(shape, dtype=torch.float64, device="cuda")
        sim.wall_sensitivity_post(xbuf, lam, d)
        return torch.isnan(d).cpu().numpy()

    checked = 0
    for _ in range(12):
        b = int(rng.integers(1, q))
        m = (int(rng.integers(0, nz)), int(rng.integers(0, ny)), int(rng.integers(0, nx)))
        lam = lam_base.clone()
        lam[(b,) + m] = float("nan")
        want = np.zeros(shape, dtype=bool)
        t2 = shifted(m, b, -1)
        if fluid[m] and fluid[t2]:
            want[m] = want[t2] = True
            checked += 1
        assert np.array_equal(run(lam, x), want), (b, m)
    for _ in range(12):
        a = int(rng.integers(1, q))
        s = (int(rng.integers(0, nz)), int(rng.integers(0, ny)), int(rng.integers(0, nx)))
        xh = x_h.copy()
        xh[(a,) + s] = np.nan
        xbuf = sim.import_populations(torch.from_numpy(xh))
        want = np.zeros(shape, dtype=bool)
        t = shifted(s, a, +1)
        if fluid[s] and fluid[t]:
            want[t] = True
            checked += 1
        assert np.array_equal(run(lam_base, xbuf), want), (a, s)
    assert checked >= 8
