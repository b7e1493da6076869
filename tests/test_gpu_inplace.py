"""GPU parity of the in-place (one-buffer) step, through the C ABI.

Against the FP64 oracle: FP64 storage, 1e-12 relative (max norm over fluid
nodes), in both phases of the buffer: after a parity-0 call the reversed slots
hold the oracle's post-collision populations, after a parity-1 call the slots
hold its pre-collision populations two steps on.  Against the two-buffer step:
every storage type bit-identical (the same collision code on the same rounded
stored values), read back as populations, density, velocity and FP64 totals.
"""
import numpy as np
import pytest
import torch

import lbm_inputs as inp
from gpu_helpers import gpu_setup, lib, oracle_run, rel_err, to_dev
from oracle import collision, lbm
from oracle.lattice import LATTICES

pytestmark = pytest.mark.gpu

F64, F32, F16, BF16 = 0, 1, 2, 3


def _fields(shape, seed, umax=0.05):
    rng = np.random.default_rng(seed)
    return 1.0 + 0.01 * rng.standard_normal(shape), umax * rng.uniform(-1, 1, (3,) + shape)


def _force(kind, shape):
    if kind == "uniform":
        return np.array([2e-4, -1e-4, 5e-5])
    return inp.gaussian_force(shape, 1e-4, 3)


def _mask(kind, shape):
    nz, ny, nx = shape
    if kind is None:
        return None
    if kind == "duct":
        return inp.duct_mask(nx, ny, nz)
    solid = np.zeros(shape, dtype=bool)
    solid[0] = True
    solid[nz // 2, ny // 2, nx // 3] = True
    solid[nz // 2, 1, 2 * nx // 3] = True
    return solid


def _inplace_buffer(sim, rho0, u0):
    """Phase-0 buffer holding fbar(0), and the two-buffer post-collision state."""
    f_post, f_pre = sim.init_equilibrium(to_dev(rho0, sim.real), to_dev(u0, sim.real))
    return sim.import_populations(f_pre), f_post


def _unreverse(lat, a):
    """Phase-1 slots (slot abar of x holds direction a) -> direction order."""
    return a[list(lat.opp)]


CASES = [
    # q, (nz, ny, nx), force, mask
    (27, (5, 6, 70), "uniform", None),
    (27, (6, 5, 67), "field", "walls"),
    (27, (9, 8, 66), "uniform", "duct"),
    (15, (5, 6, 70), "field", None),
    (15, (6, 5, 67), "uniform", "walls"),
    (27, (1, 1, 1), "uniform", None),
    (27, (2, 3, 1), "field", None),
    (15, (1, 1, 5), "field", None),
]


@pytest.mark.parametrize("case", CASES, ids=[f"q{c[0]}-{'x'.join(map(str, c[1]))}-{c[2]}-{c[3]}" for c in CASES])
def test_inplace_matches_oracle(case):
    q, shape, fkind, mkind = case
    print(f"case {case}", flush=True)
    lat = LATTICES[q]
    omega = list(np.random.default_rng(7).uniform(0.7, 1.9, q - 4))
    F = _force(fkind, shape)
    solid = _mask(mkind, shape)
    fluid = None if solid is None else ~solid
    rho0, u0 = _fields(shape, 5)
    sim = gpu_setup(q, shape, F64, omega, F, solid)
    buf, _ = _inplace_buffer(sim, rho0, u0)
    steps = 4
    states = oracle_run(q, rho0, u0, F, omega, steps, solid)
    Fo = np.asarray(F, dtype=float)
    for n in range(steps):
        sim.step_inplace(buf, n & 1)
        got = sim.export_populations(buf).double().cpu().numpy()
        if n & 1 == 0:          # phase 1: reversed post-collision populations of fbar(n)
            want = lbm.collide_field(lat, states[n], Fo, omega, solid)
            got = _unreverse(lat, got)
        else:                   # phase 0: fbar(n + 1)
            want = states[n + 1]
        err = rel_err(got, want, fluid)
        assert err < 1e-12, (n, err)
    # read-outs of the phase-0 buffer against the oracle
    rho, u = sim.macroscopic_pre(buf)
    rho_o, u_o = lbm.macroscopic_fields(lat, states[steps], Fo, solid)
    fl = np.ones(shape, dtype=bool) if fluid is None else fluid
    assert np.abs(rho.cpu().numpy() - rho_o)[fl].max() < 1e-13
    assert np.abs(u.cpu().numpy() - u_o)[:, fl].max() < 1e-13
    tot = sim.totals_pre(buf)
    tot_o = lbm.totals(lat, states[steps], Fo, solid)
    assert np.allclose(tot, tot_o, rtol=1e-12, atol=1e-15)


EXACT = [
    # q, precision, (nz, ny, nx), force, mask, steps
    (27, F64, (6, 5, 67), "field", "walls", 4),
    (27, F32, (6, 5, 67), "field", "walls", 6),
    (27, F32, (4, 3, 300), "uniform", None, 6),
    (27, F16, (6, 5, 67), "field", "walls", 6),
    (27, BF16, (5, 6, 70), "uniform", None, 6),
    (15, F64, (5, 6, 70), "field", None, 4),
    (15, F32, (6, 5, 67), "uniform", "walls", 6),
    (15, F16, (4, 3, 300), "field", None, 6),
    (15, BF16, (9, 8, 66), "uniform", "duct", 6),
    (27, F32, (9, 8, 66), "uniform", "duct", 6),
    # 16-bit storage without walls takes the aligned-store scatter phase: rows
    # of one node, a one-node tail block, a one-node last segment, two full segments
    (27, F16, (3, 4, 1), "field", None, 4),
    (15, F16, (3, 2, 65), "field", None, 4),
    (27, BF16, (2, 3, 257), "uniform", None, 4),
    (27, F16, (2, 2, 512), "uniform", None, 4),
]


def _exact_id(c):
    return f"q{c[0]}-p{c[1]}-{'x'.join(map(str, c[2]))}-{c[3]}-{c[4]}-n{c[5]}"


@pytest.mark.parametrize("case", EXACT, ids=[_exact_id(c) for c in EXACT])
def test_inplace_equals_two_buffer(case):
    q, prec, shape, fkind, mkind, steps = case
    print(f"case {_exact_id(case)}", flush=True)
    omega = list(np.random.default_rng(11).uniform(0.7, 1.9, q - 4))
    F = _force(fkind, shape)
    solid = _mask(mkind, shape)
    rho0, u0 = _fields(shape, 9)
    sim = gpu_setup(q, shape, prec, omega, F, solid)
    buf, f_post = _inplace_buffer(sim, rho0, u0)
    last = sim.run(f_post, sim.populations(), steps)
    sim.run_inplace(buf, steps)
    fl = slice(None) if solid is None else torch.from_numpy(~solid).cuda()
    a = sim.gather(last)[:, fl]
    b = sim.export_populations(buf)[:, fl]
    assert torch.equal(a, b), float((a - b).abs().max())
    r1, u1 = sim.macroscopic(last)
    r2, u2 = sim.macroscopic_pre(buf)
    assert torch.equal(r1, r2) and torch.equal(u1, u2)
    assert sim.totals(last) == sim.totals_pre(buf)


def test_inplace_full_size_equals_two_buffer():
    """512^3 D3Q27 FP32, the benchmark's Kolmogorov force and rates, in the
    benchmark's launch shape: density, velocity and totals after 4 steps."""
    n = 512
    print("case 512^3 D3Q27 FP32 in-place vs two-buffer", flush=True)
    cm = lib()
    dev = torch.device("cuda", 0)
    sim = cm.Sim(27, n, n, n, cm.F32)
    sim.set_rates([1.9] * 5 + [1.0] * 18)
    sim.set_force(torch.from_numpy(inp.kolmogorov_force(n, amplitude=1e-6, waves=4)).to(dev, torch.float32))
    u0 = torch.from_numpy(inp.taylor_green(n, u0=0.02)).to(dev, torch.float32)
    f_post, f_pre = sim.init_equilibrium(torch.ones((n, n, n), device=dev), u0)
    del u0
    buf = sim.import_populations(f_pre)
    del f_pre
    last = sim.run(f_post, sim.populations(), 4)
    sim.run_inplace(buf, 4)
    r1, u1 = sim.macroscopic(last)
    r2, u2 = sim.macroscopic_pre(buf)
    assert torch.equal(r1, r2)
    assert torch.equal(u1, u2)
    assert sim.totals(last) == sim.totals_pre(buf)


def test_inplace_errors_and_zero_steps():
    cm = lib()
    sim = gpu_setup(27, (3, 4, 5), F32, [1.2] * 23)
    rho0, u0 = _fields((3, 4, 5), 1)
    buf, _ = _inplace_buffer(sim, rho0, u0)
    before = buf.clone()
    sim.run_inplace(buf, 0)
    assert torch.equal(buf, before)
    for bad in (lambda: sim.step_inplace(buf, 2), lambda: sim.step_inplace(buf, -1),
                lambda: sim.run_inplace(buf, 3), lambda: sim.run_inplace(buf, -2)):
        with pytest.raises(cm.CmlbmError) as exc:
            bad()
        assert exc.value.code == -1
    lib_ = cm.load_library()
    assert lib_.cmlbm_step_inplace(sim.h, None, 0, None) == -1
    assert lib_.cmlbm_run_inplace(sim.h, None, 2, None) == -1
    assert lib_.cmlbm_macroscopic_pre(sim.h, None, None, None, None) == -1
    assert torch.equal(buf, before)


@pytest.mark.parametrize("q,prec,mkind", [(27, F64, "walls"), (27, F32, None), (27, BF16, "duct"), (15, F16, "walls"),
                                          (15, F64, None)])
def test_init_inplace_equals_import(q, prec, mkind):
    shape = (9, 8, 66)
    print(f"case init q{q} p{prec} {mkind}", flush=True)
    solid = _mask(mkind, shape)
    sim = gpu_setup(q, shape, prec, [1.3] * (q - 4), _force("field", shape), solid)
    rho0, u0 = _fields(shape, 4)
    want, _ = _inplace_buffer(sim, rho0, u0)
    got = sim.init_equilibrium_inplace(to_dev(rho0, sim.real), to_dev(u0, sim.real))
    assert torch.equal(got, want)


def _blocked_index(q, n, z, y, x, a):
    """Element index of slot a of node (z, y, x) in a population buffer of an
    n^3 lattice (blocked rows, n a multiple of 64)."""
    b = x // 64
    return ((z * n + y) * n * q + b * 64 * q + a * 64 + (x - 64 * b)).astype(np.int64)


def test_inplace_1024_fp64_sampled_nodes():
    """1024^3 D3Q27 FP64 stepped in place: 216 GiB of state, a lattice whose two
    ping-pong buffers (432 GiB) do not fit on one MI355X.  Random density and
    velocity, uniform force, shear rate 1.9.  Checks at sampled nodes (corners
    of the periodic box included), against the oracle: the initial state; the
    collide phase (reversed slots = collision of the initial state); the
    scatter phase (pre-collision state two steps on, recomputed by the oracle
    from the phase-1 buffer around each node)."""
    n, q = 1024, 27
    need = q * 8 * n**3 + 4 * 8 * n**3
    torch.cuda.empty_cache()           # blocks cached by earlier tests
    free, _ = torch.cuda.mem_get_info()
    if free < need + (2 << 30):
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} GiB free")
    print("case 1024^3 D3Q27 FP64 in place", flush=True)
    lat = LATTICES[q]
    omega = [1.9] * 5 + [1.0] * 18
    Fv = np.array([1e-6, -2e-7, 3e-7])
    sim = gpu_setup(q, (n, n, n), F64, omega, Fv)
    buf = sim.populations()
    g = torch.Generator(device="cuda").manual_seed(5)
    rho0 = torch.rand((n, n, n), device="cuda", dtype=torch.float64, generator=g).sub_(0.5).mul_(0.02).add_(1.0)
    u0 = torch.rand((3, n, n, n), device="cuda", dtype=torch.float64, generator=g).sub_(0.5).mul_(0.1)
    sim.init_equilibrium_inplace(rho0, u0, buf)
    rng = np.random.default_rng(17)
    pts = rng.integers(0, n, (120, 3))
    corners = np.array([[z, y, x] for z in (0, n - 1) for y in (0, n - 1) for x in (0, n - 1)])
    pts = np.concatenate([corners, pts, [[5, 63, 64], [700, 1, 127], [1023, 512, 191]]])
    Z, Y, X = pts.T
    flat = buf.view(-1)

    def read(zz, yy, xx, slots):
        idx = np.stack([_blocked_index(q, n, zz, yy, xx, a) for a in slots], axis=-1)
        return flat[torch.from_numpy(idx.reshape(-1)).cuda()].cpu().numpy().reshape(idx.shape)

    zt, yt, xt = [torch.from_numpy(c).cuda() for c in (Z, Y, X)]
    r_s = rho0[zt, yt, xt].cpu().numpy()
    u_s = u0[:, zt, yt, xt].cpu().numpy()
    del rho0, u0
    Fn = np.tile(Fv, (len(pts), 1))
    f0 = read(Z, Y, X, range(q))
    want0 = lbm.initial_state(lat, r_s[None, None, :], u_s[:, None, None, :], Fv)[:, 0, 0, :].T
    assert np.abs(f0 - want0).max() < 1e-13
    # collide phase
    sim.step_inplace(buf, 0)
    torch.cuda.synchronize()
    post0 = read(Z, Y, X, [lat.opp[a] for a in range(q)])
    want = collision.collide(lat, f0, Fn, omega)
    scale = np.abs(want).max()
    assert np.abs(post0 - want).max() / scale < 1e-12
    # phase-1 buffer around every sample: post-collision populations at t = 0
    d = np.arange(-2, 3)
    DZ, DY, DX = np.meshgrid(d, d, d, indexing="ij")
    nz_, ny_, nx_ = [(c[:, None] + D.reshape(-1)[None, :]) % n for c, D in ((Z, DZ), (Y, DY), (X, DX))]
    around = read(nz_, ny_, nx_, [lat.opp[a] for a in range(q)])      # [sample, 125, a]: fbar~_a(z, 0)
    sim.step_inplace(buf, 1)
    torch.cuda.synchronize()
    got = read(Z, Y, X, range(q))                                      # fbar_a(x, 2)
    E = lat.E.astype(int)

    def pos(v):
        return (v[..., 0] + 2) * 25 + (v[..., 1] + 2) * 5 + (v[..., 2] + 2)   # offset (dz, dy, dx) -> 0..124

    want2 = np.empty_like(got)
    for a in range(q):
        ya = -E[a][::-1]                                 # y = x - e_a, as (dz, dy, dx)
        pre1 = np.stack([around[:, pos(ya - E[b][::-1]), b] for b in range(q)], axis=-1)   # fbar_b(y, 1)
        want2[:, a] = collision.collide(lat, pre1, Fn, omega)[:, a]
    assert np.abs(got - want2).max() / scale < 1e-12


@pytest.mark.parametrize("q,prec", [(27, F32), (15, F64), (27, BF16)])
def test_inplace_time_dependent_force_and_per_mass(q, prec):
    """Per-unit-mass attractors and a force scale set before every step (the
    time-periodic forcing of Sec. 9): the in-place run stays bit-identical to
    the two-buffer run."""
    shape = (6, 5, 67)
    print(f"case q{q} p{prec} force scale per step, per-mass", flush=True)
    solid = _mask("walls", shape)
    sim = gpu_setup(q, shape, prec, list(np.random.default_rng(3).uniform(0.8, 1.9, q - 4)), _force("field", shape),
                    solid, per_mass=True)
    rho0, u0 = _fields(shape, 12)
    buf, f_post = _inplace_buffer(sim, rho0, u0)
    other = sim.populations()
    steps = 8
    for n in range(steps):
        sim.set_force_scale(np.cos(2 * np.pi * n / 5))
        sim.step(f_post, other)
        f_post, other = other, f_post
        sim.step_inplace(buf, n & 1)
    fl = torch.from_numpy(~solid).cuda()
    assert torch.equal(sim.gather(f_post)[:, fl], sim.export_populations(buf)[:, fl])


@pytest.mark.parametrize("q,prec,mkind", [(27, F64, "walls"), (27, F32, None), (15, F32, "walls"), (27, F16, None),
                                          (15, BF16, None)])
def test_inplace_fused_totals(q, prec, mkind):
    """cmlbm_step_inplace_totals reduces, at every step, the same FP64 totals as
    cmlbm_step_totals of the two-buffer run (both phases; 16-bit storage without
    walls takes the aligned-store scatter phase)."""
    shape = (6, 5, 67)
    print(f"case fused totals q{q} p{prec} {mkind}", flush=True)
    solid = _mask(mkind, shape)
    sim = gpu_setup(q, shape, prec, list(np.random.default_rng(5).uniform(0.8, 1.9, q - 4)), _force("field", shape),
                    solid)
    rho0, u0 = _fields(shape, 8)
    buf, f_post = _inplace_buffer(sim, rho0, u0)
    other = sim.populations()
    t_two = torch.zeros(4, dtype=torch.float64, device="cuda")
    t_in = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    for n in range(6):
        sim.step(f_post, other, totals=t_two)
        f_post, other = other, f_post
        sim.step_inplace(buf, n & 1, totals=t_in)
        assert torch.equal(t_two, t_in), (n, t_two.tolist(), t_in.tolist())
    fl = slice(None) if solid is None else torch.from_numpy(~solid).cuda()
    assert torch.equal(sim.gather(f_post)[:, fl], sim.export_populations(buf)[:, fl])
    cm = lib()
    assert cm.load_library().cmlbm_step_inplace_totals(sim.h, _ptr_of(buf), 0, None, None) == -1


def _ptr_of(t):
    return t.data_ptr()
