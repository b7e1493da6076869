"""GPU parity of the forward step (through the C ABI) against the FP64 oracle.

Tolerances: FP64 mode 1e-12 relative (populations, max norm); FP32 mode 2e-5
relative velocity L2 and 2e-6 absolute on populations; 16-bit deviation
storage: half a unit in the last place of the stored deviation plus 2e-6.
"""
import math

import numpy as np
import pytest
import torch

import lbm_inputs as inp
from gpu_helpers import (gpu_initial, gpu_pre, gpu_setup, lib, oracle_run, rel_err, shear_rates, to_dev,
                         velocity_l2)
from oracle import collision, lbm
from oracle.lattice import LATTICES

pytestmark = pytest.mark.gpu

F64, F32, F16, BF16 = 0, 1, 2, 3


def _fields(shape, seed, umax=0.05):
    rng = np.random.default_rng(seed)
    rho0 = 1.0 + 0.01 * rng.standard_normal(shape)
    u0 = umax * rng.uniform(-1, 1, (3,) + shape)
    return rho0, u0


def _force(kind, shape, seed):
    if kind is None:
        return None
    if kind == "uniform":
        return np.array([2e-4, -1e-4, 5e-5])
    return inp.gaussian_force(shape, 1e-4, seed)


def _mask(kind, shape):
    nz, ny, nx = shape
    if kind is None:
        return None
    if kind == "duct":
        return inp.duct_mask(nx, ny, nz)
    solid = np.zeros(shape, dtype=bool)          # scattered obstacles + one wall
    solid[0] = True
    solid[nz // 2, ny // 2, nx // 3] = True
    solid[nz // 2, 1, 2 * nx // 3] = True
    return solid


CASES = [
    # q, precision, (nz, ny, nx), force, mask, steps
    (27, F64, (5, 6, 70), "uniform", None, 3),
    (27, F64, (6, 5, 67), "field", "walls", 3),
    (27, F64, (9, 8, 66), "uniform", "duct", 4),
    (15, F64, (5, 6, 70), "field", None, 3),
    (15, F64, (6, 5, 67), "uniform", "walls", 3),
    (27, F32, (5, 6, 70), "field", None, 3),
    (27, F32, (9, 8, 66), "uniform", "duct", 3),
    (15, F32, (5, 6, 70), "field", "walls", 3),
    # degenerate lattices: every neighbour is the node itself or its mirror
    (27, F64, (1, 1, 1), "uniform", None, 2),
    (27, F64, (2, 3, 1), "field", None, 2),
    (15, F64, (1, 1, 5), "field", None, 2),
    (27, F32, (3, 1, 129), None, None, 2),
    # per-unit-mass factorized attractors (rho varies by ~1% here)
    (27, F64, (6, 5, 67), "field", "walls", 3, True),
    (15, F64, (5, 6, 70), "uniform", "walls", 3, True),
    (27, F32, (5, 6, 70), "field", None, 3, True),
]


def _ids(c):
    pm = "-per_mass" if len(c) > 6 and c[6] else ""
    return f"q{c[0]}-p{c[1]}-{'x'.join(map(str, c[2]))}-{c[3]}-{c[4]}-n{c[5]}{pm}"


@pytest.mark.parametrize("case", CASES, ids=[_ids(c) for c in CASES])
def test_forward_matches_oracle(case):
    q, prec, shape, fkind, mkind, steps = case[:6]
    per_mass = len(case) > 6 and case[6]
    print(f"case {_ids(case)}", flush=True)
    rng = np.random.default_rng(7)
    omega = list(rng.uniform(0.7, 1.9, q - 4))
    F = _force(fkind, shape, 3)
    solid = _mask(mkind, shape)
    rho0, u0 = _fields(shape, 5)
    fluid = None if solid is None else ~solid
    sim = gpu_setup(q, shape, prec, omega, F, solid, per_mass)
    f_post, f_pre0 = gpu_initial(sim, rho0, u0)
    states = oracle_run(q, rho0, u0, F, omega, steps, solid, per_mass)
    tol = 1e-12 if prec == F64 else None
    # initial pre-collision state, from the kernel that builds it and from the
    # post-collision buffer through the pull
    for got in (f_pre0.double().cpu().numpy(), gpu_pre(sim, f_post)):
        if prec == F64:
            assert rel_err(got, states[0], fluid) < tol
        else:
            assert _absdiff(got, states[0], fluid) < 5e-7      # FP32 rounding of the init
    other = sim.populations()
    for n in range(1, steps + 1):
        sim.step(f_post, other)
        f_post, other = other, f_post
        got = gpu_pre(sim, f_post)
        want = states[n]
        if prec == F64:
            assert rel_err(got, want, fluid) < tol, (n, rel_err(got, want, fluid))
        else:
            assert _absdiff(got, want, fluid) < 2e-6, (n, _absdiff(got, want, fluid))
    lat = LATTICES[q]
    Fo = np.zeros(3) if F is None else F
    rho_o, u_o = lbm.macroscopic_fields(lat, states[-1], Fo, solid)
    rho_g, u_g = sim.macroscopic(f_post)
    rho_g = rho_g.double().cpu().numpy()
    u_g = u_g.double().cpu().numpy()
    if prec == F64:
        assert rel_err(rho_g, rho_o, fluid) < 1e-12
        assert velocity_l2(u_g, u_o, fluid) < 1e-11
    else:
        assert velocity_l2(u_g, u_o, fluid) < 2e-5
    tot = np.array(sim.totals(f_post))
    tot_o = lbm.totals(lat, states[-1], Fo, solid)
    nodes = int(np.prod(shape))
    assert np.abs(tot - tot_o).max() < (1e-12 if prec == F64 else 1e-6) * nodes


def _absdiff(a, b, fluid):
    d = a - b
    if fluid is not None:
        d = d[:, fluid]
    return float(np.abs(d).max())


def _ulp16(x, fmt):
    a = np.abs(x)
    a = np.where(a == 0, 1e-30, a)
    e = np.floor(np.log2(a))
    mant = 10 if fmt == F16 else 7
    sub = -14 if fmt == F16 else -126
    return 2.0 ** (np.maximum(e, sub) - mant)


@pytest.mark.parametrize("q", [27, 15])
@pytest.mark.parametrize("prec", [F16, BF16])
@pytest.mark.parametrize("shape,mkind", [((6, 7, 68), None), ((5, 3, 70), "walls")])
def test_deviation_storage_one_step(q, prec, shape, mkind):
    # (5, 3, 70): an odd number of rows, for the launch that updates two rows
    # per thread
    print(f"case dev16 q{q} p{prec} {shape} {mkind}", flush=True)
    rng = np.random.default_rng(11)
    omega = list(rng.uniform(0.7, 1.9, q - 4))
    F = inp.gaussian_force(shape, 1e-4, 2)
    rho0, u0 = _fields(shape, 9)
    solid = _mask(mkind, shape)
    sim = gpu_setup(q, shape, prec, omega, F, solid)
    f_post, _ = gpu_initial(sim, rho0, u0)
    pre = gpu_pre(sim, f_post)                       # decoded stored state
    other = sim.populations()
    sim.step(f_post, other)
    got = gpu_pre(sim, other)
    lat = LATTICES[q]
    want = lbm.step(lat, pre, F, omega, solid)       # oracle from the same decoded input
    w = collision.equilibrium(lat, np.array(1.0), np.zeros(3))
    dev = want - w[:, None, None, None]
    bound = 0.5 * _ulp16(dev, prec) + 2e-6
    fluid = np.ones(shape, bool) if solid is None else ~solid
    assert (np.abs(got - want)[:, fluid] <= bound[:, fluid]).all(), np.abs(got - want)[:, fluid].max()


def test_fp32_taylor_green_velocity_l2():
    # Taylor-Green of the 32^3 configuration, 10 steps, FP32 GPU vs FP64 oracle.
    print("case tg32 f32", flush=True)
    n, steps = 32, 10
    q = 27
    omega = shear_rates(q, 1.6)
    u0 = inp.taylor_green(n, 0.02)
    rho0 = np.ones((n, n, n))
    F = np.array([1e-6, 0, 0])
    sim = gpu_setup(q, (n, n, n), F32, omega, F)
    f_post, _ = gpu_initial(sim, rho0, u0)
    f_last = sim.run(f_post, sim.populations(), steps)
    _, u_g = sim.macroscopic(f_last)
    states = oracle_run(q, rho0, u0, F, omega, steps)
    _, u_o = lbm.macroscopic_fields(LATTICES[q], states[-1], F)
    assert velocity_l2(u_g.double().cpu().numpy(), u_o) < 2e-5


@pytest.mark.parametrize("q,prec,shape,force,mask", [
    (27, F32, (6, 5, 300), "field", "walls"),
    (27, F64, (5, 6, 70), "uniform", None),
    (15, F32, (6, 5, 67), "field", None),
    (15, BF16, (5, 6, 70), "uniform", "walls"),
    (27, F16, (3, 1, 129), None, None),
])
def test_step_totals_fused(q, prec, shape, force, mask):
    # The fused FP64 totals of a step's input state equal cmlbm_totals of the
    # same buffer (same populations, different summation order), and the step
    # output equals the plain step's bit for bit.
    print(f"case step_totals q{q} p{prec} {shape}", flush=True)
    rho0, u0 = _fields(shape, 17)
    F = _force(force, shape, 5)
    solid = _mask(mask, shape)
    sim = gpu_setup(q, shape, prec, shear_rates(q, 1.7), F, solid)
    f_post, _ = gpu_initial(sim, rho0, u0)
    f_post = sim.run(f_post, sim.populations(), 2)
    want = np.array(sim.totals(f_post))
    out_a, out_b = sim.populations().zero_(), sim.populations().zero_()   # solid nodes are not written
    tot = torch.zeros(4, dtype=torch.float64, device="cuda")
    sim.step(f_post, out_a, totals=tot)
    sim.step(f_post, out_b)
    got = tot.cpu().numpy()
    n = int(np.prod(shape))
    assert np.abs(got - want).max() <= 1e-13 * n, (got, want)
    assert torch.equal(out_a.view(torch.uint8), out_b.view(torch.uint8))
    with pytest.raises(lib().CmlbmError):
        sim.step(f_post, out_a, totals=torch.zeros(4, dtype=torch.float32, device="cuda"))


def test_run_ping_pong_and_errors():
    cm = lib()
    sim = gpu_setup(27, (4, 4, 64), F32, shear_rates(27, 1.5))
    f_post, _ = gpu_initial(sim, np.ones((4, 4, 64)), np.zeros((3, 4, 4, 64)))
    b = sim.populations()
    assert sim.run(f_post, b, 3) is b
    assert sim.run(f_post, b, 2) is f_post
    before = f_post.clone()
    assert sim.run(f_post, b, 0) is f_post                # zero steps: nothing happens
    assert torch.equal(before, f_post)
    with pytest.raises(cm.CmlbmError):
        sim.run(f_post, b, -1)
    with pytest.raises(cm.CmlbmError):
        sim.step(f_post, f_post)                        # aliasing is rejected
    with pytest.raises(cm.CmlbmError):
        sim.set_rates([2.5] * 23)                      # outside (0, 2)
    with pytest.raises(cm.CmlbmError):
        sim.set_rates([1.0] * 11)                      # wrong count
    with pytest.raises(cm.CmlbmError) as e:
        sim.adjoint_step(f_post, f_post, b, b, b)             # aliasing is rejected
    assert e.value.code == -1
    assert cm.load_library().cmlbm_set_attractor_per_mass(sim.h, 2) == -1   # only 0 or 1


def test_misaligned_buffers_rejected():
    # Pointers not aligned to their element size are refused before any launch.
    # The shifted pointers lie inside a buffer with 16 spare elements, so even a
    # launch would stay in bounds; the buffer staying zero shows none happened.
    print("case misaligned", flush=True)
    L = lib().load_library()
    sim = gpu_setup(27, (4, 4, 64), F32, shear_rates(27, 1.5))
    f_post, _ = gpu_initial(sim, np.ones((4, 4, 64)), np.zeros((3, 4, 4, 64)))
    big = torch.zeros(f_post.numel() + 16, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    base = big.data_ptr()
    assert L.cmlbm_step(sim.h, f_post.data_ptr(), base + 2, st) == -1
    assert b"aligned" in L.cmlbm_last_error(sim.h)
    assert L.cmlbm_step(sim.h, base + 2, base + 32, st) == -1
    assert L.cmlbm_step_inplace(sim.h, base + 1, 0, st) == -1
    assert L.cmlbm_set_force_field(sim.h, base + 2) == -1
    assert L.cmlbm_macroscopic(sim.h, f_post.data_ptr(), base + 2, base + 512, st) == -1
    assert L.cmlbm_step_totals(sim.h, f_post.data_ptr(), base, base + 4, st) == -1   # FP64 totals on 4 B
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(big)) == 0
    # The binding checks each tensor's device, dtype and size before the call.
    short = torch.zeros(f_post.numel() - 1, dtype=torch.float32, device="cuda")
    for bad in (short, big.double(), big.cpu()):
        with pytest.raises(lib().CmlbmError):
            sim.step(f_post, bad)
    with pytest.raises(lib().CmlbmError):
        sim.set_force(torch.zeros((3, 4, 4, 63), device="cuda"))
    with pytest.raises(lib().CmlbmError):
        sim.macroscopic_pre(short)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(short)) == 0


@pytest.mark.parametrize("q,prec,duct", [(27, F32, False), (15, F32, False), (27, F16, False), (15, BF16, False),
                                          (27, F32, True)])
def test_full_size_sampled_nodes(q, prec, duct):
    # The benchmark configuration: 512^3 FP32 D3Q27 (and D3Q15) with the
    # Kolmogorov force field F_x = 1e-6 sin(2 pi 4 y / 512), shear rate 1.9,
    # the same lattice with 16-bit deviation storage, and (duct) inside the
    # square duct of the benchmark's wall-bounded measurement.  One step from a
    # perturbed state; the oracle collides 4096 sampled fluid nodes from the
    # pre-collision populations the GPU pulled (decoded, for 16-bit storage).
    # With walls the pulled populations themselves are checked first, bit for
    # bit, against the stored state streamed by the half-way bounce-back rule.
    print(f"case full512 q{q} p{prec} duct={duct}", flush=True)
    n = 512
    lat = LATTICES[q]
    solid = inp.duct_mask(n, n, n) if duct else None
    sim = gpu_setup(q, (n, n, n), prec, shear_rates(q, 1.9), None, solid)
    F = torch.from_numpy(inp.kolmogorov_force(n)).to("cuda", torch.float32)
    sim.set_force(F)
    rho0 = torch.ones((n, n, n), device="cuda", dtype=torch.float32)
    g = torch.Generator(device="cuda").manual_seed(1)
    u0 = 0.03 * (torch.rand((3, n, n, n), device="cuda", generator=g) - 0.5)
    if duct:
        u0[:, torch.from_numpy(solid).cuda()] = 0.0
    f_post, f_pre = sim.init_equilibrium(rho0, u0)
    del u0, rho0
    out = sim.populations()
    sim.step(f_post, out)
    pre = sim.gather(f_post, out=f_pre)
    rng = np.random.default_rng(3)
    if duct:   # fluid nodes, half of them beside a wall
        z, y, xx = rng.integers(1, n - 1, 4096), rng.integers(1, n - 1, 4096), rng.integers(0, n, 4096)
        z[:2048:2] = 1 + (n - 3) * rng.integers(0, 2, 1024)
        y[1:2048:2] = 1 + (n - 3) * rng.integers(0, 2, 1024)
        idx = z * n * n + y * n + xx
    else:
        idx = rng.integers(0, n**3, 4096)
        idx[:4] = [0, n - 1, n * n - 1, n**3 - 1]          # corners of the periodic box
    idx_t = torch.from_numpy(idx).to("cuda")
    f_in = pre.reshape(q, -1)[:, idx_t].double().cpu().numpy().T
    if duct:
        zz, yy, xs = idx // (n * n), (idx // n) % n, idx % n
        sflat = solid.reshape(-1)
        assert not sflat[idx].any()
        stored = sim.export_populations(f_post).reshape(q, -1)
        for a in range(q):
            ex, ey, ez = (int(c) for c in lat.E[a])
            src = ((zz - ez) % n) * n * n + ((yy - ey) % n) * n + (xs - ex) % n
            fwd = stored[a, torch.from_numpy(src).to("cuda")].double().cpu().numpy()
            back = stored[lat.opp[a], idx_t].double().cpu().numpy()
            assert np.array_equal(f_in[:, a], np.where(sflat[src], back, fwd)), a
        del stored
        torch.cuda.empty_cache()
    post = sim.export_populations(out, out=f_pre)          # pre no longer needed past this point
    f_gpu = post.reshape(q, -1)[:, idx_t].double().cpu().numpy().T
    Fs = F.reshape(3, -1)[:, idx_t].double().cpu().numpy().T
    want = collision.collide(lat, f_in, Fs, shear_rates(q, 1.9))
    if prec == F32:
        assert np.abs(f_gpu - want).max() < 2e-6
    else:   # the stored deviation f - w_a rounded to 16 bits: half an ulp of it, plus FP32 arithmetic
        w = collision.equilibrium(LATTICES[q], np.array(1.0), np.zeros(3))
        bound = 0.5 * _ulp16(want - w[None, :], prec) + 2e-6
        assert (np.abs(f_gpu - want) <= bound).all(), np.abs(f_gpu - want).max()


def test_duct_128_transient_closed_form():
    # 128^3 D3Q27 FP32 duct: walls y, z in {0, 127}, F_x = 1e-6, omega 1.8,
    # 20000 steps from rest vs the closed-form start-up series (same momentum
    # equation the paper's steady duct profile solves).
    print("case duct128", flush=True)
    n, steps, omega, Fx = 128, 20000, 1.8, 1e-6
    solid = inp.duct_mask(n, n, n)
    sim = gpu_setup(27, (n, n, n), F32, shear_rates(27, omega), np.array([Fx, 0, 0]), solid)
    f_post, _ = gpu_initial(sim, np.ones((n, n, n)), np.zeros((3, n, n, n)))
    f_last = sim.run(f_post, sim.populations(), steps)
    _, u = sim.macroscopic(f_last)
    ux = u[0, 1:-1, 1:-1, n // 2].double().cpu().numpy()
    from test_oracle_flows import duct_startup, nu_of
    c = np.arange(1, n - 1) - (n - 1) / 2
    Z, Y = np.meshgrid(c, c, indexing="ij")
    ua = duct_startup(Y, Z, (n - 2) / 2, Fx, nu_of(omega), steps, nterms=60)
    err = np.linalg.norm(ux - ua) / np.linalg.norm(ua)
    print(f"duct128 relative L2 {err:.3e}  center {ux[62, 62]:.6e} vs {ua[62, 62]:.6e}", flush=True)
    assert err < 1e-2


def test_duct_128_steady_series():
    # The same duct run to steady state: 4e5 steps, the slowest start-up mode
    # (rate 2 nu (pi/2a)^2 = 2.3e-5 per step) is down to e^-9.2; against the
    # steady Fourier series (Eq. ductFourier) and its centre value
    # 0.2946854 a^2 F / (rho nu).
    print("case duct128 steady", flush=True)
    n, steps, omega, Fx = 128, 400000, 1.8, 1e-6
    solid = inp.duct_mask(n, n, n)
    sim = gpu_setup(27, (n, n, n), F32, shear_rates(27, omega), np.array([Fx, 0, 0]), solid)
    f_post, _ = gpu_initial(sim, np.ones((n, n, n)), np.zeros((3, n, n, n)))
    f_last = sim.run(f_post, sim.populations(), steps)
    _, u = sim.macroscopic(f_last)
    u = u.double().cpu().numpy()
    ux = u[0, 1:-1, 1:-1, n // 2]
    from test_oracle_flows import duct_steady_paper, nu_of
    a, nu = (n - 2) / 2, nu_of(omega)
    c = np.arange(1, n - 1) - (n - 1) / 2
    Z, Y = np.meshgrid(c, c, indexing="ij")
    ua = duct_steady_paper(Y, Z, a, Fx, nu)
    err = np.linalg.norm(ux - ua) / np.linalg.norm(ua)
    centre = 0.25 * (ux[62, 62] + ux[62, 63] + ux[63, 62] + ux[63, 63])   # the centre lies between nodes
    print(f"duct128 steady: relative L2 {err:.3e}; centre {centre:.6e} vs series "
          f"{duct_steady_paper(0.0, 0.0, a, Fx, nu):.6e} (0.2946854 a^2 F/nu = {0.2946854 * a * a * Fx / nu:.6e})",
          flush=True)
    assert err < 2e-3                                                       # measured 1.8e-4
    assert abs(centre / (0.2946854 * a * a * Fx / nu) - 1) < 2e-3           # measured 3.3e-4
    assert np.abs(u[1:, 1:-1, 1:-1]).max() < 1e-3 * np.abs(ux).max()        # no cross flow


@pytest.mark.parametrize("prec", [F64, F32, F16, BF16])
@pytest.mark.parametrize("q,nx", [(27, 130), (15, 64), (27, 5)])
def test_population_buffer_layout(prec, q, nx):
    # The documented blocked layout: index(a, r, x) = r*nx*q + b*64*q + a*len + (x - 64 b),
    # b = x // 64, len = min(64, nx - 64 b); export/import round trip.
    print(f"case layout q{q} nx{nx} p{prec}", flush=True)
    cm = lib()
    ny, nz = 3, 2
    sim = cm.Sim(q, nx, ny, nz, prec)
    rng = np.random.default_rng(1)
    lat = LATTICES[q]
    w = collision.equilibrium(lat, np.array(1.0), np.zeros(3))
    soa = w[:, None, None, None] + 0.01 * rng.standard_normal((q, nz, ny, nx))
    buf = sim.import_populations(torch.from_numpy(soa))
    raw = buf.reshape(-1).double().cpu().numpy()
    for a, z, y, x in [(0, 0, 0, 0), (q - 1, 1, 2, nx - 1), (q // 2, 1, 0, min(70, nx - 1)), (3, 0, 1, nx // 2)]:
        r = z * ny + y
        b = x // 64
        ln = min(64, nx - 64 * b)
        idx = r * nx * q + b * 64 * q + a * ln + (x - 64 * b)
        stored = raw[idx] + (w[a] if prec in (F16, BF16) else 0.0)
        assert abs(stored - soa[a, z, y, x]) <= (1e-15 if prec == F64 else 2e-7 if prec == F32 else 3e-4)
    back = sim.export_populations(buf).double().cpu().numpy()
    if prec in (F16, BF16):
        tol = 0.5 * _ulp16(soa - w[:, None, None, None], prec) + 1e-7
    else:
        tol = {F64: 0.0, F32: 1e-7}[prec]
    assert (np.abs(back - soa) <= tol).all()


@pytest.mark.parametrize("q,prec", [(27, 2), (15, 2), (27, 3), (15, 3)])
def test_deviation_decode_every_bit_pattern(q, prec):
    # Every finite 16-bit pattern (FP16 subnormals included) stored in a
    # population buffer reads back, through the kernels' decode, as w_a + value
    # rounded once in FP32.  nx = 64: one 64-node block per row, so the buffer
    # is [row][a][x].
    print(f"case decode-every-pattern q{q} p{prec}", flush=True)
    from paper_1202_6081_amd import cmlbm
    nx, ny, nz = 64, 16, 8
    sim = cmlbm.Sim(q, nx, ny, nz, prec)
    bits = np.arange(65536, dtype=np.uint16)
    if prec == 2:
        finite = ((bits >> 10) & 0x1F) != 0x1F
    else:
        finite = ((bits >> 7) & 0xFF) != 0xFF
    pat = bits[finite]
    total = q * nx * ny * nz
    assert total >= pat.size
    flat = np.resize(pat, total)
    buf = sim.populations()
    buf.view(torch.int16).reshape(-1).copy_(torch.from_numpy(flat.view(np.int16)))
    soa = sim.export_populations(buf).cpu().numpy()           # [q][nz][ny][nx], float32
    if prec == 2:
        vals = flat.view(np.float16).astype(np.float32)
    else:
        vals = (flat.astype(np.uint32) << 16).view(np.float32)
    vals = vals.reshape(nz * ny, q, nx)
    # rest weights by the number of nonzero velocity components
    nz_comp = np.abs(LATTICES[q].E).sum(axis=1)
    table = {27: [8 / 27, 2 / 27, 1 / 54, 1 / 216], 15: [2 / 9, 1 / 9, None, 1 / 72]}[q]
    w = np.array([table[k] for k in nz_comp], dtype=np.float64)
    want = (w.astype(np.float32)[None, :, None] + vals).astype(np.float32)       # one FP32 rounding
    got = np.transpose(soa.reshape(q, nz * ny, nx), (1, 0, 2))
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
