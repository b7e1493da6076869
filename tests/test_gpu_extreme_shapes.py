"""GPU parity on lattice shapes at the limits the library accepts.

* The longest row: nx = 65535, the largest dimension per axis.  A row holds
  1023 full 64-node sub-blocks and one of 63 nodes, the step cuts it into 256
  row segments, and its FP64 populations span 14 MB, all addressed by 32-bit
  offsets inside the row.
* A million 3-node rows: one ragged sub-block per row, 2^20 row segments, and
  more lanes idle than busy.
* Both shapes with random walls (a fifth of the nodes solid): the masked pull,
  which reads its neighbours' mask bytes in one round before its population
  loads, on ragged rows.

One step from a perturbed state (Eq. cascadedstreaming1, then Eq.
cascadedcollision1): the pulled pre-collision populations must equal the
stored state streamed periodically, bit for bit, over the whole lattice (with
walls, the half-way bounce-back of Sec. 9 on links from solid nodes); the
oracle then collides sampled nodes (row ends, sub-block and segment edges,
random nodes) from those populations: 1e-12 relative in FP64, 2e-6 absolute in
FP32.  Two steps on one buffer in place must give the two-buffer run's
populations bit for bit.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import gpu_setup, shear_rates, to_dev
from oracle import collision
from oracle.lattice import LATTICES

pytestmark = pytest.mark.gpu

F64, F32 = 0, 1

CASES = [
    # q, precision, (nz, ny, nx), force, fraction of solid nodes (random walls)
    (27, F64, (2, 3, 65535), "field", 0.0),
    (15, F32, (3, 2, 65535), "uniform", 0.0),
    (27, F32, (1024, 1024, 3), "field", 0.0),
    (27, F32, (3, 4, 65535), "field", 0.2),
    (15, F64, (512, 512, 3), "uniform", 0.2),
]


def _ids(c):
    walls = f"-solid{c[4]}" if len(c) > 4 and c[4] else ""
    return f"q{c[0]}-p{c[1]}-{'x'.join(map(str, c[2]))}-{c[3]}{walls}"


def _sample(shape, rng):
    """Flat node indices: the row ends and the sub-block and row-segment
    edges of the first, the last and 64 random rows, plus 1024 random nodes."""
    nz, ny, nx = shape
    rows = ny * nz
    xs = sorted({x for x in (0, 1, 62, 63, 64, 65, 255, 256, nx - 65, nx - 64, nx - 63, nx - 2, nx - 1)
                 if 0 <= x < nx})
    pick_rows = np.unique(np.concatenate([[0, rows - 1], rng.integers(0, rows, 64)]))
    idx = [r * nx + x for r in pick_rows for x in xs]
    idx += list(rng.integers(0, nx * rows, 1024))
    return np.unique(np.array(idx, dtype=np.int64))


@pytest.mark.parametrize("case", CASES, ids=[_ids(c) for c in CASES])
def test_extreme_shape_step(case):
    q, prec, shape, fkind, frac = case
    print(f"case extreme {_ids(case)}", flush=True)
    lat = LATTICES[q]
    rng = np.random.default_rng(5)
    F = (np.array([3e-5, -1e-5, 2e-5]) if fkind == "uniform"
         else 2e-5 * rng.standard_normal((3,) + shape))
    rates = shear_rates(q, 1.9)
    solid = rng.random(shape) < frac if frac else None
    sim = gpu_setup(q, shape, prec, rates, F, solid)
    rho0 = 1.0 + 0.01 * rng.standard_normal(shape)
    u0 = 0.04 * (rng.random((3,) + shape) - 0.5)
    if solid is not None:
        u0[:, solid] = 0.0
    f_post, _ = sim.init_equilibrium(to_dev(rho0, sim.real), to_dev(u0, sim.real))

    # streaming: the gathered pre-collision state is the stored state moved
    # by e_a, periodic in every axis; with walls, a link from a solid node
    # takes the node's own opposite population (half-way bounce-back), and
    # solid nodes read zero
    stored = sim.export_populations(f_post).cpu().numpy()
    pre = sim.gather(f_post).cpu().numpy()
    for a in range(q):
        ex, ey, ez = (int(c) for c in lat.E[a])
        want = np.roll(stored[a], shift=(ez, ey, ex), axis=(0, 1, 2))
        if solid is not None:
            from_solid = np.roll(solid, shift=(ez, ey, ex), axis=(0, 1, 2))
            want = np.where(from_solid, stored[lat.opp[a]], want)
            want[solid] = 0.0
        assert np.array_equal(pre[a], want), a
    del stored

    # collision of sampled nodes against the oracle
    out = sim.populations()
    sim.step(f_post, out)
    post = sim.export_populations(out).cpu().numpy().reshape(q, -1)
    idx = _sample(shape, rng)
    if solid is not None:
        idx = idx[~solid.reshape(-1)[idx]]
    f_in = pre.reshape(q, -1)[:, idx].T.astype(np.float64)
    Fs = np.broadcast_to(F, (idx.size, 3)) if fkind == "uniform" else F.reshape(3, -1)[:, idx].T
    want = collision.collide(lat, f_in, np.ascontiguousarray(Fs, dtype=np.float64), rates)
    got = post[:, idx].T.astype(np.float64)
    if prec == F64:
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    else:
        assert np.abs(got - want).max() < 2e-6
    del pre, post

    # two steps in place against two two-buffer steps
    last = sim.run(f_post, out, 2)
    two_buffer = sim.gather(last).cpu().numpy()
    g = sim.init_equilibrium_inplace(to_dev(rho0, sim.real), to_dev(u0, sim.real))
    sim.run_inplace(g, 2)
    in_place = sim.export_populations(g).cpu().numpy()
    assert np.array_equal(two_buffer, in_place)
    sim.close()
    torch.cuda.empty_cache()


ADJ_CASES = [(27, F64, (2, 3, 65535)), (15, F64, (3, 2, 65535)), (27, F32, (1024, 1024, 3))]


@pytest.mark.parametrize("case", ADJ_CASES, ids=[_ids(c + ("field",)) for c in ADJ_CASES])
def test_extreme_shape_adjoint_step(case):
    """One adjoint step on the same shapes: at the sampled nodes, lam(x) and
    dL/dF(x) against the transposed Jacobian of the oracle's collision (complex
    step at the pre-collision state the GPU pulled) applied to the
    reverse-streamed adjoint lam_next(x + e_a)_a, periodic.  1e-10 relative in
    FP64, 1e-5 in FP32."""
    q, prec, shape = case
    print(f"case extreme adjoint {_ids(case + ('field',))}", flush=True)
    H = 1e-30
    lat = LATTICES[q]
    nz, ny, nx = shape
    rng = np.random.default_rng(6)
    F = 2e-5 * rng.standard_normal((3,) + shape)
    om = shear_rates(q, 1.9)
    sim = gpu_setup(q, shape, prec, om, F)
    rho0 = 1.0 + 0.01 * rng.standard_normal(shape)
    u0 = 0.04 * (rng.random((3,) + shape) - 0.5)
    x, _ = sim.init_equilibrium(to_dev(rho0, sim.real), to_dev(u0, sim.real))
    lam_next_h = rng.standard_normal((q,) + shape)
    lam_next = to_dev(lam_next_h, sim.real)
    lam = sim.real_populations()
    dLdF = torch.zeros((3,) + shape, dtype=torch.float64, device="cuda")
    dLdw = torch.zeros(q - 4, dtype=torch.float64, device="cuda")
    sim.adjoint_step(x, lam_next, lam, dLdF, dLdw)
    pre = sim.gather(x).cpu().numpy().reshape(q, -1)
    idx = _sample(shape, rng)
    z, y, xx = idx // (nx * ny), (idx // nx) % ny, idx % nx
    f_in = pre[:, idx].T.astype(np.float64)
    Fs = F.reshape(3, -1)[:, idx].T
    if prec == F32:   # the force as the device holds it
        Fs = Fs.astype(np.float32).astype(np.float64)
    ln = lam_next.double().cpu().numpy().reshape(q, -1)
    post = np.empty((idx.size, q))
    for a in range(q):
        ex, ey, ez = (int(c) for c in lat.E[a])
        post[:, a] = ln[a, ((z + ez) % nz) * nx * ny + ((y + ey) % ny) * nx + (xx + ex) % nx]
    got = lam.double().cpu().numpy().reshape(q, -1)[:, idx].T
    got_F = dLdF.cpu().numpy().reshape(3, -1)[:, idx].T
    fc = f_in[:, None, :] + 1j * H * np.eye(q)[None, :, :]
    Cc = collision.collide(lat, fc, np.repeat(Fs[:, None, :], q, axis=1).astype(complex), np.array(om, dtype=complex))
    want = np.einsum("na,nba->nb", post, Cc.imag / H)
    Fc = Fs[:, None, :] + 1j * H * np.eye(3)[None, :, :]
    CF = collision.collide(lat, np.repeat(f_in[:, None, :], 3, axis=1).astype(complex), Fc, np.array(om, dtype=complex))
    want_F = np.einsum("na,nca->nc", post, CF.imag / H)
    err = np.abs(got - want).max() / np.abs(want).max()
    err_F = np.abs(got_F - want_F).max() / np.abs(want_F).max()
    print(f"extreme adjoint {_ids(case + ('field',))}: lam rel err {err:.2e}, dL/dF rel err {err_F:.2e}", flush=True)
    tol = 1e-10 if prec == F64 else 1e-5
    assert err < tol and err_F < tol
    sim.close()
    torch.cuda.empty_cache()
