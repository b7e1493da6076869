"""GPU tests of the stability check cmlbm_check_finite, through the C ABI.

The count it returns has a plain definition: the stored populations of fluid
nodes that are NaN or +-Inf.  The tests plant such values at known slots
(cmlbm_import_populations of an SoA array) and compare the count with the one
numpy takes of the same array, over fluid nodes only; a random mask and a row
length of 130 (sub-blocks of 64, 64 and 2 nodes) make a slot-to-node mistake
change the count.  One step of a periodic lattice spreads a single planted NaN
to exactly the Q populations of the node that pulls it, which also checks that
the pull reads that slot and no other.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import gpu_setup, lib, shear_rates, to_dev
from oracle.lattice import LATTICES

pytestmark = pytest.mark.gpu

F64, F32, F16, BF16 = 0, 1, 2, 3
PRECS = [F64, F32, F16, BF16]
SHAPE = (5, 4, 130)   # nz, ny, nx


def _state(sim, shape, seed):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.01 * rng.standard_normal(shape)
    u = 0.05 * rng.uniform(-1, 1, (3,) + shape)
    f_post, _ = sim.init_equilibrium(to_dev(rho, sim.real), to_dev(u, sim.real))
    return sim.export_populations(f_post).double().cpu().numpy()


def _plant(f, rng, values):
    """Write `values` at distinct random (a, z, y, x) slots; returns the slots."""
    flat = rng.choice(f.size, size=len(values), replace=False)
    slots = [np.unravel_index(i, f.shape) for i in flat]
    for s, v in zip(slots, values):
        f[s] = v
    return slots


@pytest.mark.parametrize("q", [27, 15])
@pytest.mark.parametrize("prec", PRECS)
def test_clean_state_counts_zero(q, prec):
    sim = gpu_setup(q, SHAPE, prec, shear_rates(q, 1.6))
    f = _state(sim, SHAPE, 1)
    assert sim.check_finite(sim.import_populations(torch.from_numpy(f))) == 0


@pytest.mark.parametrize("q", [27, 15])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("masked", [False, True])
def test_planted_values_counted_at_fluid_nodes(q, prec, masked):
    rng = np.random.default_rng(100 + q + 10 * prec + masked)
    solid = rng.random(SHAPE) < 0.3 if masked else None
    sim = gpu_setup(q, SHAPE, prec, shear_rates(q, 1.6), solid=solid)
    f = _state(sim, SHAPE, 2)
    values = [np.nan, np.inf, -np.inf] * 12
    slots = _plant(f, rng, values)
    buf = sim.import_populations(torch.from_numpy(f))
    fluid = [s for s in slots if solid is None or not solid[s[1:]]]
    want = len(fluid)
    if masked:
        assert 0 < want < len(slots), "the draw must hit fluid and solid nodes"
    assert sim.check_finite(buf) == want
    # the same count numpy takes of what the buffer holds
    back = sim.export_populations(buf).double().cpu().numpy()
    bad = ~np.isfinite(back)
    if solid is not None:
        bad &= ~solid[None]
    assert int(bad.sum()) == want


def test_f16_overflow_counts():
    """FP16 deviation storage rounds |fbar_a - w_a| > 65504 to +-Inf."""
    q = 27
    sim = gpu_setup(q, SHAPE, F16, shear_rates(q, 1.6))
    f = _state(sim, SHAPE, 3)
    rng = np.random.default_rng(7)
    _plant(f, rng, [7.0e4, -7.0e4, 6.0e4])   # the last one still fits
    assert sim.check_finite(sim.import_populations(torch.from_numpy(f))) == 2
    sim_bf = gpu_setup(q, SHAPE, BF16, shear_rates(q, 1.6))
    assert sim_bf.check_finite(sim_bf.import_populations(torch.from_numpy(f))) == 0


@pytest.mark.parametrize("q", [27, 15])
@pytest.mark.parametrize("prec", PRECS)
def test_one_nan_spreads_to_one_node(q, prec):
    """A NaN post-collision population a of node n is pulled by n + e_a only,
    whose collision turns all its Q populations NaN."""
    lat = LATTICES[q]
    sim = gpu_setup(q, SHAPE, prec, shear_rates(q, 1.6), F=[1e-4, 0, 0])
    f = _state(sim, SHAPE, 4)
    rng = np.random.default_rng(11 + q + prec)
    for a in [0, int(rng.integers(1, q)), int(rng.integers(1, q))]:
        g = f.copy()
        n = tuple(int(rng.integers(0, m)) for m in SHAPE)
        g[(a,) + n] = np.nan
        f_in = sim.import_populations(torch.from_numpy(g))
        f_out = sim.populations()
        assert sim.check_finite(f_in) == 1
        sim.step(f_in, f_out)
        assert sim.check_finite(f_out) == q
        pre = sim.export_populations(f_out).double().cpu().numpy()
        nz, ny, nx = SHAPE
        ex, ey, ez = (int(c) for c in lat.E[a])
        t = ((n[0] + ez) % nz, (n[1] + ey) % ny, (n[2] + ex) % nx)
        assert np.isnan(pre[(slice(None),) + t]).all()


@pytest.mark.parametrize("q", [27, 15])
def test_inplace_buffer_both_phases(q):
    """In-place buffer: one NaN in phase 0 at node n; the parity-0 step
    collides n from its own slots and writes all Q results back there."""
    sim = gpu_setup(q, SHAPE, F32, shear_rates(q, 1.6))
    f = _state(sim, SHAPE, 5)
    f[(3, 2, 1, 65)] = np.nan
    buf = sim.import_populations(torch.from_numpy(f))
    assert sim.check_finite(buf) == 1
    sim.step_inplace(buf, 0)
    assert sim.check_finite(buf) == q


def test_errors():
    cm = lib()
    sim = gpu_setup(27, SHAPE, F32, shear_rates(27, 1.6))
    with pytest.raises(cm.CmlbmError):
        cm.cmlbm_check_finite(sim.h, None)
    with pytest.raises(cm.CmlbmError):
        sim.check_finite(torch.empty(3, device="cuda", dtype=torch.float32))


def test_full_size_buffer_64bit_offsets():
    """560^3 D3Q27 FP32 buffer (rows of 8 full sub-blocks and one of 48
    nodes): 4.7e9 stored values, more than 2^32, with planted values at the
    first and last slots and on both sides of slot 2^32 (unmasked, so the
    count does not depend on where a slot's node is)."""
    n = 560
    sim = lib().Sim(27, n, n, n, F32)
    buf = sim.populations()
    flat = buf.view(-1)
    flat.fill_(0.03)
    assert sim.check_finite(buf) == 0
    for i, v in ((0, float("nan")), (flat.numel() - 1, float("inf")), (1 << 32, float("-inf")),
                 ((1 << 32) - 1, float("nan"))):
        flat[i] = v
    assert sim.check_finite(buf) == 4
    del flat, buf
    sim.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("q", [27, 15])
@pytest.mark.parametrize("prec", PRECS)
def test_one_nan_through_the_scatter_phase(q, prec):
    """The in-place scatter phase (parity 1) on a 300-node row (four full
    64-node sub-blocks and one of 44; row segments of 256): a NaN in slot s of
    node n is read by t = n - e_s alone, whose collision turns its Q results
    NaN, and those are written to slot b of t + e_b, one slot each: after the
    step exactly the Q values fbar_b(t + e_b) of the exported state are NaN.
    The nodes t sit on wavefront and row-segment edges, where the 16-bit
    scatter exchanges values across lanes and through LDS."""
    lat = LATTICES[q]
    shape = (3, 4, 300)
    nz, ny, nx = shape
    sim = gpu_setup(q, shape, prec, shear_rates(q, 1.6), F=[1e-4, 0, 0])
    f = _state(sim, shape, 6)
    rng = np.random.default_rng(21 + q + prec)
    for tx in (0, 63, 64, 127, 255, 256, 257, nx - 1):
        tz, ty = int(rng.integers(0, nz)), int(rng.integers(0, ny))
        s = int(rng.integers(0, q))
        ex, ey, ez = (int(c) for c in lat.E[s])
        n = ((tz + ez) % nz, (ty + ey) % ny, (tx + ex) % nx)     # t = n - e_s
        g = f.copy()
        g[(s,) + n] = np.nan
        buf = sim.import_populations(torch.from_numpy(g))
        assert sim.check_finite(buf) == 1
        sim.step_inplace(buf, 1)
        assert sim.check_finite(buf) == q, (tx, s)
        bad = np.isnan(sim.export_populations(buf).double().cpu().numpy())
        want = np.zeros_like(bad)
        for b in range(q):
            bx, by, bz = (int(c) for c in lat.E[b])
            want[b, (tz + bz) % nz, (ty + by) % ny, (tx + bx) % nx] = True
        assert np.array_equal(bad, want), (tx, s)
