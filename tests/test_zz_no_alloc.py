"""The allocation-free fused-totals step against cmlbm_step_totals, through the C ABI.

cmlbm_step_totals_noalloc keeps its per-block partial sums in the library's
static device array instead of the handle's scratch; its populations and FP64
totals must equal cmlbm_step_totals' bit for bit.  Two calls in a row, the
second on a smaller lattice (a second handle on the same device, whose call
reads only what it wrote into the shared array), and a check that the device's
free memory does not move across the calls.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import gpu_setup, to_dev

pytestmark = pytest.mark.gpu


def _free_bytes():
    return torch.cuda.mem_get_info()[0]     # hipMemGetInfo of the current device


def _case(q, shape, precision, seed, solid=None):
    from paper_1202_6081_amd import cmlbm
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    F = 1e-4 * rng.standard_normal((3, nz, ny, nx))
    sim = gpu_setup(q, shape, precision, list(rng.uniform(0.6, 1.9, q - 4)), F=F, solid=solid)
    rho0 = 1 + 0.01 * rng.standard_normal(shape)
    u0 = 0.05 * rng.uniform(-1, 1, (3,) + shape)
    f_post, _ = sim.init_equilibrium(to_dev(rho0, sim.real), to_dev(u0, sim.real))
    a, b = sim.populations().zero_(), sim.populations().zero_()   # solid nodes are never written
    ta = torch.zeros(4, dtype=torch.float64, device="cuda")
    tb = torch.full((4,), -1.0, dtype=torch.float64, device="cuda")
    return cmlbm, sim, f_post, a, b, ta, tb


def _compare(cmlbm, sim, f_post, a, b, ta, tb, steps=3):
    # both entry points from the same input, step after step; the device's free
    # memory is read right around each allocation-free call
    cur = f_post
    for _ in range(steps):
        cmlbm.cmlbm_step_totals(sim.h, cur, a, ta)
        torch.cuda.synchronize()
        free0 = _free_bytes()
        cmlbm.cmlbm_step_totals_noalloc(sim.h, cur, b, tb)
        torch.cuda.synchronize()
        assert _free_bytes() == free0
        assert torch.equal(a.view(torch.uint8), b.view(torch.uint8))
        assert torch.equal(ta, tb), (ta.tolist(), tb.tolist())
        assert float(ta[0]) > 0
        f_post.copy_(a)
        cur = f_post


@pytest.mark.parametrize("q,precision", [(27, 1), (15, 0), (27, 2)])
def test_noalloc_equals_step_totals_two_calls(q, precision):
    # first call: a lattice spanning several row segments with a ragged tail;
    # second: a smaller one on a new handle (the static array still holds the
    # first call's larger partials)
    _compare(*_case(q, (6, 9, 300), precision, seed=1))
    solid = np.zeros((4, 5, 70), dtype=bool)
    solid[:, 0] = True
    _compare(*_case(q, (4, 5, 70), precision, seed=2, solid=solid))


def test_noalloc_refuses_lattices_beyond_its_scratch():
    from paper_1202_6081_amd import cmlbm
    # ceil(256/256) * 1024 * 513 = 525,312 step blocks > 2^19: refused before any launch
    sim = cmlbm.Sim(27, 256, 1024, 513, cmlbm.F32)
    dummy = torch.zeros(64, dtype=torch.float32, device="cuda")
    tot = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(cmlbm.CmlbmError) as e:
        cmlbm.cmlbm_step_totals_noalloc(sim.h, dummy, dummy[32:], tot)
    assert e.value.code == -1 and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert float(tot.abs().sum()) == 0.0
