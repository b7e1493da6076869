"""Host logic of the checkpoint-and-recompute sweeps (no GPU): a fake
simulator whose states are step counters checks that every adjoint step sees
the right forward state, in reverse order, with the predicted number of
recomputed steps and a bounded number of live buffers."""
import pytest

from paper_1202_6081_amd import autograd as ag


class _State:
    def __init__(self):
        self.t = None


class FakeSim:
    def __init__(self):
        self.steps = 0
        self.seen = []

    def populations(self):
        return _State()

    def step(self, src, dst):
        assert src is not dst and src.t is not None
        dst.t = src.t + 1
        self.steps += 1

    def adjoint_step(self, x, lam, lam_tmp, dLdF, dLdw):
        self.seen.append(x.t)


def _run(nsteps, every=None, snapshots=None, keep_x0=True):
    sim = FakeSim()
    pool = ag._Pool(sim)
    x0 = pool.get()
    x0.t = 0
    stored, last = ag.forward_sweep(sim, pool, x0, nsteps, ag.keep_positions(nsteps, every, snapshots),
                                    keep_x0=keep_x0)
    assert last.t == nsteps and sim.steps == nsteps
    assert (0 in stored) == keep_x0
    forward_buffers = pool.allocated
    if not any(last is v for v in stored.values()):
        pool.put(last)
    sim.steps = 0
    sw = ag._Sweep(sim, pool, None, None, None, None)
    rebuilt = []

    def rebuild_x0():
        b = pool.get()
        b.t = 0
        rebuilt.append(b)
        return b

    ag.backward_sweep(sw, stored, nsteps, every, snapshots, None if keep_x0 else rebuild_x0)
    assert sim.seen == list(range(nsteps - 1, -1, -1))
    assert len(rebuilt) == (0 if keep_x0 or nsteps == 0 else 1)
    sim.forward_buffers = forward_buffers
    return sim, sw, pool, stored


@pytest.mark.parametrize("nsteps,every", [(200, 20), (37, 5), (10, 10), (7, 1), (1, 3)])
def test_uniform_checkpoints(nsteps, every):
    sim, sw, pool, stored = _run(nsteps, every=every)
    assert sw.recomputed == sim.steps
    # each segment of length L replays L - 1 steps
    nseg = -(-nsteps // every)
    assert sw.recomputed == nsteps - nseg


@pytest.mark.parametrize("nsteps,s", [(100, 10), (100, 4), (50, 1), (30, 0), (12, 20), (1, 2), (2, 1)])
def test_binomial_schedule(nsteps, s):
    sim, sw, pool, stored = _run(nsteps, snapshots=s)
    assert sw.recomputed == sim.steps == ag.recompute_steps(nsteps, s)
    # live buffers: x0, at most s snapshots, two work buffers
    assert pool.allocated <= s + 3


def test_binomial_cost_closed_cases():
    assert ag._cost(1, 3)[0] == 0
    assert ag._cost(10, 0)[0] == 45
    assert ag._cost(10, 9)[0] == 9            # enough slots: one pass storing everything
    # more slots never cost more
    for n in (20, 60, 100):
        costs = [ag._cost(n, s)[0] for s in range(0, 12)]
        assert all(a >= b for a, b in zip(costs, costs[1:]))


@pytest.mark.parametrize("nsteps,s", [(100, 10), (100, 4), (50, 1), (30, 0), (12, 20), (1, 2), (2, 1)])
def test_binomial_schedule_rebuilding_x0(nsteps, s):
    """x(0) released after the first forward step and rebuilt once for the
    first interval: the same adjoint order and recompute count, and the
    forward pass holds one buffer fewer."""
    sim, sw, pool, stored = _run(nsteps, snapshots=s, keep_x0=False)
    assert sw.recomputed == sim.steps == ag.recompute_steps(nsteps, s)
    kept = _run(nsteps, snapshots=s)[0]
    if nsteps > 1 and s > 0:
        assert sim.forward_buffers == kept.forward_buffers - 1
    assert pool.allocated <= s + 3


@pytest.mark.parametrize("nsteps,every", [(200, 20), (37, 5), (10, 10), (7, 1), (1, 3)])
def test_uniform_checkpoints_rebuilding_x0(nsteps, every):
    sim, sw, pool, stored = _run(nsteps, every=every, keep_x0=False)
    assert sw.recomputed == sim.steps == nsteps - (-(-nsteps // every))


def test_binomial_cost_against_the_recursion_and_closed_form():
    # The schedule's costs and splits use Griewank and Walther's closed form for
    # the optimal recompute count; check it against the defining recursion,
    # evaluated here by brute force over every split.
    import functools

    @functools.lru_cache(maxsize=None)
    def rec(n, s):
        if n <= 1:
            return 0
        if s == 0:
            return n * (n - 1) // 2
        return min(m + rec(n - m, s - 1) + rec(m, s) for m in range(1, n))

    for s in range(0, 10):
        for n in range(1, 160):
            assert ag._min_recompute(n, s) == rec(n, s) == ag._cost(n, s)[0], (n, s)
    # two values worked by hand from the closed form: 10 steps with 2
    # checkpoints -> 3*10 - C(5, 3) = 20 (r = 3); 100 steps with 6 -> 4*100 -
    # C(10, 7) = 280 (r = 4)
    assert ag._min_recompute(10, 1) == 20 and ag._min_recompute(100, 5) == 280


def test_binomial_schedule_long_run_is_cheap():
    import time
    t0 = time.perf_counter()
    total = ag.recompute_steps(20000, 12)
    assert time.perf_counter() - t0 < 20.0
    # the forward pass places the first chain of snapshots for free: at most
    # n steps below the bound for a reversal that starts from x(0) alone
    bound = ag._min_recompute(20000, 12)
    assert bound - 20000 <= total <= bound


@pytest.mark.parametrize("keep_x0", [True, False])
@pytest.mark.parametrize("schedule", [{"every": 1}, {"every": 4}, {"snapshots": 0}, {"snapshots": 3}])
@pytest.mark.parametrize("nsteps", [0, 1, 2])
def test_short_runs_take_one_adjoint_step_per_step(nsteps, schedule, keep_x0):
    # nsteps forward steps are reversed by exactly nsteps adjoint steps, in
    # reverse order, each on its own forward state: none for an empty run (its
    # gradient is the initial state's alone), and no buffer handed back twice.
    sim, sw, pool, stored = _run(nsteps, keep_x0=keep_x0 or nsteps == 0, **schedule)
    assert sw.adjoint_steps == nsteps
    assert sim.seen == list(range(nsteps - 1, -1, -1))
    assert len(pool.free) == len({id(b) for b in pool.free})


def test_empty_ranges_are_no_ops():
    sim = FakeSim()
    pool = ag._Pool(sim)
    x = pool.get()
    x.t = 0
    sw = ag._Sweep(sim, pool, None, None, None, None)
    for s in (0, 1, 5):
        sw.binomial(3, 3, x, s)
    sw.segment(2, 2, x)
    assert sw.adjoint_steps == 0 and sim.steps == 0 and pool.free == []


def test_run_rejects_negative_step_counts():
    class _Q:
        q = 27

    with pytest.raises(ValueError):
        ag.run(_Q(), None, None, None, [1.0] * 23, -1, every=1)
    with pytest.raises(ValueError):
        ag.run(_Q(), None, None, None, [1.0] * 23, 2.5, every=1)


class WallFakeSim(FakeSim):
    """Also tracks which adjoint each lam buffer holds, and the wall terms."""

    def __init__(self):
        super().__init__()
        self.wall = []

    def adjoint_step(self, x, lam, lam_tmp, dLdF, dLdw):
        super().adjoint_step(x, lam, lam_tmp, dLdF, dLdw)
        assert lam.t == x.t + 1          # lam(t + 1) in, lam(t) out
        lam_tmp.t = x.t

    def wall_sensitivity_post(self, x, lam, dLdphi):
        assert lam.t == x.t              # the streaming of x(t) into fbar(t)
        self.wall.append(x.t)


@pytest.mark.parametrize("nsteps,schedule", [(12, {"every": 4}), (12, {"snapshots": 2}), (9, {"snapshots": 0}),
                                             (1, {"every": 1}), (2, {"snapshots": 1})])
def test_wall_terms_follow_their_adjoint_steps(nsteps, schedule):
    # With a wall fraction every adjoint step from x(t), t > 0, is followed by
    # the wall term of the streaming x(t) -> fbar(t), taken with lam(t) just
    # computed; the last streaming's term (x(N), the incoming gradient) is the
    # backward pass's own, before the sweep.
    sim = WallFakeSim()
    pool = ag._Pool(sim)
    x0 = pool.get()
    x0.t = 0
    stored, last = ag.forward_sweep(sim, pool, x0, nsteps, ag.keep_positions(nsteps, schedule.get("every"),
                                                                            schedule.get("snapshots")))
    lam, lam_tmp = _State(), _State()
    lam.t = nsteps
    sw = ag._Sweep(sim, pool, lam, lam_tmp, None, None, dLdphi=object())
    ag.backward_sweep(sw, stored, nsteps, schedule.get("every"), schedule.get("snapshots"))
    assert sim.seen == list(range(nsteps - 1, -1, -1))
    assert sim.wall == list(range(nsteps - 1, 0, -1))
