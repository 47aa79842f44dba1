"""Host logic of the serving loop, on the CPU: with stand-ins for the GPU
library (a batch's footprint is 10 bytes per point, plus 12 for its input
buffer; every launch completes at once), the scheduler serves every request,
keeps resident memory within the budget, evicts under pressure instead of
stalling, reuses planned batches of the same systems, and rejects a request
that cannot fit an empty budget."""
import numpy as np
import pytest

import paper_1301_1704_amd.serving as S


class _Batch:
    made = 0

    def __init__(self, off, lev, stream=None):
        self.nbytes = int(off[-1]) * 10
        self.freed = False
        _Batch.made += 1

    def launch(self, x, capture=False):
        assert not self.freed

    def wait(self):
        pass

    def free(self):
        assert not self.freed
        self.freed = True

    def tree(self, i):
        return ("tree", i)


class _Event:
    def record(self, stream):
        pass

    def query(self):
        return True


class _Tensor:
    shape = (1, 3)

    def cuda(self):
        return self

    def add_(self, *a, **k):
        return self

    def clamp_(self, *a):
        return self

    def clone(self):
        return self

    def __getitem__(self, k):
        return self

    def copy_(self, o):
        return self


class _Ctx:
    def __enter__(self):
        pass

    def __exit__(self, *a):
        pass


class _Torch:
    float32 = None

    class cuda:
        Event = _Event

        @staticmethod
        def synchronize():
            pass

        @staticmethod
        def stream(s):
            return _Ctx()

    @staticmethod
    def from_numpy(x):
        return _Tensor()

    @staticmethod
    def empty(*a, **k):
        return _Tensor()


class _Lib:
    Batch = _Batch
    ERR_NOMEM = 3

    class FmmdsError(RuntimeError):
        def __init__(self, status, msg=""):
            super().__init__(msg)
            self.status = status

    @staticmethod
    def batch_footprint(off, lev):
        return int(off[-1]) * 10

    @staticmethod
    def displace(items, sigma, out=None, stream=None):
        pass


SIZES = (100, 200, 300, 400, 500, 600, 700, 800)


def _server(budget, slots=4):
    srv = S.Server.__new__(S.Server)
    srv.torch, srv.F = _Torch, _Lib
    srv.x0 = [np.zeros((n, 3), np.float32) for n in SIZES]
    srv.levels = [3] * len(SIZES)
    srv.n = list(SIZES)
    srv.sigma, srv.seed = 1e-3, 8
    srv.max_batch_points, srv.max_batch_sets = 1 << 24, 64
    srv.slots = [S._Slot(stream=None) for _ in range(slots)]
    srv.budget, srv.keep_inputs, srv.stall_seconds = budget, set(), 5.0
    srv.graphs = True
    srv.reset()
    return srv


PER_POINT = 22  # stand-in footprint (10) + input buffer (12)


@pytest.mark.parametrize("budget", [10 ** 6, 66000, 19800, 17600])
def test_all_requests_served_within_budget(budget):
    arr = np.linspace(0, 0.005, 300)
    pick = np.random.default_rng(1).integers(0, len(SIZES), 300)
    srv = _server(budget)
    peak = []
    reqs = srv.run(arr, pick, on_complete=lambda s, r: peak.append(s.resident))
    assert all(r.done >= r.arrival >= 0 for r in reqs)
    assert max(peak) <= budget
    # each system's steps were taken in arrival order
    per = {}
    for r in reqs:
        per.setdefault(r.system, []).append(r.step)
    for steps in per.values():
        assert steps == sorted(steps) and len(set(steps)) == len(steps)
    if budget >= sum(SIZES) * PER_POINT * 2:
        assert srv.evictions == 0
    srv.close()


def test_batches_hold_several_requests():
    arr = np.zeros(64)
    pick = np.arange(64) % len(SIZES)
    srv = _server(10 ** 7, slots=1)
    reqs = srv.run(arr, pick)
    by_launch = {}
    for r in reqs:
        by_launch.setdefault(r.launched, []).append(r.system)
    assert max(len(v) for v in by_launch.values()) == len(SIZES)  # one per system per batch
    srv.close()


def test_oversize_request_rejected():
    srv = _server(800 * PER_POINT - 1)
    with pytest.raises(_Lib.FmmdsError) as e:
        srv.run(np.zeros(3), np.asarray([7, 0, 1]))
    assert e.value.status == _Lib.ERR_NOMEM


def test_repeated_batches_reuse_their_plan():
    """Four systems on one slot: every batch whose systems were batched
    together before replays that plan instead of making a new one."""
    arr = np.linspace(0, 0.002, 80)
    pick = np.arange(80) % 4
    srv = _server(10 ** 7, slots=1)
    made = _Batch.made
    reqs = srv.run(arr, pick)
    assert all(r.done >= r.arrival for r in reqs)
    assert _Batch.made - made == len(srv.entries)
    launches = len({r.launched for r in reqs})
    assert srv.reused == launches - len(srv.entries) > 0
    srv.close()
