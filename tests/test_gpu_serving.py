"""The serving loop: every request's tables and lists in the continuous-
batching mix equal the CPU oracle's build of the same displaced coordinates
and a plain GPU build of them alone (tolerance 0: all outputs are integers or
bit copies); memory admission waits instead of overcommitting and rejects a
request that can never fit."""
import os

import numpy as np
import pytest

from paper_1301_1704_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1301_1704_amd as F
    if not os.path.exists(F.LIB_PATH):
        from paper_1301_1704_amd import _compile
        _compile.build()
    F._lib()
    return F


def _digest(t):
    out = [t.host_perm(0)]
    for l in range(t.depth + 1):
        out += [t.host_keys(0, l), t.host_begin(0, l)]
        if l >= 1:
            out.append(t.host_parent(0, l))
    for l in range(2, t.depth + 1):
        for k in (2, 4):
            out += list(t.host_list(k, l))
    return out


def _oracle_digest(o):
    """The same arrays as _digest, from the oracle (shared set, 64-bit keys)."""
    out = [o.perm(0)]
    for l in range(o.depth + 1):
        out += [o.keys(0, l), o.begin(0, l)]
        if l >= 1:
            out.append(o.parent(0, l))
    for l in range(2, o.depth + 1):
        for k in (2, 4):
            out += list(o.list(k, l))
    return out


def _systems(n=10, seed=3):
    return I.serving_systems(n, seed, 10, 16)


def test_mix_equals_alone(F, oracle_lib):
    import torch
    from paper_1301_1704_amd import serving as S
    systems, levels = _systems()
    arr, pick = I.poisson_trace(80, 4000.0, len(systems), seed=4)
    keep = set(range(0, 80, 3))
    srv = S.Server(systems, levels, n_slots=3, keep_inputs=keep)
    got = {}

    def grab(server, r):
        if r.rid in keep:
            got[r.rid] = _digest(server.tree_of(r.rid))

    reqs = srv.run(arr, pick, on_complete=grab)
    assert all(r.done >= r.arrival for r in reqs)
    assert len(got) == len(keep)
    for rid in sorted(keep):
        r = reqs[rid]
        x = srv.kept_inputs[rid]
        t = F.build(x, None, max_level=int(levels[r.system]), key_bits=64)
        torch.cuda.synchronize()
        alone = _digest(t)
        t.free()
        assert len(alone) == len(got[rid])
        for a, b in zip(alone, got[rid]):
            assert np.array_equal(a, b), rid
        o = oracle_lib.OracleTree(x.cpu().numpy(), None, key_bits=64,
                                  max_level=int(levels[r.system]), with_lists=True)
        ref = _oracle_digest(o)
        o.close()
        assert len(ref) == len(got[rid])
        for i, (a, b) in enumerate(zip(ref, got[rid])):
            assert a.dtype == b.dtype and np.array_equal(a, b), (rid, i)
    # several requests shared a batch (continuous batching actually batched)
    launched = {}
    for r in reqs:
        launched.setdefault(r.launched, []).append(r.rid)
    assert max(len(v) for v in launched.values()) > 1
    srv.close()


def displace_ref(x, seed, sigma):
    """fmmds_displace's definition in FP64: coordinate c = 3i + d moves by
    sigma * sqrt(-2 ln u1) cos(2 pi u2), u1 = ((h >> 40) + 1) 2^-24,
    u2 = ((h >> 16) & 0xFFFFFF) 2^-24, h = output c of splitmix64 stream
    `seed`; then clamped into [0, 1 - 2^-24]."""
    n = x.shape[0]
    h = I.splitmix64(seed, 3 * n)
    u1 = ((h >> np.uint64(40)) + np.uint64(1)).astype(np.float64) * 2.0 ** -24
    u2 = ((h >> np.uint64(16)) & np.uint64(0xFFFFFF)).astype(np.float64) * 2.0 ** -24
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    v = x.astype(np.float64).reshape(-1) + sigma * z
    return np.clip(v, 0.0, 1.0 - 2.0 ** -24).reshape(n, 3)


# FP32 evaluation (logf, cosf, one rounding of x + sigma z) against FP64:
# well under one unit in the last place of a coordinate in [0, 1).
DISPLACE_TOL = 2.0 ** -23


def test_displace_matches_definition_and_is_batch_independent(F):
    import torch
    sizes = [1, 63, 64, 1000, 4097] + [7 + 13 * k for k in range(35)]  # 40 sets: two launches
    xs = [I.uniform_points(100 + k, n) for k, n in enumerate(sizes)]
    seeds = [I.displacement_seed(8, k, 3) for k in range(len(sizes))]
    sigma = 1e-3
    ref = [displace_ref(x, s, sigma) for x, s in zip(xs, seeds)]
    # the reference itself: zero-mean, sigma-wide steps
    d = np.concatenate([(r - x).reshape(-1) for r, x in zip(ref, xs)])
    inner = np.abs(d) < 0.5  # clamped coordinates excluded
    assert abs(d[inner].mean()) < 5e-5 and abs(d[inner].std() / sigma - 1) < 0.05
    # all systems in one call, gathered into one batch input
    dev = [torch.from_numpy(x).cuda() for x in xs]
    first = np.concatenate([[0], np.cumsum(sizes)])
    out = torch.full((int(first[-1]), 3), -1.0, device="cuda")
    F.displace([(x, s, int(f)) for x, s, f in zip(dev, seeds, first)], sigma, out=out)
    torch.cuda.synchronize()
    got = [x.cpu().numpy() for x in dev]
    o = out.cpu().numpy()
    for k in range(len(sizes)):
        assert np.max(np.abs(got[k].astype(np.float64) - ref[k])) <= DISPLACE_TOL, k
        assert np.array_equal(o[first[k]:first[k + 1]], got[k])
        assert got[k].min() >= 0.0 and got[k].max() <= np.float32(1.0 - 2.0 ** -24)
    # each system alone gives the same bits
    for k in (0, 4, 39):
        x = torch.from_numpy(xs[k]).cuda()
        F.displace([(x, seeds[k], 0)], sigma)
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), got[k])


def test_displacement_sequence_matches_sequential_baseline(F):
    """The server and the one-at-a-time baseline apply the same seeded
    displacements in the same per-system order: the final coordinates agree
    bit for bit, and with the FP64 definition replayed on the host."""
    import torch
    from paper_1301_1704_amd import serving as S
    systems, levels = _systems(6, 5)
    arr, pick = I.poisson_trace(40, 3000.0, len(systems), seed=6)
    srv = S.Server(systems, levels, n_slots=2)
    srv.run(arr, pick)
    torch.cuda.synchronize()
    final_server = [x.cpu().numpy() for x in srv.x]
    srv.close()
    seq = []
    reqs = S.run_sequential(systems, levels, arr, pick, final=seq)
    assert all(r.done >= r.arrival for r in reqs)
    steps = [0] * len(systems)
    x = [np.ascontiguousarray(p) for p in systems]
    for r in reqs:
        x[r.system] = displace_ref(x[r.system], I.displacement_seed(8, r.system,
                                                                    steps[r.system]), 1e-3)
        steps[r.system] += 1
    for k, a in enumerate(final_server):
        assert np.max(np.abs(a.astype(np.float64) - x[k])) <= len(reqs) * DISPLACE_TOL
    assert len(seq) == len(final_server)
    for a, b in zip(final_server, seq):
        assert np.array_equal(a, b)


def test_admission_waits_for_memory_and_rejects_oversize(F):
    from paper_1301_1704_amd import serving as S
    systems, levels = _systems(8, 7)
    one = max(F.batch_footprint(np.asarray([0, p.shape[0]], np.uint64),
                                np.asarray([lv], np.uint8)) for p, lv in zip(systems, levels))
    # room for the resident tables of all systems plus about two builds
    budget = 8 * one + 2 * one
    arr, pick = I.poisson_trace(40, 1e5, len(systems), seed=9)
    srv = S.Server(systems, levels, n_slots=4, hbm_budget=budget)
    peak = []

    def watch(server, r):
        peak.append(server.resident)

    reqs = srv.run(arr, pick, on_complete=watch)
    assert all(r.done > 0 for r in reqs)
    assert max(peak) <= budget
    srv.close()
    small = S.Server(systems, levels, hbm_budget=one // 4)
    with pytest.raises(F.FmmdsError) as e:
        small.run(arr[:3], pick[:3])
    assert e.value.status == F.ERR_NOMEM
    small.close()
