"""Builds from several host threads at once, each thread on its own stream and
with separate receivers, so that every call also runs its receivers' chain on
the library's shared receiver stream: every tree must equal the tree the same
build gives when it runs alone."""
import os
import sys
import threading

import numpy as np
import pytest

import parity
from paper_1301_1704_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


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


def _snapshot(t):
    """Every output array of a tree, copied to the host."""
    out = []
    for s in (0, 1):
        out.append(t.host_perm(s))
        out.append(t.host_sorted_xyz(s))
        for l in range(t.depth + 1):
            out.append(t.host_keys(s, l))
            out.append(t.host_begin(s, l))
    for l in range(2, t.depth + 1):
        for kind in (2, 4):
            out.extend(t.host_list(kind, l))
    return out


def test_concurrent_builds_from_threads(F):
    import torch
    cases = [(I.uniform_points(300 + i, 150000 + 20011 * i),
              I.sphere_cluster_points(310 + i, 311, 90000 + 7001 * i), 6 + i % 2)
             for i in range(4)]
    ref = []
    for src, recv, L in cases:
        t = F.build(parity.to_gpu(src), parity.to_gpu(recv), max_level=L)
        torch.cuda.synchronize()
        ref.append(_snapshot(t))
        t.free()
    dev = [(parity.to_gpu(src), parity.to_gpu(recv)) for src, recv, _ in cases]
    torch.cuda.synchronize()
    results = [None] * len(cases)
    errors = []

    def work(i):
        try:
            s = torch.cuda.Stream()
            trees = [F.build(dev[i][0], dev[i][1], max_level=cases[i][2], stream=s)
                     for _ in range(3)]
            s.synchronize()
            results[i] = trees
        except Exception as e:  # reported by the main thread
            errors.append((i, e))

    _say("case 4 threads x 3 builds, separate receivers")
    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(cases))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for i, trees in enumerate(results):
        for k, t in enumerate(trees):
            got = _snapshot(t)
            assert len(got) == len(ref[i])
            for a, b in zip(got, ref[i]):
                assert a.tobytes() == b.tobytes(), (i, k)
            t.free()
