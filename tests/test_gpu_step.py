"""GPU: the benchmark's step in its two forms computes the same thing.

The stream-ordered step (lists from the stream-ordered build, the queued
multipole + dipole call, HAL on a second stream beside the solve, nothing
read back inside the step) must give bitwise the outputs of the synchronous
step (host-sized lists, the synchronous multipole + dipole call, HAL after
it), whose results the other tests check against the oracle.
"""
import numpy as np
import pytest

from paper_1906_01211_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    import torch
    from paper_1906_01211_amd import tk as _tk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _tk.load()
    return _tk


@pytest.fixture(scope="module")
def ctx(tk):
    c = tk.Context(0)
    yield c
    c.close()


def flat(out):
    (e, f, v), mu, (ev, fv, vv) = out
    return [t.detach().cpu().numpy() for t in (e, f, v, mu, ev, fv, vv)]


@pytest.mark.parametrize("name", ["water216", "water7853"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("serial", [False, True])
def test_stream_ordered_step_equals_synchronous_step(ctx, tk, name, prec, serial):
    import bench
    w = synth.make(name)
    ref = bench.AmoebaStep(ctx, tk, w, prec)
    ref()
    if prec == tk.MIXED and ref.info["refinements"]:
        pytest.skip("the synchronous mixed solve refined (the queued one does not)")
    q = bench.QueuedAmoebaStep(ctx, tk, w, prec, ref.info["iters"], serial=serial)
    for _ in range(3):   # back to back, nothing read in between
        q()
    info = q.check()     # every step's list statuses and solve outcome
    assert info == ref.info
    for a, b in zip(flat(q.out), flat(ref.out)):
        assert np.array_equal(a, b)
