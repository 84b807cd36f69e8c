"""The allocation-free entry point ms_transmission_batch_noalloc, through the C ABI, against
ms_transmission_batch (the entry point it is a variant of) on the same inputs: two calls in a
row, the second with a smaller input, then a call that needs sub-batches inside the fixed
scratch, and one that does not fit it at all (rejected before anything is enqueued)."""
import numpy as np
import pytest
import torch

import msgen
from gpu_common import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ms():
    import paper_1504_01462_amd as m
    return m


def _both(ms, ctx, s, es, prec="fp64"):
    ref = [x.cpu().numpy() for x in ms.ms_transmission_batch(ctx, s, es, prec)]
    n = len(es)
    outs = (torch.full((n,), -1.0, dtype=torch.float64, device=dev()),
            torch.full((n,), -1.0, dtype=torch.float64, device=dev()),
            torch.full((n,), -7, dtype=torch.int64, device=dev()),
            torch.full((n,), 99, dtype=torch.int32, device=dev()))
    got = [x.cpu().numpy() for x in ms.ms_transmission_batch_noalloc(ctx, s, es, *outs, prec=prec)]
    ctx.sync()
    return ref, got


def _same(ref, got, tol=1e-12):
    assert np.array_equal(ref[3], got[3]) and np.all(got[3] == 0)
    assert np.array_equal(ref[2], got[2])
    assert np.max(np.abs(ref[0] - got[0])) <= tol and np.max(np.abs(ref[1] - got[1])) <= tol


def test_noalloc_matches_batch_twice_then_smaller(ms):
    ctx = ms.Context(0)
    j = msgen.config1()
    inp = msgen.junction_inputs(j, j.kpars[0])
    s = ms.prepare_from_inputs(ctx, inp)
    es = np.linspace(0.1, 3.9, 10)
    ref, got = _both(ms, ctx, s, es)
    _same(ref, got)
    # second call: a smaller input (fewer plane waves and slices, fewer energies)
    j2 = msgen.config1()
    j2.dz = np.full(9, 6.0 / 9)
    s2 = ms.prepare_from_inputs(ctx, msgen.junction_inputs(j2, (0.07, -0.11), 21))
    ref, got = _both(ms, ctx, s2, [0.4, 1.7, 2.2])
    _same(ref, got)
    ref, got = _both(ms, ctx, s2, [0.4, 1.7, 2.2], "fp32")
    _same(ref, got, 0.0)
    ctx.close()


def test_noalloc_sub_batches_inside_the_scratch(ms):
    """N_G = 300 with 48 energies: about 10 instances fit the scratch at once, so the call folds
    them in several sub-batches, with the results of one batch of all 48."""
    ctx = ms.Context(0)
    j = msgen.config2("AA", n_slices=40)
    j.dz = np.full(40, 0.4)
    s = ms.prepare_from_inputs(ctx, msgen.junction_inputs(j, j.kpars[5]))
    ref, got = _both(ms, ctx, s, np.linspace(0.1, 1.0, 48))
    _same(ref, got)
    ctx.close()


def test_noalloc_full_basis_size(ms):
    """One instance at N_G = 1200 (about 104 MB of scratch) fits: the same T, R, N_open as the
    allocating entry point."""
    ctx = ms.Context(0)
    j = msgen.config3(6.3, "AA", n_slices=2)
    j.dz = np.full(2, 0.05)
    s = ms.prepare_from_inputs(ctx, msgen.junction_inputs(j, j.kpars[3]))
    ref, got = _both(ms, ctx, s, [0.5])
    _same(ref, got)
    ctx.close()


def test_noalloc_rejects_what_does_not_fit(ms):
    """One instance at N_G = 1500 needs more than the scratch (about 158 MB): MS_ERR_UNSUPPORTED,
    outputs untouched; the next call on the context works."""
    ctx = ms.Context(0)
    j = msgen.config3(6.3, "AA", n_g=1500, n_slices=2)
    j.dz = np.full(2, 0.05)
    s = ms.prepare_from_inputs(ctx, msgen.junction_inputs(j, j.kpars[3]))
    T = torch.full((1,), -1.0, dtype=torch.float64, device=dev())
    outs = (T, torch.zeros_like(T), torch.zeros(1, dtype=torch.int64, device=dev()),
            torch.zeros(1, dtype=torch.int32, device=dev()))
    with pytest.raises(ms.MSError) as ei:
        ms.ms_transmission_batch_noalloc(ctx, s, [0.5], *outs)
    assert ei.value.status == ms.MS_ERR_UNSUPPORTED
    ctx.sync()
    assert float(T.cpu()[0]) == -1.0
    j1 = msgen.config1()
    s1 = ms.prepare_from_inputs(ctx, msgen.junction_inputs(j1, j1.kpars[0]))
    ref, got = _both(ms, ctx, s1, [0.3, 0.8])
    _same(ref, got)
    ctx.close()
