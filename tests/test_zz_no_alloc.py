"""pr_run_batch_static (the batch entry point that allocates nothing: its
descriptors and counters live in the library's fixed device scratch) through
the C-ABI against pr_run_batch on the same simulations and history ids, on two
calls in a row, the second with a smaller batch; and its size limit."""
import numpy as np
import pytest

from paper_2304_06226_amd import binding as B
from paper_2304_06226_amd import workloads as W

pytestmark = pytest.mark.gpu


def _close(a, b):
    for (sw, sw2, nh), (rw, rw2, rn) in zip(a, b):
        assert nh == rn
        np.testing.assert_allclose(sw, rw, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(sw2, rw2, rtol=1e-9, atol=1e-12)


def test_static_batch_equals_run_batch():
    import torch
    assert torch.cuda.is_available()
    ctx = B.Context(device=0, seed=4096)
    try:
        batch = W.sample_batch(scale=0.01, imaging_histories=50_000, n_sims=24)
        ref = B.BatchRun(ctx, batch, base=5_000_000)
        got = B.BatchRun(ctx, batch, base=5_000_000)
        for k, count in enumerate((len(batch.problems), 7)):
            print(f"[case] static batch call {k}: {count} simulations", flush=True)
            ref.reset()
            got.reset()
            torch.cuda.synchronize()
            shift = k * ref.span
            ctx.run_batch(ref.descriptors(shift)[:count])
            ctx.run_batch_static(got.descriptors(shift)[:count])
            torch.cuda.synchronize()
            for i in range(count):
                r, g = ref.sims[i].results(), got.sims[i].results()
                assert r[0][2] == batch.problems[i].n_histories
                _close(g, r)
            for i in range(count, len(batch.problems)):
                for sw, sw2, nh in got.sims[i].results():
                    assert nh == 0 and not sw.any()
        # descriptors beyond the 2 MiB scratch: refused before any device work
        one = got.descriptors()[0]
        with pytest.raises(B.PromptError) as e:
            ctx.run_batch_static([one] * 8000)
        assert e.value.code == B.PR_EWORKSPACE
    finally:
        ctx.close()
