"""The allocation-free entry point (fim_mine_noalloc) against fim_mine.

Two calls in a row through the C ABI, the second on a smaller database,
each compared element by element with fim_mine's result on the same input
(integer work: bit-exact), plus the sizes reported when the caller's
arrays are too small.
"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fim():
    import paper_2108_05038_amd as F
    F.lib()
    return F


def test_noalloc_matches_fim_mine_twice(fim):
    ctx = fim.Context(0)
    big = synth.basket(424242, 20000, 800, 10.0, 1600, 4.0)
    small = synth.basket(777, 3001, 150, 10.0, 300, 4.0)
    for name, (o_, it, ni), m in (("20000 tx", big, 40), ("3001 tx", small, 12)):
        say("noalloc", name)
        d = fim.Database(ctx, o_, it, ni)
        ref = fim.mine(ctx, d, m)
        off, items, supp = fim.mine_noalloc(ctx, d, m, len(ref) + 10, len(ref.items) + 10)
        assert len(ref) > 100
        assert np.array_equal(off, ref.offsets)
        assert np.array_equal(items, ref.items)
        assert np.array_equal(supp, ref.supports)
        # arrays too small: an error, and the sizes the result needs
        st, _, _, _, n, nit = fim.fim_mine_noalloc(ctx.handle, d.handle, m, len(ref) - 1,
                                                   len(ref.items), None)
        assert st == fim.FIM_E_OUTPUT_LIMIT
        assert (n, nit) == (len(ref), len(ref.items))
        d.close()
    ctx.close()
