"""The no-allocation weight setter: through the C ABI, its result equals the
allocating entry point's, on two calls in a row (the second with a smaller
network) and on a world created after them."""
import numpy as np
import pytest

import oracle
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_weights_equal_the_allocating_entry_point(prec):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_09654_amd import binding as B
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(40 + prec)
    # first call: the largest network; second call: a smaller one
    for layers, hidden in [(3, 64), (2, 32)]:
        init = gh.heterogeneous_world(24, 20, n_genomes=4, layers=layers, hidden=hidden,
                                      precision=prec, seed=7)
        w = gh.make_world(init, stream)
        d = gh.oracle_desc(init.spec)
        size = oracle.net_size(d)
        flat = rng.standard_normal(size).astype(np.float32)
        B.coralai_debug_set_weights_noalloc(w.h, 1, flat)   # the new entry point
        B.coralai_debug_set_weights(w.h, 2, flat)           # the existing one
        a = w.debug_get_weights(1, size)
        b = w.debug_get_weights(2, size)
        np.testing.assert_array_equal(a, b)
        rtol = 2.5e-7 if prec == 0 else 2 ** -8
        np.testing.assert_allclose(a, flat, rtol=rtol, atol=0)
        # both slots drive identical steps: cells of genome 1 and of genome 2
        G = np.where(init.G % 2 == 0, 1, 2).astype(np.int32)
        w.set_state(init.E, init.I, init.C, G, init.R)
        act = w.debug_actuators()
        w.close()
        w2 = gh.make_world(init, stream)
        B.coralai_debug_set_weights(w2.h, 1, flat)
        B.coralai_debug_set_weights(w2.h, 2, flat)
        w2.set_state(init.E, init.I, init.C, G, init.R)
        np.testing.assert_array_equal(w2.debug_actuators(), act)
        w2.close()


def test_noalloc_rejects_bad_arguments():
    from paper_2406_09654_amd import binding as B
    init = gh.heterogeneous_world(8, 8, n_genomes=2, seed=1)
    w = gh.make_world(init, torch.cuda.Stream())
    flat = np.zeros(oracle.net_size(gh.oracle_desc(init.spec)), np.float32)
    with pytest.raises(B.CoralaiError):
        B.coralai_debug_set_weights_noalloc(w.h, init.spec.genome_capacity, flat)
    w.close()
