"""GPU parity on inputs where the order inside a phase decides pixels: the
filling's thinning (priority: distance to the background of the filled set)
and the cutting's thickening (priority: distance to the thinned set). On most
images these phases reach the same set in any order; the oracle's wiring on
these inputs is pinned by tests/test_oracle_compose.py."""
import numpy as np
import pytest

import oracle
import topo_checks as tc
from gpu_util import ctx, dev, host, say
from test_oracle_compose import _bern_case, _constrained_case

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,r", [(4, 3), (24, 5), (28, 3)])
def test_filter_where_the_filling_order_decides(k, r):
    X = _bern_case(k)
    say("filter, order-deciding image", k, X.shape, "r =", r)
    x = dev(X)
    ctx().filter(x, None, r)
    ctx().sync()
    assert np.array_equal(host(x), oracle.hasf(X, None, r))


@pytest.mark.parametrize("k,i", [(97, 3), (100, 3), (283, 3), (556, 4)])
def test_thicken_where_the_cutting_order_decides(k, i):
    """The cutting's thickening as the standalone *H(Y, V): Y the thinned set,
    V its ball dilation inside X; its priority is the distance to Y."""
    X, C = _constrained_case(k)
    Y, _ = tc.hc_composed(X, C, i, tc.simple_table(8))
    V = (tc.dilate_stamp(Y, i) & (X != 0)).astype(np.uint8)
    say("thicken, order-deciding pair", k, X.shape, "i =", i)
    y, v = dev(Y), dev(V)
    ctx().homotopic_thicken(y, v)
    ctx().sync()
    assert np.array_equal(host(y), oracle.homotopic_thicken(Y, V))
