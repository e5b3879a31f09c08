"""Host logic of the serving loop: the list-size bound used for admission
holds against the oracle's exact tile lists, and footprints grow with the
request's size."""
import numpy as np
import pytest

from oracle import Oracle


def _serving():
    pytest.importorskip("torch")
    try:
        from paper_2504_12905_amd import serving
    except ImportError as e:          # the HIP library is not built in this checkout
        pytest.skip(str(e))
    return serving


@pytest.mark.parametrize("n,deg,V,res,seed", [(1000, 0, 4, 64, 0), (3000, 2, 5, 128, 3), (2500, 3, 4, 256, 7)])
def test_instances_bound_holds(n, deg, V, res, seed):
    serving = _serving()
    req = serving.FitRequest(seed=seed, n=n, sh_degree=deg, n_views=V, res=res)
    prob = serving.make_problem(req)
    for beta in (prob.beta_gt, prob.beta_init):
        exact = Oracle(n, deg, beta, prob.cams, res, res).lists()[1].size
        assert exact <= prob.instances_bound, (exact, prob.instances_bound)
        assert prob.instances_bound <= 4 * exact + 1000        # a bound, not a blank cheque


def test_footprint_grows_with_request_size():
    serving = _serving()
    small = serving.footprint_bytes(serving.FitRequest(seed=0, n=2000, sh_degree=0, n_views=4, res=256), 10_000)
    more_views = serving.footprint_bytes(serving.FitRequest(seed=0, n=2000, sh_degree=0, n_views=8, res=256), 10_000)
    more_sh = serving.footprint_bytes(serving.FitRequest(seed=0, n=2000, sh_degree=3, n_views=4, res=256), 10_000)
    more_lists = serving.footprint_bytes(serving.FitRequest(seed=0, n=2000, sh_degree=0, n_views=4, res=256), 10 ** 6)
    assert small < more_views and small < more_sh and small < more_lists
    # targets alone: 4 views of 256^2 RGB floats
    assert small > 4 * 256 * 256 * 12
