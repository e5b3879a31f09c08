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


def test_admission_order():
    """Shortest estimated work first among the requests that have arrived and
    fit the budget ("sjf"); arrival order without overtaking ("fifo")."""
    serving = _serving()

    def prob(i, n, views, res, t, fp):
        req = serving.FitRequest(seed=i, n=n, sh_degree=0, n_views=views, res=res, arrival_t=t, id=i)
        return serving.Problem(req, None, None, None, 0, fp)

    big = prob(0, 100_000, 24, 800, 0.0, 10)
    small = prob(1, 2_000, 4, 256, 0.1, 10)
    mid = prob(2, 20_000, 8, 512, 0.2, 10)
    late = prob(3, 1_000, 2, 128, 5.0, 10)
    huge_fp = prob(4, 1_500, 2, 128, 0.0, 10 ** 9)
    pending = [big, huge_fp, small, mid, late]
    sjf = serving.Server(hbm_budget_bytes=100, policy="sjf")
    assert serving.work_estimate(small.req) < serving.work_estimate(mid.req) < serving.work_estimate(big.req)
    # at t = 1: late has not arrived and huge_fp does not fit, so the least work is small
    assert sjf._pick(pending, 1.0, 0) == 2
    assert sjf._pick(pending, 0.15, 0) == 2
    assert sjf._pick(pending, 0.05, 0) == 0        # only big has arrived (and fits)
    assert sjf._pick(pending, 6.0, 0) == 4          # late (the least work) has arrived
    assert sjf._pick(pending, 6.0, 95) is None     # nothing fits next to 95 of 100
    fifo = serving.Server(hbm_budget_bytes=100, policy="fifo")
    assert fifo._pick(pending, 1.0, 0) == 0
    assert fifo._pick(pending[1:], 1.0, 0) is None  # the head does not fit: no overtaking
