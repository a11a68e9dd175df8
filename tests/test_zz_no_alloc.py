"""ladder_forward_noalloc (the forward on the library's static device scratch, for callers
that cannot allocate) against ladder_forward, through the C ABI: two calls in a row, the
second on a smaller input, so the second runs on whatever the first left in the scratch."""
import numpy as np
import pytest
import torch

import paper_2202_02019_amd as P
from helpers import gaussian_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch.device("cuda:0")


def g(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


@pytest.mark.parametrize("precision,n_abatch,flags", [(P.FP64, 0, 0), (P.SPLIT_BF16, 0, 0), (P.FP64, 4, P.FLAG_DENSE),
                                                      (P.SPLIT_BF16, 3, 0), (P.SPLIT_INT8, 0, 0),
                                                      (P.SPLIT_INT8, 3, P.FLAG_DENSE)])
def test_noalloc_forward_matches_forward(dev, precision, n_abatch, flags):
    opts = P.Options(precision=precision, n_abatch=n_abatch, flags=flags)
    for k, (o, v, n) in enumerate([(5, 37, 70), (3, 20, 33)]):   # the second call is smaller
        L, tau, w = gaussian_inputs(600 + 10 * k + precision, o, v, n)
        Lg, tg, wg = g(L, dev), g(tau, dev), g(w, dev)
        R1, E1 = P.forward(Lg, tg, wg, o=o, v=v, n=n, opts=opts)
        R2 = torch.full_like(R1, float("nan"))
        E2 = torch.full((), float("nan"), dtype=torch.float64, device=dev)
        P.forward_noalloc(Lg, tg, wg, o=o, v=v, n=n, R=R2, E=E2, opts=opts)
        torch.cuda.synchronize()
        print("noalloc (%d, %d, %d) precision %d n_abatch %d: E %.17g vs %.17g" % (o, v, n, precision, n_abatch,
                                                                                 float(E2), float(E1)))
        # the same plan and kernels as ladder_forward: bitwise equal
        assert torch.equal(R1, R2) and torch.equal(E1, E2)


def test_noalloc_forward_beta_and_no_energy(dev):
    o, v, n = 4, 29, 40
    L, tau, w = gaussian_inputs(650, o, v, n)
    Lg, tg = g(L, dev), g(tau, dev)
    R0 = g(np.random.default_rng(651).standard_normal((o, o, v, v)), dev)
    R1, _ = P.forward(Lg, tg, None, o=o, v=v, n=n, R=R0.clone(), beta=0.5)
    R2 = R0.clone()
    P.forward_noalloc(Lg, tg, None, o=o, v=v, n=n, R=R2, beta=0.5)
    torch.cuda.synchronize()
    assert torch.equal(R1, R2)
