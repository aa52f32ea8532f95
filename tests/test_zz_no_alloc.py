"""The non-allocating gradient entry point (mrip_mlp_grad_noalloc, partial
rows in the library's fixed device array) against the allocating
mrip_mlp_grad through the C ABI: bit for bit on two calls in a row, the
second with fewer samples (the array keeps the first call's rows), with and
without multipliers, and the size limit refused."""
import numpy as np
import pytest
import torch

from gpu_util import announce
from paper_1501_01405_amd import inputs, mrip

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _grads(fn, theta, x, z, y, n):
    grad = torch.empty(mrip.MRIP_MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    fn(theta, x, z, y, n, grad, loss, mrip.current_stream())
    torch.cuda.synchronize()
    return grad.cpu().numpy(), float(loss.cpu()[0])


@pytest.mark.parametrize("mult", [True, False])
def test_noalloc_gradient_equals_the_allocating_call(gpu, mult):
    theta = _dev(inputs.he_uniform_init(5))
    for n in (mrip.MRIP_MLP_GRAD_NOALLOC_MAX, 777):
        announce("mlp grad noalloc", n, mult)
        rng = np.random.default_rng(n)
        x = _dev(rng.normal(size=(n, 10)))
        y = _dev(rng.normal(size=n))
        z = _dev(rng.normal(size=(n, 4))) if mult else None
        ref = _grads(mrip.mrip_mlp_grad, theta, x, z, y, n)
        got = _grads(mrip.mrip_mlp_grad_noalloc, theta, x, z, y, n)
        assert np.array_equal(got[0], ref[0]), n
        assert got[1] == ref[1]


def test_noalloc_refuses_more_samples_than_its_array(gpu):
    announce("mlp grad noalloc limit")
    n = mrip.MRIP_MLP_GRAD_NOALLOC_MAX + 1
    theta = torch.zeros(mrip.MRIP_MLP_PARAMS, dtype=torch.float32, device="cuda")
    x = torch.zeros((n, 10), dtype=torch.float32, device="cuda")
    y = torch.zeros(n, dtype=torch.float32, device="cuda")
    grad = torch.empty(mrip.MRIP_MLP_PARAMS, dtype=torch.float32, device="cuda")
    with pytest.raises(mrip.MripError):
        mrip.mrip_mlp_grad_noalloc(theta, x, None, y, n, grad, None, mrip.current_stream())
