"""The no-allocation closure training entry point against the allocating one
(through the C ABI): the same Adam updates bit for bit on two calls in a
row, the second with fewer pairs and a smaller minibatch, both calls on
caller-owned device memory and the library's fixed workspace."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _pkg():
    import paper_2107_03550_amd as pkg
    return pkg


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 33)).astype(np.float32)
    X[:, 0] = rng.uniform(0.0, 0.6, n)
    Y = (0.5 * rng.standard_normal((n, 2))).astype(np.float32)
    return X, Y


def test_no_alloc_training_equals_allocating_training():
    import torch
    from paper_2107_03550_amd.closure_train import init_params
    pkg = _pkg()
    dev = torch.device("cuda:0")
    p0 = init_params(3)
    ref = pkg.ClosureTrainer(p0)
    P = torch.tensor(p0, device=dev)
    M = torch.zeros(pkg.CLOSURE_PARAMS, dtype=torch.float32, device=dev)
    V = torch.zeros_like(M)
    t = ctypes.c_int64(0)
    stream = torch.cuda.current_stream().cuda_stream
    for n, batch, steps, seed in ((1000, 256, 5, 1), (300, 64, 3, 2)):
        X, Y = _data(n, seed)
        ref_losses = ref.train(X, Y, batch, steps, 1e-3)
        dX = torch.tensor(X, device=dev)
        dY = torch.tensor(Y, device=dev)
        dL = torch.zeros(steps, dtype=torch.float64, device=dev)
        st = pkg.closure_train_noalloc(dX.data_ptr(), dY.data_ptr(), n, batch, steps, 1e-3,
                                       P.data_ptr(), M.data_ptr(), V.data_ptr(), t, dL.data_ptr(),
                                       stream)
        assert st == 0, pkg.lib.sbiem_last_error(None)
        torch.cuda.synchronize()
        assert t.value == ref.t.value
        assert np.array_equal(P.cpu().numpy(), ref.params)
        assert np.array_equal(M.cpu().numpy(), ref.m) and np.array_equal(V.cpu().numpy(), ref.v)
        assert np.array_equal(dL.cpu().numpy(), ref_losses)
    # no loss output, then a minibatch past the workspace: a clear error
    st = pkg.closure_train_noalloc(dX.data_ptr(), dY.data_ptr(), n, 32, 1, 1e-3, P.data_ptr(),
                                   M.data_ptr(), V.data_ptr(), t, None, stream)
    torch.cuda.synchronize()
    assert st == 0
    st = pkg.closure_train_noalloc(dX.data_ptr(), dY.data_ptr(), n, pkg.CLOSURE_TRAIN_MAX_BATCH + 1,
                                   1, 1e-3, P.data_ptr(), M.data_ptr(), V.data_ptr(), t, None, stream)
    assert st == -1
    assert b"workspace" in pkg.lib.sbiem_last_error(None)
