"""The no-allocation gradient entry point (dgh_mlp_grad_static) against the
entry point it varies (dgh_mlp_grad with a caller-owned work buffer), through
the C ABI: two calls in a row on the same GPU, the second with a smaller
batch, and the largest batch the fixed array holds.  Same kernels, so the
gradients and losses agree bitwise; both are also checked against the FP64
reference network."""
import numpy as np
import pytest

from oracle.closure import NPARAM, init_params, loss_and_grad

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    X = (0.4 * rng.standard_normal((n, 11))).astype(np.float32)
    T = (0.2 * rng.standard_normal(n)).astype(np.float32)
    return X, T


def test_static_gradient_equals_gradient_with_work_buffer():
    import torch
    from paper_1610_05023_amd import binding as B
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(3)
    wts = init_params(4, in_scale=2.0, g_max=0.3)
    wts[2:] += 0.02 * rng.standard_normal(NPARAM - 2)
    Wd = torch.from_numpy(wts.astype(np.float32)).to(dev)
    for n, seed in ((B.MLP_STATIC_BATCH, 5), (1000, 6), (1, 7)):
        print(f"[no-alloc] batch {n}", flush=True)
        X, T = _inputs(n, seed)
        Xd, Td = torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev)
        G1 = torch.full_like(Wd, float("nan"))
        work = torch.empty(B.mlp_work_size(n), dtype=torch.float32, device=dev)
        loss1 = B.mlp_grad(Wd, Xd, Td, G1, work)
        G2 = torch.full_like(Wd, float("nan"))
        loss2 = B.mlp_grad_static(Wd, Xd, Td, G2)
        g1, g2 = G1.cpu().numpy(), G2.cpu().numpy()
        assert np.array_equal(g1, g2) and loss1 == loss2, (n, np.abs(g1 - g2).max(), loss1, loss2)
        lr_, gr = loss_and_grad(wts.astype(np.float32).astype(np.float64), X.astype(np.float64),
                                T.astype(np.float64))
        eg = float(np.linalg.norm(g2 - gr) / np.linalg.norm(gr))
        assert abs(loss2 - lr_) <= 1e-5 * lr_ and eg < 1e-4, (n, loss2, lr_, eg)


def test_static_gradient_rejects_batches_beyond_its_array():
    import torch
    from paper_1610_05023_amd import binding as B
    dev = torch.device("cuda", 0)
    W = torch.zeros(NPARAM, dtype=torch.float32, device=dev)
    n = B.MLP_STATIC_BATCH + 1
    X = torch.zeros((n, 11), dtype=torch.float32, device=dev)
    T = torch.zeros(n, dtype=torch.float32, device=dev)
    G = torch.zeros_like(W)
    with pytest.raises(B.DghError, match="EINVAL"):
        B.mlp_grad_static(W, X, T, G)
