"""Training driver of the learned boundary closure.

The teacher is the plain method (HABC of order P with the edge and corner
systems) run by the library; at step ends it records, at every absorbing
face node, the closure's sample row (p and Z |u_t| now and at the 4
previous step ends, then r+) and the incoming characteristic r- the method
produced there.  The network is then fitted on the GPU by the library's
forward, backward and Adam kernels (binding.mlp_grad / mlp_adam); this
module only samples batches and moves arrays.
"""
from __future__ import annotations

import numpy as np

from . import binding as B

NIN, NH = 10, 64


def gaussian_state(solver, center, width):
    """Zero state with the pressure pulse exp(-|x - c|^2 / w^2) in q3."""
    x = solver.node_coords()
    q3 = np.zeros((solver.counts["K"], 4, solver.counts["Np"]))
    q3[:, 0] = np.exp(-np.sum((x - np.asarray(center)) ** 2, axis=-1) / width ** 2)
    return {"q3": q3}


def teacher_samples(VX, EToV, N, P, rho, c, dt, centers, width, steps, every, start):
    """(X[m][11], Y[m]) float32 from one teacher run per centre."""
    xs, ys = [], []
    for ctr in centers:
        s = B.Solver(VX, EToV, N, P, rho, c).bind()
        s.set_state(gaussian_state(s, ctr, width))
        s.closure_record(True)
        for k in range(1, steps + 1):
            s.step(1, dt, (k - 1) * dt)
            if k >= start and (k - start) % every == 0:
                x, y = s.closure_sample()
                xs.append(x)
                ys.append(y)
        s.close()
    return np.concatenate(xs), np.concatenate(ys)


def init_params(rng, in_scale, g_max):
    """Glorot-uniform weights, zero biases, the two fixed entries first."""
    parts = [np.array([in_scale, g_max])]
    for fan_in, fan_out in ((NIN, NH), (NH, NH), (NH, NH)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        parts += [rng.uniform(-lim, lim, fan_out * fan_in), np.zeros(fan_out)]
    lim = np.sqrt(6.0 / (NH + 1))
    parts += [rng.uniform(-lim, lim, NH), np.zeros(1)]
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == B.CLOSURE_PARAMS
    return w


def train(X, Y, iters=3000, batch=4096, lr=1e-3, seed=5, log_every=0, g_max=0.95):
    """Adam on the mean squared error of r-; returns (parameters, losses).
    The network's reflection gain is bounded by g_max (|g_max| <= 1)."""
    import torch
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(seed)
    in_scale = 1.0          # the inputs reach the network at unit root mean square
    W = torch.from_numpy(init_params(rng, in_scale, g_max)).to(dev)
    G, M, V = torch.zeros_like(W), torch.zeros_like(W), torch.zeros_like(W)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    Yd = torch.from_numpy(np.ascontiguousarray(Y, dtype=np.float32)).to(dev)
    batch = min(batch, len(Yd))
    work = torch.empty(B.mlp_work_size(batch), dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    losses = []
    for t in range(1, iters + 1):
        idx = torch.randint(0, len(Yd), (batch,), device=dev, generator=gen)
        xb, yb = Xd[idx].contiguous(), Yd[idx].contiguous()
        want = log_every and (t % log_every == 0 or t == iters)
        loss = B.mlp_grad(W, xb, yb, G, work, with_loss=bool(want))
        if want:
            losses.append((t, loss))
        B.mlp_adam(W, G, M, V, t, lr)
    torch.cuda.synchronize()
    return W.cpu().numpy(), losses
