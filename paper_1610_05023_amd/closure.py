"""Training driver of the learned boundary closure.

The teacher is the plain method (HABC of order P with the edge and corner
systems) run by the library; at step ends it records, at every absorbing
face node, the closure's sample row (p and Z |u_t| now, their root mean
squares over the recent past at the closure's four time scales, then r+)
and the incoming characteristic r- the method produced there.  The network is then fitted on the GPU by the library's
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


def teacher_samples(VX, EToV, N, P, rho, c, dt, centers, width, steps, every, start,
                    tau=None):
    """(X[m][11], Y[m]) float32 from one teacher run per centre; tau: the
    closure's time scales (None: the library's default for this mesh),
    which the closure must use too."""
    xs, ys = [], []
    for ctr in centers:
        s = B.Solver(VX, EToV, N, P, rho, c).bind()
        s.set_closure_memory(tau)
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


def train(X, Y, iters=3000, batch=4096, lr=1e-3, seed=5, log_every=0, g_max=0.95, bf16=False):
    """Adam on the mean squared error of r-; returns (parameters, losses).
    The network's reflection gain is bounded by g_max (|g_max| <= 1).
    bf16: the gradient's products in BF16 on the matrix cores (FP32 master
    weights and Adam)."""
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
        loss = B.mlp_grad(W, xb, yb, G, work, with_loss=bool(want), bf16=bf16)
        if want:
            losses.append((t, loss))
        B.mlp_adam(W, G, M, V, t, lr)
    torch.cuda.synchronize()
    return W.cpu().numpy(), losses


class GuardedRun:
    """Steps a context that uses the closure and falls back to the plain
    method when the failure check trips.  Every `check_every` steps it runs
    dgh_check: the state must be finite and, when `rel_tol` is given, its
    energy must not exceed the energy at the last checkpoint by more than
    rel_tol (with no source the closed loop cannot gain energy).  A passing
    check makes the state the new checkpoint; a failing one restores the
    last checkpoint into a context of the plain method with HABC of order
    `fallback_P` (same mesh, medium and source; auxiliary fields from zero)
    and continues there, reporting the step at which it switched."""

    def __init__(self, make_solver, closure_weights, tau=None, fallback_P=6, check_every=100,
                 rel_tol=None, source=None):
        self.make_solver, self.fallback_P = make_solver, fallback_P
        self.check_every, self.rel_tol, self.source = check_every, rel_tol, source
        self.s = make_solver(0)
        self.s.set_closure_memory(tau)
        self.s.set_closure(closure_weights)
        if source is not None:
            self.s.set_source(*source)
        self.switched_at = None
        self.steps_done = 0
        self._ckpt, self._e_ckpt, self._t_ckpt = None, None, 0.0

    def set_state(self, arrays):
        self.s.set_state(arrays)
        self._checkpoint(0.0)

    def _checkpoint(self, t):
        self._ckpt = self.s.read_fields(["q3", "res3"])
        self._e_ckpt = self.s.energy()
        self._t_ckpt, self._n_ckpt = t, self.steps_done

    def step(self, n_steps, dt, t_start=0.0):
        t = t_start
        left = n_steps
        while left > 0:
            k = min(left, self.check_every)
            self.s.step(k, dt, t)
            t += k * dt
            self.steps_done += k
            left -= k
            if self.switched_at is not None:
                continue
            e_ref = self._e_ckpt if self.rel_tol is not None else 0.0
            st, _ = self.s.check(e_ref=e_ref, rel_tol=self.rel_tol or 0.0)
            if st == "DGH_OK":
                self._checkpoint(t)
                continue
            # back to the last good state, in the plain method
            self.s.close()
            self.s = self.make_solver(self.fallback_P)
            if self.source is not None:
                self.s.set_source(*self.source)
            self.s.set_state(self._ckpt)
            self.switched_at = self._n_ckpt
            redo = self.steps_done - self._n_ckpt
            self.s.step(redo, dt, self._t_ckpt)
        return t

    def read_fields(self, names=None):
        return self.s.read_fields(names)
