"""Learned warm start for GN: a two-layer message-passing network (hidden 64,
bfloat16 matrix-core products) that predicts x0 from per-vertex weight and degree
features, trained on the sets that GN itself reaches.

Protocol (measured on held-out unit-disk graphs of 100,000 vertices): the start
keeps only the network's confident vertices (gate 0.49: p < 0.01 or p > 0.99),
every other vertex starts at the neutral 1/2 of plain GN, and GN then runs a
300-step gamma ramp 0.9 -> 1.5 instead of the paper's 1000 steps.

Every computation runs in libgn (gn_mpnn_forward / gn_mpnn_backward /
gn_adam_step / gn_solve); this module holds parameters and drives the loop.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import libgn

NPARAMS = 9409
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_U, OFF_C = 0, 1024, 1088, 9280, 9344, 9408


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights (fan-in 8 for layer 1, 128 for layer 2, 64 for the head),
    zero biases, zero padding rows 8-15 of W1."""
    rng = np.random.default_rng(seed)
    th = np.zeros(NPARAMS, dtype=np.float32)
    w1 = rng.standard_normal((16, 64)) * math.sqrt(2.0 / 8)
    w1[8:] = 0.0
    th[OFF_W1:OFF_B1] = w1.reshape(-1)
    th[OFF_W2:OFF_B2] = (rng.standard_normal((128, 64)) * math.sqrt(2.0 / 128)).reshape(-1)
    th[OFF_U:OFF_C] = rng.standard_normal(64) * math.sqrt(1.0 / 64)
    return th


class WarmStart:
    def __init__(self, params: np.ndarray | None = None, seed: int = 0, device: str = "cuda"):
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        assert p.size == NPARAMS
        self.device = torch.device(device)
        self.params = torch.tensor(p, device=self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, device=self.device)
        self.t = 0
        self._cache = {}

    def _cache_for(self, n: int) -> torch.Tensor:
        c = self._cache.get(n)
        if c is None:
            c = torch.empty(libgn.gn_mpnn_cache_bytes(n), dtype=torch.uint8, device=self.device)
            self._cache = {n: c}  # keep one buffer (the last size)
        return c

    def predict(self, graph: "libgn.Graph", gate: float = 0.0, x0: torch.Tensor | None = None,
                z: torch.Tensor | None = None):
        """x0 on the device (user vertex order): p = sigmoid(net(graph)) clamped to
        [1e-3, 1] where |p - 1/2| > gate, 1/2 elsewhere."""
        if x0 is None:
            x0 = torch.empty(graph.n, dtype=torch.float32, device=self.device)
        libgn.gn_mpnn_forward(graph.handle, self.params, x0, z, self._cache_for(graph.n), gate)
        return x0

    def train_step(self, graph: "libgn.Graph", labels: torch.Tensor, lr: float = 3e-3) -> torch.Tensor:
        """One forward + backward + Adam step on one graph; returns the loss (device)."""
        x0 = torch.empty(graph.n, dtype=torch.float32, device=self.device)
        cache = self._cache_for(graph.n)
        libgn.gn_mpnn_forward(graph.handle, self.params, x0, None, cache, 0.0)
        libgn.gn_mpnn_backward(graph.handle, self.params, labels, cache, self.grad, self.loss)
        self.t += 1
        libgn.gn_adam_step(self.params, self.grad, self.m, self.v, lr, 0.9, 0.999, 1e-8, self.t)
        return self.loss

    def state(self) -> np.ndarray:
        return self.params.detach().cpu().numpy().copy()


def gn_labels(graph: "libgn.Graph", schedule: dict, starts: int = 1, seed: int = 0):
    """Labels from GN's own results: the best set (by weight) over `starts` solves,
    the first from x0 = 1/2, the others from random points of the simplex
    (exponential sampling normalised by its maximum and clamped to [1e-3, 1], the
    random start of the paper's code appendix).  Returns (labels, best result)."""
    dev = torch.device("cuda")
    best, best_sel = None, None
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    for s in range(starts):
        if s == 0:
            x = torch.full((graph.n,), 0.5, device=dev)
        else:
            u = 1.0 - torch.rand(graph.n, device=dev, generator=gen)  # uniforms in (0, 1]
            x = torch.empty_like(u)
            graph.random_starts(1, u, x)
        sel = torch.zeros(graph.n, dtype=torch.uint8, device=dev)
        r = graph.solve(x, sel, **schedule)
        if best is None or r.set_objective > best.set_objective:
            best, best_sel = r, sel
    return best_sel.to(torch.float32), best


GATE = 0.49
WARM_SCHEDULE = dict(gamma0=0.9, gamma1=1.5, ramp_steps=300, max_steps=4000, tau=1e-4, check_every=1)
PLAIN_SCHEDULE = dict(gamma0=0.9, gamma1=1.5, ramp_steps=1000, max_steps=4000, tau=1e-4, check_every=1)


def warm_solve(net: WarmStart, graph: "libgn.Graph", sel: torch.Tensor, gate: float = GATE, schedule=None):
    """Network inference, then GN to binarisation from the gated start."""
    x0 = net.predict(graph, gate)
    return graph.solve(x0, sel, **(schedule or WARM_SCHEDULE)), x0


def train(net: WarmStart, graphs, labels, steps: int, lr: float = 3e-3, log_every: int = 0):
    """Cycle over (graph, labels) pairs for `steps` Adam steps; returns the loss trace."""
    trace = []
    for k in range(steps):
        i = k % len(graphs)
        loss = net.train_step(graphs[i], labels[i], lr)
        if log_every and (k % log_every == 0 or k == steps - 1):
            trace.append((k, float(loss.item())))
    return trace
