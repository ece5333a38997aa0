"""Learned starting guess for the Riemann star pressure: a 6 -> 32 -> 32 -> 1
network with ReLU activations, BF16 weights on the MFMA units and FP32
accumulation, trained on interface states the solver itself logs.

Every computation runs in libhydro.so's kernels (features, forward, the fused
forward/backward gradient, Adam, BF16 packing); this module holds the device
buffers and drives the training loop.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from ._lib import check

N_PARAMS = 1313
N_IN, N_HIDDEN = 6, 32
OFF_W1, OFF_B1 = 0, 192
OFF_W2, OFF_B2 = 224, 1248
OFF_W3, OFF_B3 = 1280, 1312
LOG_FIELDS = 8
# Training targets ln(p*/p_ptr) (the correction of the two-rarefaction guess
# p_ptr) are clipped to +-TARGET_CLIP: near-vacuum interfaces (p* at the
# pressure floor, ln ratios down to about -60) would otherwise dominate the
# squared error; the guess only has to point Newton the right way there, and
# the residual test hands such interfaces to the two-rarefaction fallback.
TARGET_CLIP = 8.0


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights (ReLU layers), zero biases, FP32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(N_PARAMS, dtype=np.float32)
    p[OFF_W1:OFF_B1] = rng.uniform(-1, 1, N_HIDDEN * N_IN) * math.sqrt(6.0 / N_IN)
    p[OFF_W2:OFF_B2] = rng.uniform(-1, 1, N_HIDDEN * N_HIDDEN) * math.sqrt(6.0 / N_HIDDEN)
    p[OFF_W3:OFF_B3] = rng.uniform(-1, 1, N_HIDDEN) * math.sqrt(3.0 / N_HIDDEN)
    return p


class GuessNetwork:
    """FP32 master parameters, Adam moments and the packed device network."""

    def __init__(self, params: np.ndarray | None = None, seed: int = 0, device="cuda",
                 stream: torch.cuda.Stream | None = None):
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        self.params = torch.tensor(p, device=self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.dev = torch.zeros(self.lib.hydro_mlp_dev_bytes(), dtype=torch.uint8, device=self.device)
        self.step_count = 0
        self._scratch = None
        self.pack()

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    # The kernels run on self.stream; inputs come from, and outputs go back to,
    # torch's current stream, so both directions are ordered explicitly.
    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def pack(self) -> None:
        self._enter()
        check(self.lib.hydro_mlp_pack(_ptr(self.params), _ptr(self.dev), self._s()))

    def set_params(self, p) -> None:
        self.params.copy_(torch.as_tensor(np.asarray(p, dtype=np.float32)))
        torch.cuda.synchronize(self.device)
        self.pack()

    def features(self, records: torch.Tensor, gamma: float = 1.4):
        """records float32 [n, 8] on the device -> (X [n, 6], Y [n]): features
        (a, b, w, q, -a, -b) and targets ln(p*/p_ptr)."""
        n = records.shape[0]
        X = torch.empty((n, N_IN), dtype=torch.float32, device=self.device)
        Y = torch.empty(n, dtype=torch.float32, device=self.device)
        self._enter()
        check(self.lib.hydro_mlp_features(_ptr(records), n, gamma, _ptr(X), _ptr(Y), self._s()))
        self._leave()
        return X, Y

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        n = X.shape[0]
        Y = torch.empty(n, dtype=torch.float32, device=self.device)
        self._enter()
        check(self.lib.hydro_mlp_forward(_ptr(self.dev), _ptr(X), _ptr(Y), n, self._s()))
        self._leave()
        return Y

    def loss_grad(self, X: torch.Tensor, T: torch.Tensor):
        """(grad, loss) of the mean squared error on the device (synchronises)."""
        n = X.shape[0]
        need = self.lib.hydro_mlp_grad_scratch_bytes(n) // 4
        if self._scratch is None or self._scratch.numel() < need:
            self._scratch = torch.empty(need, dtype=torch.float32, device=self.device)
        self._enter()
        check(self.lib.hydro_mlp_grad(_ptr(self.dev), _ptr(X), _ptr(T), n, _ptr(self._scratch),
                                      _ptr(self.grad), _ptr(self.loss), self._s()))
        self.stream.synchronize()
        return self.grad.clone(), float(self.loss.item())

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
        self.step_count += 1
        self._enter()
        check(self.lib.hydro_mlp_adam(_ptr(self.params), _ptr(self.m), _ptr(self.v),
                                      _ptr(self.grad), self.step_count, lr, beta1, beta2, eps,
                                      self._s()))
        self.pack()

    def train(self, X: torch.Tensor, T: torch.Tensor, epochs=4, batch=8192, lr=1e-3, seed=0):
        """Mini-batch Adam on the device; returns the mean loss of each epoch."""
        n = X.shape[0]
        batch = min(batch, n)
        self._enter()
        with torch.cuda.stream(self.stream):
            T = T.clamp(-TARGET_CLIP, TARGET_CLIP)
        g = torch.Generator(device=self.device)
        g.manual_seed(seed)
        history = []
        need = self.lib.hydro_mlp_grad_scratch_bytes(batch) // 4
        if self._scratch is None or self._scratch.numel() < need:
            self._scratch = torch.empty(need, dtype=torch.float32, device=self.device)
        epoch_loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        for _ in range(epochs):
            with torch.cuda.stream(self.stream):
                perm = torch.randperm(n, device=self.device, generator=g)
                epoch_loss.zero_()
            nb = 0
            for b0 in range(0, n - batch + 1, batch):
                with torch.cuda.stream(self.stream):
                    idx = perm[b0:b0 + batch]
                    xb = X.index_select(0, idx)
                    tb = T.index_select(0, idx)
                check(self.lib.hydro_mlp_grad(_ptr(self.dev), _ptr(xb), _ptr(tb), batch,
                                              _ptr(self._scratch), _ptr(self.grad),
                                              _ptr(self.loss), self._s()))
                with torch.cuda.stream(self.stream):
                    epoch_loss.add_(self.loss)
                self.adam(lr)
                nb += 1
            self.stream.synchronize()
            history.append(float(epoch_loss.item()) / max(nb, 1))
        return history

    def params_numpy(self) -> np.ndarray:
        self.stream.synchronize()
        return self.params.detach().cpu().numpy().copy()
