"""Training and use of the learned inversion guess through the C ABI.

Marshalling only: the forward, backward, Adam and BF16 matrix-core inference
all run in libgrmhd.so.  Parameters are FP32 device tensors in the layout of
include/grmhd.h (W1[64][5] b1 W2[64][64] b2 W3[64][64] b3 W4[2][64] b4).
"""
import ctypes
import math

import numpy as np

from . import grmhd as G

LAYERS = [5, 64, 64, 64, 2]


def init_params(seed=0):
    """He-uniform weights, zero biases, flattened in the ABI layout (numpy FP64)."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(4):
        fi, fo = LAYERS[l], LAYERS[l + 1]
        lim = math.sqrt(6.0 / fi)
        out.append(rng.uniform(-lim, lim, (fo, fi)).ravel())
        out.append(np.zeros(fo))
    flat = np.concatenate(out)
    assert flat.size == G.MLP_NPARAM
    return flat


def unflatten(flat):
    """Flat ABI layout -> list of (W, b) pairs."""
    P, o = [], 0
    for l in range(4):
        fi, fo = LAYERS[l], LAYERS[l + 1]
        W = flat[o:o + fi * fo].reshape(fo, fi)
        o += fi * fo
        b = flat[o:o + fo]
        o += fo
        P.append((W, b))
    return P


def _scratch(torch, batch, device):
    nb = G.lib().grmhd_mlp_scratch_bytes(batch)
    buf = torch.zeros(nb + 256, dtype=torch.uint8, device=device)
    return buf, (buf.data_ptr() + 255) // 256 * 256, nb


_streams = {}


def _stream(torch, dev):
    """One private default-priority stream per device for the MLP calls."""
    if dev not in _streams:
        _streams[dev] = torch.cuda.Stream(device=dev)
    return _streams[dev]


def grad(params, X, Y):
    """(loss, gradient) of the FP32 kernels; all arguments float32 device tensors."""
    import torch
    dev = params.device
    B = X.shape[0]
    buf, ptr, nb = _scratch(torch, B, dev)
    g = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    s = _stream(torch, dev)
    stream = s.cuda_stream
    torch.cuda.synchronize(dev)
    G._check(G.lib().grmhd_mlp_grad(params.data_ptr(), X.data_ptr(), Y.data_ptr(), B,
                                    g.data_ptr(), loss.data_ptr(), ptr, nb, stream))
    s.synchronize()
    return float(loss.item()), g


def infer(params, mean, std, Xraw):
    """BF16 matrix-core inference: raw features [n,5] -> outputs [n,2]."""
    import torch
    dev = params.device
    n = Xraw.shape[0]
    buf, ptr, nb = _scratch(torch, 1, dev)
    Y = torch.zeros((n, 2), dtype=torch.float32, device=dev)
    s = _stream(torch, dev)
    torch.cuda.synchronize(dev)
    G._check(G.lib().grmhd_mlp_infer(params.data_ptr(), mean.data_ptr(), std.data_ptr(),
                                     Xraw.data_ptr(), Y.data_ptr(), n, ptr, nb, s.cuda_stream))
    s.synchronize()
    return Y


class Trainer:
    """Adam on FP32 master weights with cosine learning-rate decay."""

    def __init__(self, params0, batch=4096, device="cuda:0"):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.p = torch.tensor(params0, dtype=torch.float32, device=self.dev)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.batch = batch
        self.buf, self.ptr, self.nb = _scratch(torch, batch, self.dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.dev)
        self.t = 0

    def step(self, Xb, Yb, lr):
        self.t += 1
        s = _stream(self.torch, self.dev)
        s.wait_stream(self.torch.cuda.current_stream(self.dev))   # the batch gather
        Xb.record_stream(s)      # keep the allocator from reusing the batch early
        Yb.record_stream(s)
        stream = s.cuda_stream
        G._check(G.lib().grmhd_mlp_train_step(
            self.p.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), Xb.data_ptr(),
            Yb.data_ptr(), Xb.shape[0], ctypes.c_float(lr), self.t, self.loss.data_ptr(),
            self.ptr, self.nb, stream))

    def fit(self, X, Y, epochs, lr0=1e-3, seed=0, log=None):
        """X: standardised features, Y: targets (float32 device tensors)."""
        torch = self.torch
        n = X.shape[0]
        steps_per_epoch = n // self.batch
        total = epochs * steps_per_epoch
        gen = torch.Generator(device=self.dev)
        gen.manual_seed(seed)
        it = 0
        hist = []
        for ep in range(epochs):
            perm = torch.randperm(n, generator=gen, device=self.dev)
            for s in range(steps_per_epoch):
                idx = perm[s * self.batch:(s + 1) * self.batch]
                lr = 0.5 * lr0 * (1.0 + math.cos(math.pi * it / total))
                self.step(X[idx].contiguous(), Y[idx].contiguous(), lr)
                it += 1
            _stream(torch, self.dev).synchronize()
            hist.append(float(self.loss.item()))
            if log:
                log(ep, hist[-1])
        return hist
