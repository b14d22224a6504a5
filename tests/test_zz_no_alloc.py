"""The allocation-free training step of the learned inversion guess
(grmhd_mlp_train_step_noalloc, for callers that cannot allocate device memory)
against grmhd_mlp_train_step with a caller scratch.  Both run the same kernels,
so parameters, Adam moments and loss agree bit for bit: two calls in a row, the
second with a smaller (ragged) batch, so that the first call's contents of the
library's scratch are still there when the second runs.  A batch above the
maximum is refused before anything is launched."""
import ctypes

import numpy as np
import pytest

from oracle import mlp as ref
from parity_util import say

pytestmark = pytest.mark.gpu

BATCHES = (4096, 1000)


def _run(torch, G, L, Xs, Yt, p0, noalloc):
    dev = Xs.device
    stream = torch.cuda.Stream(device=dev)
    p = torch.tensor(p0, device=dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    keep = []
    out = []
    for t, B in enumerate(BATCHES, start=1):
        Xb, Yb = Xs[:B].contiguous(), Yt[:B].contiguous()
        torch.cuda.synchronize(dev)
        lr = ctypes.c_float(1e-3)
        if noalloc:
            rc = L.grmhd_mlp_train_step_noalloc(p.data_ptr(), m.data_ptr(), v.data_ptr(),
                                                Xb.data_ptr(), Yb.data_ptr(), B, lr, t,
                                                loss.data_ptr(), stream.cuda_stream)
        else:
            nb = L.grmhd_mlp_scratch_bytes(B)
            buf = torch.zeros(nb + 256, dtype=torch.uint8, device=dev)
            keep.append(buf)
            ptr = (buf.data_ptr() + 255) // 256 * 256
            rc = L.grmhd_mlp_train_step(p.data_ptr(), m.data_ptr(), v.data_ptr(), Xb.data_ptr(),
                                        Yb.data_ptr(), B, lr, t, loss.data_ptr(), ptr, nb,
                                        stream.cuda_stream)
        assert rc == 0, L.grmhd_last_error(None)
        stream.synchronize()
        out.append((p.cpu().numpy().copy(), m.cpu().numpy().copy(), v.cpu().numpy().copy(),
                    float(loss.item())))
    return out, (p, m, v, loss, stream)


def test_noalloc_train_step_equals_scratch_variant():
    import torch
    assert torch.cuda.is_available(), "needs an MI355X"
    from paper_2410_09146_amd import grmhd as G
    from paper_2410_09146_amd import mlp as M
    L = G.lib()
    dev = torch.device("cuda:0")
    X, Y, _, _ = ref.dataset(max(BATCHES), seed=31)
    mean, std = X.mean(0), X.std(0)
    Xs = torch.tensor(((X - mean) / std).astype(np.float32), device=dev)
    Yt = torch.tensor(Y.astype(np.float32), device=dev)
    p0 = M.init_params(seed=8).astype(np.float32)
    a, _ = _run(torch, G, L, Xs, Yt, p0, noalloc=False)
    b, (p, m, v, loss, stream) = _run(torch, G, L, Xs, Yt, p0, noalloc=True)
    for (B, ra, rb) in zip(BATCHES, a, b):
        say("train step, batch", B, "loss", ra[3], rb[3], "max |dparams|",
            float(np.abs(ra[0] - rb[0]).max()))
        for x, y in zip(ra[:3], rb[:3]):
            assert np.array_equal(x, y)
        assert ra[3] == rb[3]
    assert not np.array_equal(a[0][0], p0) and not np.array_equal(a[1][0], a[0][0])
    # above the maximum: refused on the host, nothing launched, nothing changed
    big = G.MLP_NOALLOC_MAX_BATCH + 1
    before = p.cpu().numpy().copy()
    rc = L.grmhd_mlp_train_step_noalloc(p.data_ptr(), m.data_ptr(), v.data_ptr(), Xs.data_ptr(),
                                        Yt.data_ptr(), big, ctypes.c_float(1e-3), 3,
                                        loss.data_ptr(), stream.cuda_stream)
    msg = L.grmhd_last_error(None).decode()
    say("batch", big, "->", rc, msg)
    assert rc == -2 and "exceeds" in msg
    torch.cuda.synchronize(dev)
    assert np.array_equal(p.cpu().numpy(), before)
