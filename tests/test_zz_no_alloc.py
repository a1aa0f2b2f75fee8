"""The allocation-free training step (rir_mlp_train_step_noalloc: gradient
records in the library's fixed device array instead of a buffer it
allocates) against the allocating one (rir_mlp_train_step), through the C
ABI: same loss, gradient and updated weights on two calls in a row, the
second with a smaller batch, and rejection of batches beyond the array."""
import ctypes

import numpy as np
import pytest

import paper_2112_02779_amd as rir

pytestmark = pytest.mark.gpu


def _net_params(seed):
    rng = np.random.default_rng(seed)
    P = rng.normal(size=rir.MLP_NPARAM) * 0.2
    w, b = rir.split_params(P)
    return rir.join_params(w, b)


def _batch(seed, B):
    rng = np.random.default_rng(seed)
    f = np.empty((B, 14), np.float32)
    f[:, 0] = rng.uniform(0, 1, B)
    f[:, 1:9] = np.clip(rng.normal(size=(B, 8)) * 2, -4, 4)
    n = rng.normal(size=(B, 3))
    f[:, 9:12] = n / np.linalg.norm(n, axis=1, keepdims=True)
    f[:, 12:14] = np.clip(rng.normal(size=(B, 2)), -4, 4)
    y = (rng.uniform(size=B) < 0.7).astype(np.float32)
    return f, y


def _params(net):
    # bf16 weights, FP32 biases and FP32 master weights, through the C ABI
    w = np.zeros(rir.MLP_NW, np.uint16)
    b = np.zeros(rir.MLP_NB, np.float32)
    m = np.zeros(rir.MLP_NW, np.float32)
    st = rir.lib().rir_mlp_get_params(net.handle, w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                      b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                      m.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    assert st == rir.RIR_OK
    return w, b, m


def _step(fn, net, f, y, lr, torch):
    loss = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    grads = torch.zeros(rir.MLP_NPARAM, dtype=torch.float32, device="cuda:0")
    st = fn(net.handle, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(y.data_ptr()), ctypes.c_int64(y.numel()),
            ctypes.c_float(lr), ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(grads.data_ptr()),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == rir.RIR_OK, rir.lib().rir_last_error()
    torch.cuda.synchronize()
    return float(loss.item()), grads.cpu().numpy()


def test_noalloc_train_step_matches_allocating_step():
    import torch
    assert torch.cuda.is_available()
    L = rir.lib()
    fa = L.rir_mlp_train_step
    fn = L.rir_mlp_train_step_noalloc
    P = _net_params(5)
    ref, new = rir.Mlp(P), rir.Mlp(P)
    # two calls in a row, the second smaller (the array keeps the first
    # call's records beyond the second call's; they must not leak into it)
    for k, B in enumerate((32768, 3000)):
        f, y = _batch(10 + k, B)
        fd, yd = torch.from_numpy(f).to("cuda:0"), torch.from_numpy(y).to("cuda:0")
        la, ga = _step(fa, ref, fd, yd, 1e-3, torch)
        ln, gn = _step(fn, new, fd, yd, 1e-3, torch)
        # same kernels, same number of records, same summation order
        assert la == ln, (B, la, ln)
        assert np.array_equal(ga, gn), (B, np.max(np.abs(ga - gn)))
        wa, ba, ma = _params(ref)
        wn, bn, mn = _params(new)
        assert np.array_equal(wa, wn) and np.array_equal(ba, bn) and np.array_equal(ma, mn), B


def test_noalloc_train_step_rejects_batches_beyond_the_array():
    import torch
    L = rir.lib()
    fn = L.rir_mlp_train_step_noalloc
    net = rir.Mlp(_net_params(6))
    f = torch.zeros((32769, 14), dtype=torch.float32, device="cuda:0")
    y = torch.zeros(32769, dtype=torch.float32, device="cuda:0")
    st = fn(net.handle, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(y.data_ptr()), ctypes.c_int64(32769),
            ctypes.c_float(1e-3), None, None, None)
    assert st == rir.RIR_E_INVALID
    assert b"32768" in L.rir_last_error()
