"""Helpers for the GPU parity tests (moving numpy arrays to and from the GPU)."""
import numpy as np

def torch_dtype(np_dtype):
    import torch
    return {np.dtype(np.uint32): torch.uint32, np.dtype(np.uint64): torch.uint64,
            np.dtype(np.float32): torch.float32}[np.dtype(np_dtype)]


def to_dev(x, offset=0):
    """Copy numpy array x to cuda:0.  offset > 0 places it `offset` elements
    into a larger allocation, so its base address is not 16-byte aligned."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if offset == 0:
        return t.to("cuda:0")
    big = torch.empty(x.size + offset, dtype=t.dtype, device="cuda:0")
    view = big[offset:]
    view.copy_(t)
    return view


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def same_bits(x, y):
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y)
    return x.dtype == y.dtype and x.shape == y.shape and np.array_equal(
        x.view(np.uint8), y.view(np.uint8))


def first_difference(x, y):
    """Index of the first element whose bytes differ, or None."""
    xb = np.ascontiguousarray(x).view(np.uint8).reshape(x.size, -1)
    yb = np.ascontiguousarray(y).view(np.uint8).reshape(y.size, -1)
    diff = np.nonzero(np.any(xb != yb, axis=1))[0]
    return None if diff.size == 0 else int(diff[0])
