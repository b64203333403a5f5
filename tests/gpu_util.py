"""Helpers for the GPU tests: device buffers through torch, padded-box packing
of the oracle's arrays, and comparisons."""
import numpy as np

from paper_2505_05424_amd import binding as B


def torch_mod():
    import torch
    return torch


def stream_handle():
    torch = torch_mod()
    return torch.cuda.current_stream().cuda_stream


def dev(arr, dtype=None):
    torch = torch_mod()
    a = np.ascontiguousarray(arr)
    t = torch.from_numpy(a)
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def planes_of(arrs, n, dtype=np.float64):
    """Stack exact-shape arrays as padded-box planes."""
    return np.stack([B.to_box(a, n) for a in arrs]).astype(dtype)


def host(t):
    return t.detach().cpu().numpy()


def q_shapes(g):
    return [g.cell_shape] + [g.q_shape(d) for d in range(1, g.D + 1)]


def unpack(planes, shapes):
    return [B.from_box(p, s) for p, s in zip(planes, shapes)]


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


class GpuState:
    """A state buffer allocated with torch for one plan."""

    def __init__(self, plan):
        torch = torch_mod()
        self.plan = plan
        self.info = plan.info
        self.buf = torch.zeros(int(self.info.state_bytes), dtype=torch.uint8, device="cuda")

    @property
    def ptr(self):
        return self.buf.data_ptr()

    def raw(self):
        return host(self.buf)

    def reset(self):
        B.dot_state_reset(self.plan, self.ptr, stream_handle())

    def run(self, iters):
        return B.dot_run(self.plan, self.ptr, iters, stream_handle())

    def extract(self):
        return B.dot_extract(self.plan, self.ptr, stream_handle())
