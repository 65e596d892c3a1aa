"""Helpers for GPU tests: device transfers of uint16 data and guard-banded
output buffers (sentinel pads that catch out-of-bounds writes)."""
import numpy as np
import torch

SENTINEL = 0x5A5A
PAD = 2048  # elements of sentinel before and after each guarded buffer


def dev():
    return torch.device("cuda:0")


def to_dev_u16(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint16).view(np.int16)).to(dev())


def to_host_u16(t):
    return t.detach().cpu().numpy().view(np.uint16)


def to_dev_f64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev())


class Guarded:
    """A contiguous 16-bit device tensor of `shape` inside a sentinel-padded
    allocation; `offset` extra elements shift its address (alignment tests)."""

    def __init__(self, shape, offset=0, fill=SENTINEL):
        n = int(np.prod(shape))
        self.n = n
        self.offset = offset
        self.base = torch.full((n + 2 * PAD + offset,), fill - 65536 if fill > 32767 else fill,
                               dtype=torch.int16, device=dev())
        self.t = self.base[PAD + offset: PAD + offset + n].view(*shape)

    def check_pads(self):
        h = to_host_u16(self.base)
        pre = h[:PAD + self.offset]
        post = h[PAD + self.offset + self.n:]
        assert (pre == SENTINEL).all() and (post == SENTINEL).all(), "write outside the buffer"

    def host(self):
        return to_host_u16(self.t)
